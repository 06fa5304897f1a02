"""Pins of the oracle's end-to-end low-precision emulation (the paper's
all-BF16 and all-FP16 recipes, Table 3 columns I and H): the rounding
function against torch's and NumPy's casts, the emulation without rounding
against the plain s-step oracle, representability of every iterate, and one
outer iteration inside the uniform-precision bound of Cor. 5.2."""
import numpy as np
import pytest
import torch

from oracle import reference as R
from workloads import dense_c1


def test_round_to_format_matches_library_casts():
    g = np.random.default_rng(0)
    v32 = np.concatenate([g.standard_normal(20000) * 10.0 ** g.uniform(-8, 4, 20000),
                          [0.0, -0.0, 1.0, 65504.0, 65519.9, 65520.0, 1e5, 2.0 ** -24,
                           2.0 ** -25, 3 * 2.0 ** -26, 2.0 ** -14 * 1.5]]).astype(np.float32)
    v = v32.astype(np.float64)
    bf = torch.from_numpy(v32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(R.round_to_format(v, "bf16"), bf)
    with np.errstate(over="ignore"):
        h = v.astype(np.float16).astype(np.float64)  # NumPy: correctly rounded, RNE
    assert np.array_equal(R.round_to_format(v, "f16"), h)
    # ties go to even
    assert R.round_to_format(1 + 2.0 ** -8, "bf16") == 1.0
    assert R.round_to_format(1 + 3 * 2.0 ** -8, "bf16") == 1 + 2.0 ** -6
    assert R.round_to_format(1 + 2.0 ** -11, "f16") == 1.0


@pytest.mark.parametrize("loss", ["logistic", "linear"])
def test_no_rounding_is_the_plain_oracle(loss):
    p = dense_c1(42)
    y = p.y if loss == "logistic" else (p.X @ p.w_true / 16).astype(np.float32).astype(np.float64)
    x0 = np.zeros(256)
    xe = R.casgd_e2e(p.X, y, x0, 0.5, 1e-4, 16, 4, 42, 0, 6, None, loss=loss)
    xo = R.casgd(p.X, y, x0, 0.5, 1e-4, 16, 4, 42, 0, 6, loss=loss)
    assert np.linalg.norm(xe - xo) <= 1e-12 * np.linalg.norm(xo)


@pytest.mark.parametrize("fmt", ["bf16", "f16"])
def test_iterates_are_representable_and_step_within_uniform_bound(fmt):
    p = dense_c1(42)
    Xn = p.X / np.linalg.norm(p.X, axis=1, keepdims=True)
    stored = R.round_to_format(Xn, fmt)
    b, s, eta = 16, 4, 0.5
    x, snaps = R.casgd_e2e(stored, p.y, np.zeros(256), eta, 0.0, b, s, 42, 0, 5, fmt,
                           snapshots=True)
    for xs in snaps:
        assert np.array_equal(R.round_to_format(xs, fmt), xs)
    # one outer iteration from a representable x against the exact step on
    # the unrounded rows: inside Cor. 5.2 with u = the format's unit roundoff
    u = R.unit_roundoff(fmt)
    xin = snaps[-1]
    h = 5
    idx = R.sample_indices(42, h * s * b, s * b, 4096)
    x1 = R.casgd_e2e(stored, p.y, xin, eta, 0.0, b, s, 42, h, 1, fmt)
    bnd = R.uniform_precision_bound(Xn[idx], xin, p.y[idx], b, s, eta, u)
    err = np.linalg.norm(x1 - bnd["x_exact"])
    assert err <= bnd["bound"], (err, bnd["bound"])
    # and the rounding is visible: the FP16 / BF16 step is not the exact one
    assert err > 0.0
