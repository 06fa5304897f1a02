"""End-to-end low-precision baselines (the paper's all-BF16 and all-FP16
recipes, Table 3 columns I and H) on the GPU (on an MI355X).

Per outer iteration, from the GPU's own previous iterate: every iterate is
representable in the format; the step is within the first-order bound of
one rounding to the format at every slot's output (tests/_bounds.py) of the
exact step; and most entries equal the oracle's emulation (casgd_e2e, the
same rounding points with FP64 sums) bitwise -- entries differ only where
an FP32 sum and its FP64 counterpart fall on two sides of a rounding
boundary.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import reference as R  # noqa: E402
from workloads import dense_glm  # noqa: E402
from _bounds import U32, assert_within, outer_bound  # noqa: E402

U_FMT = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}


@pytest.fixture(scope="module")
def cg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_18463_amd as cg
    cg._lib.load()
    return cg


def _dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("fmt", ["bf16", "f16"])
@pytest.mark.parametrize("loss", ["logistic", "linear"])
@pytest.mark.parametrize("b,s,kw", [(64, 16, {}), (32, 8, dict(exec_mode=2)),
                                    (16, 4, dict(exec_mode=1, fused_variant=1)),
                                    (64, 4, dict(exec_mode=1, fused_variant=2)), (24, 3, {})])
def test_e2e_each_outer_iteration(cg, fmt, loss, b, s, kw):
    p = dense_glm(20000, 264, 31, loss, var=1 / 264, dtype=np.float32)
    code = {"bf16": cg.BF16, "f16": cg.F16}[fmt]
    v, sc = cg.casgd_quantize(_dev(p.X), code)
    X = cg.dense_matrix(v, sc, n=264)
    exact = R.quantize(p.X, fmt)[2]
    eta, lam, seed, H = (0.5 if loss == "logistic" else 0.1), 1e-4, 3, 5
    hist = torch.zeros(H, 264, device="cuda")
    x = torch.zeros(264, device="cuda")
    e2e = 1 if fmt == "bf16" else 2
    o = cg.opts(snapshot_every=1, x_history=hist, loss=loss, e2e=e2e, **kw)
    ws = cg.casgd_fit(X, _dev(p.y), x, eta, lam, b, s, seed, 0, H, opts=o)
    cg.casgd_check(ws)
    xs = hist.cpu().numpy().astype(np.float64)
    prev = np.zeros(264)
    same = []
    for h in range(H):
        assert np.array_equal(R.round_to_format(xs[h], fmt), xs[h]), h
        idx = R.sample_indices(seed, h * s * b, s * b, 20000)
        bound, ex = outer_bound(exact[idx], prev, p.y[idx].astype(np.float64), b, s, eta, lam,
                                loss, u_acc=U32, u_round=U_FMT[fmt])
        assert_within(xs[h], ex["x"], bound, f"{fmt} {loss} outer {h}")
        xe = R.casgd_e2e(exact, p.y, prev, eta, lam, b, s, seed, h, 1, fmt, loss=loss)
        same.append(float(np.mean(xe == xs[h])))
        prev = xs[h]
    print(f"\n[e2e] {fmt} {loss} b={b} s={s} {kw}: bitwise-equal fraction per outer "
          f"{[round(v, 3) for v in same]}")
    assert min(same) >= 0.5


def test_e2e_rejects_mismatched_storage_and_fp64(cg):
    p = dense_glm(2000, 64, 1, "logistic", var=1 / 64, dtype=np.float32)
    X = cg.dense_matrix(_dev(p.X))
    x = torch.zeros(64, device="cuda")
    with pytest.raises(cg.CasgdError):
        cg.casgd_fit(X, _dev(p.y), x, 0.5, 0.0, 16, 4, 1, 0, 2, opts=cg.opts(e2e=1))
    v, _ = cg.casgd_quantize(_dev(p.X), cg.BF16)
    Xb = cg.dense_matrix(v, None, n=64)
    with pytest.raises(cg.CasgdError):
        cg.casgd_fit(Xb, _dev(p.y), x, 0.5, 0.0, 16, 4, 1, 0, 2, opts=cg.opts(e2e=2))
    with pytest.raises(cg.CasgdError):
        cg.casgd_fit(Xb, _dev(p.y), x, 0.5, 0.0, 16, 4, 1, 0, 2,
                     opts=cg.opts(e2e=1, recur_prec=64))
