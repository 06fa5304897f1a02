"""Precision modes on the 4096 x 256 workload (MI355X).

* Whole fits with X stored in BF16 / FP16 / FP8-e4m3 (row scales), Gram and
  margins on MFMA with FP32 accumulation, the recurrence in FP32 (s*b < 512) or
  FP64: the GPU trajectory matches the FP64 oracle run on the exact values of
  the same stored elements (arithmetic error), and the error against the
  unquantised FP64 oracle (storage + arithmetic) is reported.
* One outer iteration from the same x and rows stays within the local
  forward-error bound of Thm. 5.1 (one device: the all-reduce terms vanish),
  on l2-normalised rows (Assumption 1), for each storage format.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import reference as R  # noqa: E402
from workloads import dense_c1, normalize_rows  # noqa: E402

U32 = R.U_FP32


@pytest.fixture(scope="module")
def cg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_18463_amd as cg
    cg._lib.load()
    return cg


@pytest.fixture(scope="module")
def c1():
    return dense_c1(42)


def _dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _store(cg, X32, fmt):
    code = {"f32": cg.F32, "bf16": cg.BF16, "f16": cg.F16, "fp8": cg.FP8E4M3}[fmt]
    dst, sc = cg.casgd_quantize(_dev(X32), code)
    _, _, exact = R.quantize(X32, fmt)
    return cg.dense_matrix(dst, sc, n=X32.shape[1]), exact, (dst, sc)


# (b, s) of the precision sweep and the outer iterations each runs (the
# oracle's cost grows as (s b)^2 per outer iteration)
SHAPES = [(32, 8, 200), (128, 8, 50), (32, 32, 50), (128, 32, 20)]


@pytest.mark.parametrize("fmt", ["bf16", "f16", "fp8"])
@pytest.mark.parametrize("b,s,H", SHAPES)
def test_precision_sweep_matches_oracle(cg, c1, fmt, b, s, H):
    eta, lam, seed = 0.5, 1e-4, 42
    X32 = c1.X.astype(np.float32)
    X, exact, keep = _store(cg, X32, fmt)
    y = _dev(c1.y)
    x = _dev(np.zeros(256, np.float32))
    ws = cg.casgd_fit(X, y, x, eta, lam, b, s, seed, 0, H)
    cg.casgd_check(ws)
    xg = x.cpu().numpy().astype(np.float64)
    xo = R.casgd(exact, c1.y, np.zeros(256), eta, lam, b, s, seed, 0, H)
    arith = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    xf = R.casgd(c1.X, c1.y, np.zeros(256), eta, lam, b, s, seed, 0, H)
    total = np.linalg.norm(xg - xf) / np.linalg.norm(xf)
    lg = R.logloss(c1.X_test, c1.y_test, xg)
    lf = R.logloss(c1.X_test, c1.y_test, xf)
    print(f"\n[precision] fmt={fmt} b={b} s={s} H={H} recur={'fp64' if s * b >= 512 else 'fp32'}"
          f" rel_err_vs_oracle_same_storage={arith:.3e} rel_err_vs_fp64_unquantised={total:.3e}"
          f" test_loss_gap={abs(lg - lf) / lf:.3e}")
    assert arith < 1e-4
    # storage error: the loss stays close to the unquantised FP64 run
    assert abs(lg - lf) / lf < {"bf16": 1e-2, "f16": 1e-3, "fp8": 5e-2}[fmt]


@pytest.mark.parametrize("fmt", ["f32", "bf16", "f16", "fp8"])
@pytest.mark.parametrize("b,s", [(32, 8), (16, 4), (128, 8), (32, 32)])
def test_one_outer_iteration_within_theorem_bound(cg, c1, fmt, b, s):
    """Thm. 5.1 (P = 1) with the slots of this path: storage u_A (the largest
    relative storage error of the rows actually stored), Gram and margins
    FP32-accumulated over n (+2 roundings for row scales and the store),
    recurrence in FP32 or FP64, update FP32-accumulated over s*b (+3), x in
    FP32. The theorem has no L2 term, so lambda = 0."""
    eta, seed = 0.5, 7
    Xn = normalize_rows(c1.X)                 # FP64, unit rows
    X32 = Xn.astype(np.float32)
    X, exact, keep = _store(cg, X32, fmt)
    nz = Xn != 0
    u_A = float(np.max(np.abs(exact[nz] - Xn[nz]) / np.abs(Xn[nz])))
    x0 = (np.random.default_rng(4).standard_normal(256) * 0.5).astype(np.float32)
    x = _dev(x0)
    y = _dev(c1.y)
    ws = cg.casgd_step(X, y, x, eta, 0.0, b, s, seed, 0)
    cg.casgd_check(ws)
    xg = x.cpu().numpy().astype(np.float64)
    idx = R.sample_indices(seed, 0, s * b, Xn.shape[0])
    n, sb = 256, s * b
    u_c = R.U_FP64 if sb >= 512 else U32
    res = R.local_error_bound(Xn[idx], x0.astype(np.float64), c1.y[idx].astype(np.float64), b, s,
                              eta, u_A=u_A, gamma_r=R.gamma(n + 2, U32),
                              gamma_G=R.gamma(n + 2, U32), u_c=u_c, u_sigma=u_c,
                              gamma_g=R.gamma(sb + 3, U32), u_x=U32)
    err = float(np.linalg.norm(xg - res["x_exact"]))
    print(f"\n[thm5.1] fmt={fmt} b={b} s={s} u_A={u_A:.2e} error={err:.3e} bound={res['bound']:.3e}"
          f" ratio={err / res['bound']:.3f}")
    assert err <= res["bound"]


@pytest.mark.parametrize("fmt", ["bf16", "f16", "fp8"])
@pytest.mark.parametrize("b,s", [(32, 8), (128, 8)])
def test_one_outer_iteration_within_theorem_bound_bounded_entries(cg, c1, fmt, b, s):
    """The same check on rows whose entries all have magnitudes within a factor
    of two of each other (signs and labels of the 4096 x 256 workload), so no
    stored element is subnormal and u_A is the format's own relative rounding
    error (FP16 2^-11, FP8-e4m3 2^-4 with the row scale): the bound is then
    tight enough to be informative for every format."""
    eta, seed = 0.5, 7
    mag = np.random.default_rng(11).uniform(0.5, 1.0, size=c1.X.shape)
    Xn = normalize_rows(np.sign(c1.X + (c1.X == 0)) * mag)
    X32 = Xn.astype(np.float32)
    X, exact, keep = _store(cg, X32, fmt)
    u_A = float(np.max(np.abs(exact - Xn) / np.abs(Xn)))
    assert u_A <= {"bf16": 2.0 ** -8, "f16": 2.0 ** -11, "fp8": 2.0 ** -4}[fmt] * 1.01
    x0 = (np.random.default_rng(4).standard_normal(256) * 0.5).astype(np.float32)
    x = _dev(x0)
    y = _dev(c1.y)
    ws = cg.casgd_step(X, y, x, eta, 0.0, b, s, seed, 0)
    cg.casgd_check(ws)
    xg = x.cpu().numpy().astype(np.float64)
    idx = R.sample_indices(seed, 0, s * b, Xn.shape[0])
    n, sb = 256, s * b
    u_c = R.U_FP64 if sb >= 512 else U32
    res = R.local_error_bound(Xn[idx], x0.astype(np.float64), c1.y[idx].astype(np.float64), b, s,
                              eta, u_A=u_A, gamma_r=R.gamma(n + 2, U32),
                              gamma_G=R.gamma(n + 2, U32), u_c=u_c, u_sigma=u_c,
                              gamma_g=R.gamma(sb + 3, U32), u_x=U32)
    err = float(np.linalg.norm(xg - res["x_exact"]))
    print(f"\n[thm5.1 bounded] fmt={fmt} b={b} s={s} u_A={u_A:.2e} error={err:.3e} "
          f"bound={res['bound']:.3e} ratio={err / res['bound']:.3f}")
    assert err <= res["bound"]


def test_fp8_decode_every_code(cg):
    """Every finite OCP E4M3 code decodes (hardware convert) to the oracle's
    value; the NaN codes 0x7f and 0xff decode to NaN. Two rows of the 256
    codes with unit scales: the column means are the decoded values; a
    weight vector picks them up through the margin and update passes too."""
    codes = np.tile(np.arange(256, dtype=np.uint8), (2, 1))
    Xd = torch.from_numpy(codes).cuda()
    X = cg.dense_matrix(Xd, torch.ones(2, device="cuda"), n=256)
    stats = cg.casgd_colstats(X).cpu().numpy().astype(np.float64)
    want = R.e4m3_decode(np.arange(256, dtype=np.uint8))
    nan = np.isin(np.arange(256), [0x7F, 0xFF])
    assert np.array_equal(stats[~nan, 0], want[~nan])
    assert np.all(np.isnan(stats[nan, 0]))
    # the update pass: one s = 1 step from x = 0 with eta = b gives
    # x = sum_t c_t * row_t with c_t = y_t / 2 (logistic residual at z = 0)
    fin = codes[:, ~nan].copy()
    n = fin.shape[1]
    ld = (n + 15) // 16 * 16
    pad = np.zeros((2, ld), np.uint8)
    pad[:, :n] = fin
    X2 = cg.dense_matrix(torch.from_numpy(pad).cuda(), torch.ones(2, device="cuda"), n=n)
    x = torch.zeros(n, device="cuda")
    y = torch.ones(2, device="cuda")
    ws = cg.casgd_fit(X2, y, x, 1.0, 0.0, 1, 1, 3, 0, 1)
    cg.casgd_check(ws)
    row = R.e4m3_decode(fin[0])
    assert np.array_equal(x.cpu().numpy().astype(np.float64), 0.5 * row)
