"""Parity of the dense HIP path with the FP64 oracle (on an MI355X).

Every expected value comes from the oracle on the same seeded inputs. The
GPU sees X in its storage format; the oracle sees the exact FP64 value of
the same stored elements, so the comparison measures arithmetic error only.

Tolerances (Sec. 3.2, eq. for gamma_q): an FP32-accumulated inner product of
length q is within gamma_q(u32) * |a|^T |b| of the exact one; a factor 2 is
added for the extra roundings of the row scales and the FP32 storage of the
result. Whole-trajectory comparisons use tolerances stated per test.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import reference as R  # noqa: E402
from workloads import dense_c1, dense_logreg  # noqa: E402

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def cg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_18463_amd as cg
    cg._lib.load()
    return cg


@pytest.fixture(scope="module")
def c1data():
    return dense_c1(42)


def _to_dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _stored(cg, X32, fmt):
    """Store an FP32 matrix on the GPU in `fmt` via the library's quantizer;
    returns (MatrixRef, exact FP64 values of the stored rows from the oracle)."""
    codes, scale, exact = R.quantize(X32, fmt)
    code = {"f32": cg.F32, "bf16": cg.BF16, "f16": cg.F16, "fp8": cg.FP8E4M3}[fmt]
    dst, sc = cg.casgd_quantize(_to_dev(X32), code)
    torch.cuda.synchronize()
    n = X32.shape[1]
    X = cg.dense_matrix(dst, sc, n=n)
    return X, exact, dst, sc


# ------------------------------------------------------------------ sampling

@pytest.mark.parametrize("seed,m", [(42, 4096), (7, 1 << 20), (2**63 + 5, 1), (3, 10**6 + 3),
                                    (11, 2**40 + 17)])
def test_sampler_bitexact(cg, seed, m):
    count = 1 << 20
    for t0 in (0, 123456789):
        got = cg.casgd_sample_indices(seed, t0, count, m).cpu().numpy()
        assert np.array_equal(got, R.sample_indices(seed, t0, count, m))


# ------------------------------------------------------------ storage formats

@pytest.mark.parametrize("fmt", ["f32", "bf16", "f16", "fp8"])
def test_quantize_bitexact(cg, c1data, fmt):
    X32 = c1data.X.astype(np.float32)
    X32[3] = 0.0                       # all-zero row: scale 1
    X32[5, :7] = [448.0, -500.0, 1e-6, -1e-6, 2.0 ** -10, 3 * 2.0 ** -10, 0.0]
    codes, scale, _ = R.quantize(X32, fmt)
    code = {"f32": cg.F32, "bf16": cg.BF16, "f16": cg.F16, "fp8": cg.FP8E4M3}[fmt]
    dst, sc = cg.casgd_quantize(_to_dev(X32), code)
    got = dst.cpu()
    n = X32.shape[1]
    if fmt == "bf16":
        got = got.view(torch.int16).numpy().view(np.uint16)[:, :n]
    elif fmt == "f16":
        got = got.numpy()[:, :n]
        codes = codes.astype(np.float16)
    else:
        got = got.numpy()[:, :n]
    assert np.array_equal(got, codes)
    if fmt == "fp8":
        assert np.array_equal(sc.cpu().numpy(), scale)


# --------------------------------------------------------- Gram and margin

GRAM_CASES = [
    # (m, n, ld, b, s)  -- C1 shape, ragged sb and K tail, split-K, multi-tile
    (4096, 256, 256, 16, 4),
    (3000, 203, 208, 24, 5),
    (5000, 2048, 2048, 64, 8),
    (2000, 512, 512, 128, 3),
    (1000, 96, 96, 1, 7),
]


@pytest.mark.parametrize("fmt", ["f32", "bf16", "f16", "fp8"])
@pytest.mark.parametrize("case", GRAM_CASES)
@pytest.mark.parametrize("gram_tile", [64, 128])
def test_gram_margin_vs_oracle(cg, fmt, case, gram_tile):
    m, n, ld, b, s = case
    p = dense_logreg(m, n, 9, var=1.0 / n, noise_var=0.1, dtype=np.float32)
    X32 = p.X
    code = {"f32": cg.F32, "bf16": cg.BF16, "f16": cg.F16, "fp8": cg.FP8E4M3}[fmt]
    vec = {"f32": 4, "bf16": 8, "f16": 8, "fp8": 16}[fmt]
    ld = max(ld, (n + vec - 1) // vec * vec)
    dst, sc = cg.casgd_quantize(_to_dev(X32), code, ld_dst=ld)
    X = cg.dense_matrix(dst, sc, n=n)
    _, _, exact = R.quantize(X32, fmt)
    x = np.random.default_rng(5).standard_normal(n).astype(np.float32)
    sb = s * b
    for h in (0, 3):
        G, r = cg.casgd_gram_margin(X, _to_dev(x), b, s, 42, h,
                                    opts=cg.opts(gram_tile=gram_tile))
        G = G.cpu().numpy().astype(np.float64)
        r = r.cpu().numpy().astype(np.float64)
        parts = R.outer_parts(exact, p.y, x.astype(np.float64), 0.5, 0.0, b, s, 42, h)
        Y = exact[parts["idx"]]
        mask = R.strict_block_lower_mask(b, s)
        bound = 2 * R.gamma(n + 2, U32) * (np.abs(Y) @ np.abs(Y).T) + 1e-30
        err = np.abs(G - parts["G"])
        assert np.all(err[mask] <= bound[mask]), (h, float((err / bound)[mask].max()))
        rb = 2 * R.gamma(n + 2, U32) * (np.abs(Y) @ np.abs(x.astype(np.float64))) + 1e-30
        assert np.all(np.abs(r - parts["r"]) <= rb)


@pytest.mark.parametrize("fmt", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("n,b,s", [(8200, 32, 8), (8192, 64, 2), (9000, 16, 24)])
def test_gram_ksplit_vs_oracle(cg, fmt, n, b, s):
    """128 x 128 tiles split along K (few tiles, long K; ragged K tail): every
    strict block-lower entry within the Gram bound of the oracle's, two launches
    on one workspace bitwise equal (each tags its exchange words with a new
    epoch), and equal to rounding to the unsplit tiles."""
    m = 3000
    p = dense_logreg(m, n, 11, var=1.0 / n, noise_var=0.1, dtype=np.float32)
    code = {"f32": cg.F32, "bf16": cg.BF16, "fp8": cg.FP8E4M3}[fmt]
    dst, sc = cg.casgd_quantize(_to_dev(p.X), code)
    X = cg.dense_matrix(dst, sc, n=n)
    _, _, exact = R.quantize(p.X, fmt)
    big = cg.casgd_gram_workspace_size(X, b, s)
    assert big > cg.casgd_workspace_size(X, b, s)   # this shape is split
    # a workspace full of other data: the exchange region is cleared on first use
    ws = torch.full((big,), 0x55, dtype=torch.uint8, device="cuda")
    cg.casgd_reset(ws)   # the flag words
    o = cg.opts(gram_tile=128)
    mask = R.strict_block_lower_mask(b, s)
    for h in (0, 5):
        G1, _ = cg.casgd_gram_margin(X, None, b, s, 42, h, ws=ws, opts=o)
        G2, _ = cg.casgd_gram_margin(X, None, b, s, 42, h, ws=ws, opts=o)
        G0, _ = cg.casgd_gram_margin(X, None, b, s, 42, h, opts=o,
                                     ws=cg.workspace(cg.casgd_workspace_size(X, b, s)))
        cg.casgd_check(ws)
        G1 = G1.cpu().numpy().astype(np.float64)
        assert np.array_equal(G1, G2.cpu().numpy().astype(np.float64))
        parts = R.outer_parts(exact, p.y, np.zeros(n), 0.5, 0.0, b, s, 42, h)
        Y = exact[parts["idx"]]
        bound = 2 * R.gamma(n + 2, U32) * (np.abs(Y) @ np.abs(Y).T) + 1e-30
        err = np.abs(G1 - parts["G"])
        assert np.all(err[mask] <= bound[mask]), (h, float((err / bound)[mask].max()))
        G0 = G0.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(G1 - G0)[mask] <= 2 * bound[mask])


def test_gram_ksplit_remainder_vs_oracle(cg):
    """More 128-tiles than the device holds workgroups (s*b = 4096: 528 tiles):
    whole rounds of tiles, then the remaining tiles split along K. Sampled
    rows of G against the oracle within the Gram bound."""
    m, n, b, s = 8192, 4096, 32, 128
    p = dense_logreg(m, n, 12, var=1.0 / n, noise_var=0.1, dtype=np.float32)
    dst, sc = cg.casgd_quantize(_to_dev(p.X), cg.BF16)
    X = cg.dense_matrix(dst, sc, n=n)
    _, _, exact = R.quantize(p.X, "bf16")
    big = cg.casgd_gram_workspace_size(X, b, s)
    assert big > cg.casgd_workspace_size(X, b, s)
    ws = cg.workspace(big)
    G, _ = cg.casgd_gram_margin(X, None, b, s, 42, 1, ws=ws, opts=cg.opts(gram_tile=128))
    cg.casgd_check(ws)
    G = G.cpu().numpy().astype(np.float64)
    idx = R.sample_indices(42, 1 * s * b, s * b, m)
    Y = exact[idx]
    rows = np.r_[np.arange(3968, 4096), np.random.default_rng(3).choice(4096, 256, replace=False)]
    mask = R.strict_block_lower_mask(b, s)[rows]
    ref = Y[rows] @ Y.T
    bound = 2 * R.gamma(n + 2, U32) * (np.abs(Y[rows]) @ np.abs(Y).T) + 1e-30
    err = np.abs(G[rows] - ref)
    assert np.all(err[mask] <= bound[mask]), float((err / bound)[mask].max())


# ---------------------------------------------------------------- recurrence

@pytest.mark.parametrize("b,s", [(16, 4), (32, 8), (64, 16), (24, 5), (128, 8), (3, 11)])
@pytest.mark.parametrize("prec", [32, 64])
def test_recurrence_vs_oracle(cg, c1data, b, s, prec):
    X = c1data.X
    x = np.random.default_rng(1).standard_normal(256) * 0.3
    eta, lam = 0.5, 1e-3
    parts = R.outer_parts(X, c1data.y, x, eta, lam, b, s, 42, 1)
    c = cg.casgd_recurrence(_to_dev(parts["G"]), _to_dev(parts["r"]), _to_dev(parts["yI"]),
                            b, s, eta, lam, prec)
    d = torch.empty(s * b, dtype=torch.float32, device="cuda")
    cg.casgd_recurrence(_to_dev(parts["G"]), _to_dev(parts["r"]), _to_dev(parts["yI"]),
                        b, s, eta, lam, prec, delta=d)
    c = c.cpu().numpy().astype(np.float64)
    d = d.cpu().numpy().astype(np.float64)
    # inputs rounded to FP32 (relative u32) propagate through the corrections
    # with gain <= K_s; FP32 arithmetic adds gamma_{(s-1)b}(u32)
    tol = 2e-6 if prec == 64 else 2e-6 + 4 * R.gamma((s - 1) * b + 4, U32)
    assert np.max(np.abs(d - parts["delta"])) <= tol
    assert np.max(np.abs(c - parts["c"])) <= tol


# -------------------------------------------------------------------- update

@pytest.mark.parametrize("fmt", ["f32", "bf16", "fp8"])
def test_update_vs_oracle(cg, c1data, fmt):
    X32 = c1data.X.astype(np.float32)
    Xs, exact, dst, sc = _stored(cg, X32, fmt)
    b, s, eta, lam = 16, 4, 0.5, 1e-3
    x0 = np.random.default_rng(2).standard_normal(256).astype(np.float32) * 0.2
    parts = R.outer_parts(exact, c1data.y, x0.astype(np.float64), eta, lam, b, s, 42, 2)
    xg = _to_dev(x0)
    cg.casgd_update(Xs, xg, _to_dev(parts["c"]), b, s, 42, 2, eta, lam)
    got = xg.cpu().numpy().astype(np.float64)
    Y = exact[parts["idx"]]
    c32 = parts["c"].astype(np.float32).astype(np.float64)
    expect = (1 - eta * lam) ** s * x0 + (eta / b) * Y.T @ c32
    bound = (eta / b) * 2 * R.gamma(s * b + 3, U32) * (np.abs(Y).T @ np.abs(c32)) \
        + 4 * U32 * np.abs(expect) + 1e-30
    assert np.all(np.abs(got - expect) <= bound)


# ------------------------------------------------------- whole fits (C1)

def _fit(cg, X, y, x0, eta, lam, b, s, seed, H, **kw):
    x = _to_dev(x0)
    o = cg.opts(**kw)
    ws = cg.casgd_fit(X, y, x, eta, lam, b, s, seed, 0, H, opts=o)
    cg.casgd_check(ws)
    return x.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("mode,variant", [(1, 1), (1, 2), (2, 0)])
def test_c1_fit_matches_oracle(cg, c1data, mode, variant):
    """C1: 4096 x 256, b=16, s=4, eta=0.5, lambda=1e-4, 200 outer iterations."""
    X32 = c1data.X.astype(np.float32)
    Xs = cg.dense_matrix(_to_dev(X32))
    y = _to_dev(c1data.y)
    H = 200
    xg = _fit(cg, Xs, y, np.zeros(256, np.float32), 0.5, 1e-4, 16, 4, 42, H,
              exec_mode=mode, fused_variant=variant)
    xo = R.casgd(X32, c1data.y, np.zeros(256), 0.5, 1e-4, 16, 4, 42, 0, H)
    rel = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    assert rel < 1e-4, rel
    lg = R.logloss(c1data.X_test, c1data.y_test, xg)
    lo = R.logloss(c1data.X_test, c1data.y_test, xo)
    assert abs(lg - lo) / lo < 1e-5


@pytest.mark.parametrize("b,s,prec", [(16, 16, 32), (16, 24, 64), (32, 12, 32), (64, 8, 64),
                                      (64, 16, 64), (128, 4, 32), (128, 6, 64), (64, 32, 0)])
def test_stream_ordered_multi_workgroup_recurrence(cg, b, s, prec):
    """The stream-ordered fit runs the recurrence on one chain workgroup plus
    helper workgroups (s > W + 1); its trajectory matches the FP64 oracle and
    the fused launch (single-workgroup recurrence) to rounding."""
    p = dense_logreg(3000, 136, 5, var=1 / 136, noise_var=0.1, dtype=np.float32)
    X = cg.dense_matrix(_to_dev(p.X))
    y = _to_dev(p.y)
    H = max(3, 256 // s)
    xg = _fit(cg, X, y, np.zeros(136, np.float32), 0.5, 1e-4, b, s, 9, H, exec_mode=2,
              recur_prec=prec)
    xf = _fit(cg, X, y, np.zeros(136, np.float32), 0.5, 1e-4, b, s, 9, H, exec_mode=1,
              fused_variant=2, recur_prec=prec)
    x3 = _fit(cg, X, y, np.zeros(136, np.float32), 0.5, 1e-4, b, s, 9, H, exec_mode=1,
              fused_variant=3, recur_prec=prec)
    xo = R.casgd(p.X, p.y, np.zeros(136), 0.5, 1e-4, b, s, 9, 0, H)
    for xv in (xg, xf, x3):
        assert np.linalg.norm(xv - xo) / np.linalg.norm(xo) < 1e-4
    # the fused variant 3 runs the same recurrence and margin reduction
    assert np.linalg.norm(x3 - xg) / np.linalg.norm(xo) < 1e-6


def test_exec_modes_bitwise_equal(cg, c1data):
    """The fused variants share every device function: bitwise equal. The
    stream-ordered form sums the recurrence in another order (near and far
    parts): bitwise reproducible, equal to the fused result to rounding."""
    X32 = c1data.X.astype(np.float32)
    Xs = cg.dense_matrix(_to_dev(X32))
    y = _to_dev(c1data.y)
    runs = [_fit(cg, Xs, y, np.zeros(256, np.float32), 0.5, 1e-4, 16, 4, 42, 50,
                 exec_mode=m, fused_variant=v) for m, v in [(1, 1), (1, 2), (1, 1), (2, 0), (2, 0)]]
    assert np.array_equal(runs[1], runs[0]) and np.array_equal(runs[2], runs[0])
    assert np.array_equal(runs[4], runs[3])
    assert np.linalg.norm(runs[3] - runs[0]) / np.linalg.norm(runs[0]) < 1e-5


def test_gpu_s_step_equals_gpu_sgd(cg, c1data):
    X32 = c1data.X.astype(np.float32)
    Xs = cg.dense_matrix(_to_dev(X32))
    y = _to_dev(c1data.y)
    a = _fit(cg, Xs, y, np.zeros(256, np.float32), 0.5, 1e-4, 16, 1, 42, 800)
    for s in (2, 4, 16):
        c = _fit(cg, Xs, y, np.zeros(256, np.float32), 0.5, 1e-4, 16, s, 42, 800 // s)
        assert np.linalg.norm(a - c) / np.linalg.norm(a) < 1e-5


def test_s1_matches_oracle_sgd(cg, c1data):
    X32 = c1data.X.astype(np.float32)
    Xs = cg.dense_matrix(_to_dev(X32))
    y = _to_dev(c1data.y)
    xg = _fit(cg, Xs, y, np.zeros(256, np.float32), 0.5, 1e-4, 16, 1, 42, 400)
    xo = R.sgd(X32, c1data.y, np.zeros(256), 0.5, 1e-4, 16, 42, 0, 400)
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) < 1e-4


def test_resume_and_determinism(cg, c1data):
    X32 = c1data.X.astype(np.float32)
    Xs = cg.dense_matrix(_to_dev(X32))
    y = _to_dev(c1data.y)
    x = _to_dev(np.zeros(256, np.float32))
    ws = cg.casgd_fit(Xs, y, x, 0.5, 1e-4, 16, 4, 42, 0, 30)
    full = x.cpu().numpy()
    x2 = _to_dev(np.zeros(256, np.float32))
    cg.casgd_fit(Xs, y, x2, 0.5, 1e-4, 16, 4, 42, 0, 13, ws=ws)
    cg.casgd_fit(Xs, y, x2, 0.5, 1e-4, 16, 4, 42, 13, 17, ws=ws)
    assert np.array_equal(full, x2.cpu().numpy())
    x3 = _to_dev(np.zeros(256, np.float32))
    for h in range(30):
        cg.casgd_step(Xs, y, x3, 0.5, 1e-4, 16, 4, 42, h, ws=ws)
    assert np.array_equal(full, x3.cpu().numpy())


@pytest.mark.parametrize("mode", [1, 2])
def test_snapshots(cg, c1data, mode):
    X32 = c1data.X.astype(np.float32)
    Xs = cg.dense_matrix(_to_dev(X32))
    y = _to_dev(c1data.y)
    hist = torch.zeros(4, 256, device="cuda")
    th = torch.zeros(5, dtype=torch.int64, device="cuda")
    x = _to_dev(np.zeros(256, np.float32))
    o = cg.opts(exec_mode=mode, snapshot_every=5, x_history=hist, t_history=th)
    cg.casgd_fit(Xs, y, x, 0.5, 1e-4, 16, 4, 42, 0, 20, opts=o)
    ref = _to_dev(np.zeros(256, np.float32))
    for k in range(4):
        cg.casgd_fit(Xs, y, ref, 0.5, 1e-4, 16, 4, 42, 5 * k, 5, opts=cg.opts(exec_mode=mode))
        assert torch.equal(hist[k], ref)
    if mode == 1:
        t = th.cpu().numpy()
        assert np.all(np.diff(t) >= 0) and t[-1] > t[0]


def test_nonfinite_is_reported(cg, c1data):
    X32 = (c1data.X * 1e18).astype(np.float32)
    Xs = cg.dense_matrix(_to_dev(X32))
    y = _to_dev(c1data.y)
    x = _to_dev(np.zeros(256, np.float32))
    ws = cg.casgd_fit(Xs, y, x, 1e30, 0.0, 16, 4, 42, 0, 5)
    with pytest.raises(cg.CasgdError) as e:
        cg.casgd_check(ws)
    assert e.value.status == -5
    cg.casgd_reset(ws)
    cg.casgd_check(ws)


def test_barrier_timeout_is_reported_and_recoverable(cg, c1data):
    """A spin limit of one poll makes the fused kernel's bounded barrier give
    up; every workgroup then leaves the kernel and the flag is reported."""
    X32 = c1data.X.astype(np.float32)
    Xs = cg.dense_matrix(_to_dev(X32))
    y = _to_dev(c1data.y)
    x = _to_dev(np.zeros(256, np.float32))
    o = cg.opts(exec_mode=1, fused_variant=2, spin_limit=1, grid_blocks=64)
    ws = cg.casgd_fit(Xs, y, x, 0.5, 1e-4, 16, 4, 42, 0, 20, opts=o)
    with pytest.raises(cg.CasgdError) as e:
        cg.casgd_check(ws)
    assert e.value.status == -6
    cg.casgd_reset(ws)
    x = _to_dev(np.zeros(256, np.float32))
    cg.casgd_fit(Xs, y, x, 0.5, 1e-4, 16, 4, 42, 0, 20, ws=ws)
    cg.casgd_check(ws)


# --------------------------------------------------------- loss and stats

@pytest.mark.parametrize("fmt", ["f32", "bf16", "fp8"])
def test_logloss_vs_oracle(cg, c1data, fmt):
    X32 = c1data.X_test.astype(np.float32)
    Xs, exact, _, _ = _stored(cg, X32, fmt)
    xs = np.random.default_rng(3).standard_normal((3, 256)).astype(np.float32)
    got = cg.casgd_logloss(Xs, _to_dev(c1data.y_test), _to_dev(xs)).cpu().numpy()
    for k in range(3):
        ref = R.logloss(exact, c1data.y_test, xs[k].astype(np.float64))
        assert abs(got[k] - ref) <= 1e-5 * ref


@pytest.mark.parametrize("fmt", ["f32", "bf16", "fp8"])
def test_colstats_vs_oracle(cg, fmt):
    p = dense_logreg(3000, 200, 4, var=1 / 200, scaled_cols=20, col_factor=10.0,
                     dtype=np.float32)
    X32 = p.X.copy()
    X32[:, 7] = 0
    X32[::2, 9] = 0
    Xs, exact, _, _ = _stored(cg, X32, fmt)
    got = cg.casgd_colstats(Xs).cpu().numpy().astype(np.float64)
    ref = R.column_stats(exact)
    assert np.allclose(got, ref, rtol=1e-5, atol=1e-7)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_c2_scale_sampled_check(cg, storage):
    """Full-size dense workload (2^20 x 2048 FP32, b = 64, s = 16, lambda =
    1e-5, eta = 2) in the launch configuration the benchmark times (fused,
    automatic form and grid): six outer iterations against the oracle, which
    reads only the sampled rows (for BF16 storage, of the stored values)."""
    from workloads import dense_c2
    p = dense_c2(42, m=1 << 20, n=2048, m_test=1)
    b, s, H, eta, lam, seed = 64, 16, 6, 2.0, 1e-5, 42
    X32 = torch.from_numpy(p.X).cuda()
    if storage == "f32":
        X = cg.dense_matrix(X32)
        Xo = p.X
    else:
        v, sc = cg.casgd_quantize(X32, cg.BF16)
        X = cg.dense_matrix(v, sc, n=2048)
        # the oracle reads only the sampled rows: give it their stored values
        # (in place: the FP32 copy is on the device already)
        idx = np.unique(R.sample_indices(seed, 0, H * s * b, p.X.shape[0]))
        _, _, exact = R.quantize(p.X[idx], "bf16")
        p.X[idx] = exact
        Xo = p.X
    y = torch.from_numpy(p.y).cuda()
    x = torch.zeros(2048, device="cuda")
    ws = cg.casgd_fit(X, y, x, eta, lam, b, s, seed, 0, H)
    cg.casgd_check(ws)
    xg = x.cpu().numpy().astype(np.float64)
    xo = R.casgd(Xo, p.y, np.zeros(2048), eta, lam, b, s, seed, 0, H)
    err = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    print(f"\n[c2 scale] storage={storage} outer={H} rel_err={err:.3e}")
    assert err < 1e-4
