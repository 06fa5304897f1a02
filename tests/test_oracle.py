"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here touches the GPU path. Each test checks the oracle against
something other than its own formula: a second implementation, a library
routine, finite differences, closed forms or an algebraic identity.
"""
import math

import numpy as np
import pytest

from oracle import reference as R
from workloads import dense_c1, dense_logreg, sparse_zipf_logreg


def _tiny(m=8, n=5, seed=3):
    g = np.random.default_rng(seed)
    X = g.standard_normal((m, n)) / math.sqrt(n)
    y = np.where(g.standard_normal(m) >= 0, 1.0, -1.0)
    return X, y


# ------------------------------------------------------------------ sampling

def test_sampler_two_implementations_agree():
    # C core vs pure-Python integer model of the same published generator.
    for seed in (0, 42, 2**63 + 11):
        for t0 in (0, 1, 123456789):
            a = R.sample_indices(seed, t0, 257, 1 << 20)
            b = R.py_sample_indices(seed, t0, 257, 1 << 20)
            assert np.array_equal(a, b)


def test_sampler_range_and_uniformity():
    m = 97
    idx = R.sample_indices(42, 0, 200_000, m)
    assert idx.min() >= 0 and idx.max() < m
    cnt = np.bincount(idx, minlength=m)
    e = idx.size / m
    chi2 = ((cnt - e) ** 2 / e).sum()
    # 96 dof: mean 96, sd ~13.9; 6 sd margin
    assert chi2 < 96 + 6 * 13.9
    # consecutive pairs (serial test), 97^2 cells, 9408 dof
    pairs = idx[:-1] * m + idx[1:]
    cp = np.bincount(pairs, minlength=m * m)
    ep = pairs.size / (m * m)
    chi2p = ((cp - ep) ** 2 / ep).sum()
    assert chi2p < 9408 + 6 * math.sqrt(2 * 9408)


def test_sampler_with_replacement_repeats():
    # i.i.d. with replacement: the number of distinct values among q draws
    # from m has mean m (1 - (1 - 1/m)^q); 5000 draws from 1000 cover ~993.
    many = R.sample_indices(7, 0, 5000, 1000)
    k = len(np.unique(many))
    assert 980 <= k < 1000


# ------------------------------------------------------------------ residual

def test_delta_closed_forms():
    assert R.delta(0.0, 1.0) == 0.5
    assert R.delta(0.0, -1.0) == -0.5
    assert R.delta(800.0, 1.0) == 0.0          # y z -> +inf: residual -> 0
    assert R.delta(-800.0, 1.0) == 1.0         # y z -> -inf: residual -> y
    for z in (-3.0, -0.1, 0.7, 5.0):
        assert R.delta(z, -1.0) == -R.delta(-z, 1.0)
        # -dL/dr of log(1 + exp(-y r)) by central differences
        h = 1e-6
        L = lambda r: math.log1p(math.exp(-r))
        fd = -(L(z + h) - L(z - h)) / (2 * h)
        assert abs(R.delta(z, 1.0) - fd) < 1e-8


def test_sgd_step_is_gradient_step_finite_differences():
    X, y = _tiny()
    x0 = np.linspace(-0.3, 0.4, X.shape[1])
    eta, lam, b, seed = 0.7, 0.05, 4, 11
    x1 = R.sgd(X, y, x0, eta, lam, b, seed, 0, 1)
    I = R.sample_indices(seed, 0, b, X.shape[0])

    def f(x):
        z = X[I] @ x
        return np.mean(np.log1p(np.exp(-y[I] * z))) + 0.5 * lam * x @ x

    h = 1e-6
    grad = np.array([(f(x0 + h * e) - f(x0 - h * e)) / (2 * h) for e in np.eye(len(x0))])
    expect = x0 - eta * grad
    assert np.max(np.abs(x1 - expect)) < 1e-9 * max(1.0, np.max(np.abs(x0)))


def test_sgd_c_core_matches_numpy_second_implementation(c1):
    X, y = c1.X[:512], c1.y[:512]
    x = R.sgd(X, y, np.zeros(X.shape[1]), 0.5, 1e-4, 16, 42, 0, 50)
    xp = R.py_sgd(X, y, np.zeros(X.shape[1]), 0.5, 1e-4, 16, 42, 50)
    assert np.linalg.norm(x - xp) <= 1e-12 * np.linalg.norm(xp)


# --------------------------------------------------------- s-step exactness

def test_s1_is_sgd_bitwise(c1):
    X, y = c1.X, c1.y
    x0 = np.zeros(X.shape[1])
    a = R.sgd(X, y, x0, 0.5, 1e-4, 16, 42, 0, 60)
    b = R.casgd(X, y, x0, 0.5, 1e-4, 16, 1, 42, 0, 60)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("s", [2, 4, 16])
@pytest.mark.parametrize("lam", [0.0, 1e-4, 0.05])
def test_s_step_equals_sgd_on_same_samples(c1, s, lam):
    # Algorithm 1 is the composition of s mini-batch SGD steps (exact in real
    # arithmetic), so FP64 runs agree to rounding.
    X, y = c1.X, c1.y
    b, H = 16, 48 // s * 2
    x0 = np.zeros(X.shape[1])
    a = R.sgd(X, y, x0, 0.5, lam, b, 42, 0, H * s)
    c = R.casgd(X, y, x0, 0.5, lam, b, s, 42, 0, H)
    assert np.linalg.norm(a - c) <= 1e-12 * np.linalg.norm(a)


def test_inner_residuals_equal_sgd_residuals(c1):
    # delta_j of the recurrence equals the residual SGD computes at inner step j.
    X, y = c1.X[:1024], c1.y[:1024]
    b, s, eta, lam, seed = 8, 5, 0.5, 1e-3, 9
    x0 = np.random.default_rng(0).standard_normal(X.shape[1]) * 0.1
    parts = R.outer_parts(X, y, x0, eta, lam, b, s, seed, 3)
    x = x0.copy()
    for j in range(s):
        I = R.py_sample_indices(seed, 3 * s * b + j * b, b, X.shape[0])
        assert np.array_equal(I, parts["idx"][j * b:(j + 1) * b])
        z = X[I] @ x
        dj = y[I] * (1 - 1 / (1 + np.exp(-y[I] * z)))
        assert np.allclose(parts["delta"][j * b:(j + 1) * b], dj, rtol=1e-12, atol=1e-15)
        x = (1 - eta * lam) * x + (eta / b) * X[I].T @ dj


def test_outer_parts_gram_and_margin_match_numpy(c1):
    X, y = c1.X, c1.y
    b, s = 16, 4
    x0 = np.random.default_rng(1).standard_normal(X.shape[1])
    p = R.outer_parts(X, y, x0, 0.5, 1e-4, b, s, 42, 7)
    Y = X[p["idx"]]
    mask = R.strict_block_lower_mask(b, s)
    assert np.allclose(p["G"][mask], (Y @ Y.T)[mask], rtol=1e-13, atol=1e-15)
    assert np.all(p["G"][~mask] == 0)
    assert np.allclose(p["r"], Y @ x0, rtol=1e-13, atol=1e-14)
    # the update assembled from c reproduces one outer iteration
    beta = 1 - 0.5 * 1e-4
    x1 = beta ** s * x0 + (0.5 / b) * Y.T @ p["c"]
    assert np.allclose(x1, R.casgd(X, y, x0, 0.5, 1e-4, b, s, 42, 7, 1), rtol=1e-13)


def test_resume_is_exact(c1):
    X, y = c1.X, c1.y
    x0 = np.zeros(X.shape[1])
    full = R.casgd(X, y, x0, 0.5, 1e-4, 16, 4, 42, 0, 30)
    half = R.casgd(X, y, x0, 0.5, 1e-4, 16, 4, 42, 0, 13)
    rest = R.casgd(X, y, half, 0.5, 1e-4, 16, 4, 42, 13, 17)
    assert np.array_equal(full, rest)


def test_f32_input_path_equals_promoted_f64():
    p = dense_logreg(600, 40, 5, var=1 / 40, dtype=np.float32, noise_var=0.1)
    a = R.casgd(p.X, p.y, np.zeros(40), 0.5, 1e-4, 8, 4, 1, 0, 20)
    b = R.casgd(p.X.astype(np.float64), p.y.astype(np.float64), np.zeros(40), 0.5,
                1e-4, 8, 4, 1, 0, 20)
    assert np.array_equal(a, b)
    c = R.sgd(p.X, p.y, np.zeros(40), 0.5, 1e-4, 8, 1, 0, 80)
    d = R.sgd(p.X.astype(np.float64), p.y, np.zeros(40), 0.5, 1e-4, 8, 1, 0, 80)
    assert np.array_equal(c, d)


def test_sgd_decreases_test_loss(c1):
    x = R.casgd(c1.X, c1.y, np.zeros(256), 0.5, 1e-4, 16, 4, 42, 0, 200)
    l0 = R.logloss(c1.X_test, c1.y_test, np.zeros(256))
    l1 = R.logloss(c1.X_test, c1.y_test, x)
    assert abs(l0 - math.log(2)) < 1e-12
    assert l1 < 0.85 * l0


def test_logloss_stable_for_large_margins():
    X = np.array([[1.0], [1.0]])
    y = np.array([1.0, -1.0])
    x = np.array([1000.0])
    # log(1+e^-1000) ~ 0 and log(1+e^1000) = 1000 + log1p(e^-1000)
    assert abs(R.logloss(X, y, x) - 500.0) < 1e-12


# ---------------------------------------------------------------- sparse

def test_csr_oracle_equals_dense_oracle():
    p = sparse_zipf_logreg(3000, 512, 4, nnz_mean=12.0)
    D = p.to_dense().astype(np.float64)
    x0 = np.zeros(p.n)
    a = R.casgd_csr(p.row_ptr, p.col_idx, p.values, p.n, p.y, x0, 2.0, 1e-3, 8, 4, 5, 0, 25)
    b = R.casgd(D, p.y, x0, 2.0, 1e-3, 8, 4, 5, 0, 25)
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)
    assert abs(R.logloss_csr(p.row_ptr, p.col_idx, p.values, p.y, a)
               - R.logloss(D, p.y, a)) < 1e-13


# ---------------------------------------------------------- storage formats

def test_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(0)
    v = np.concatenate([g.standard_normal(10000).astype(np.float32) * 3,
                        np.array([1.00390625, 1.01171875, -2.0078125, 0.0], np.float32)])
    ours = R.bf16_round(v)
    ref = torch.from_numpy(v).to(torch.bfloat16).float().numpy()
    assert np.array_equal(ours, ref)


def test_fp16_matches_torch():
    torch = pytest.importorskip("torch")
    v = np.random.default_rng(1).standard_normal(10000).astype(np.float32)
    assert np.array_equal(R.fp16_round(v), torch.from_numpy(v).half().float().numpy())


def test_e4m3_table_and_encoder_match_torch():
    torch = pytest.importorskip("torch")
    vals = R.e4m3_values()
    assert vals[-1] == 448.0 and vals[1] == 2.0 ** -9 and vals[8] == 2.0 ** -6
    assert np.all(np.diff(vals) > 0)
    mids = (vals[:-1] + vals[1:]) / 2          # exact ties
    g = np.random.default_rng(2)
    v = np.concatenate([vals, mids, -mids, g.uniform(-448, 448, 20000),
                        g.standard_normal(20000) * 0.01]).astype(np.float32)
    v = v[np.abs(v) <= 448]
    ours = R.e4m3_decode(R.e4m3_encode(v))
    ref = torch.from_numpy(v).to(torch.float8_e4m3fn).float().numpy().astype(np.float64)
    assert np.array_equal(ours, ref)
    assert np.all(R.e4m3_decode(R.e4m3_encode(np.array([500.0, -1e6], np.float32)))
                  == np.array([448.0, -448.0]))


def test_fp8_row_quantisation_error_bound():
    X = (np.random.default_rng(3).standard_normal((64, 256)) / 16).astype(np.float32)
    X[5] = 0.0
    codes, scale, deq = R.quantize_rows_e4m3(X)
    assert scale[5] == 1.0 and np.all(deq[5] == 0)
    amax = np.abs(X).max(axis=1)
    for i in range(64):
        if amax[i] == 0:
            continue
        err = np.abs(deq[i] - X[i].astype(np.float64))
        # normal range: relative u = 2^-4 (plus the FP32 pre-scaling rounding);
        # subnormal range: half a subnormal step times the scale
        lim = np.maximum(np.abs(X[i]) * (R.U_E4M3 + 2 * R.U_FP32), 2.0 ** -10 * scale[i])
        assert np.all(err <= lim * (1 + 1e-12))
        assert np.max(np.abs(R.e4m3_decode(codes[i]))) == 448.0


# ---------------------------------------------------------------- bounds

def test_gamma_validity_and_fp32_correction_requirement():
    assert R.gamma(10, 0.01) == pytest.approx(0.1 / 0.9)
    # (s-1) b u_c < 1 is what makes the correction-sum factor valid: BF16 fails
    # it at the paper's operating points, FP32 does not.
    assert math.isinf(R.gamma((64 - 1) * 32, R.U_BF16))
    assert R.gamma((64 - 1) * 32, R.U_FP32) < 1e-3


def test_amplification_factor_neumann_equals_inverse(c1):
    from workloads import normalize_rows
    X = normalize_rows(c1.X)
    b, s, eta = 16, 4, 0.5
    idx = R.sample_indices(42, 0, s * b, X.shape[0])
    Y = X[idx]
    res = R.uniform_precision_bound(Y, np.zeros(256), c1.y[idx], b, s, eta, R.U_FP32)
    GL = np.where(R.strict_block_lower_mask(b, s), Y @ Y.T, 0.0)
    M = 0.25 * (eta / b) * np.abs(GL)
    ref = np.linalg.norm(np.linalg.inv(np.eye(s * b) - M), 2)
    assert res["K_s"] == pytest.approx(ref, rel=1e-12)
    assert res["Omega"] < 0.5


def test_bound_dominates_fp32_simulation(c1):
    """Thm. 5.1 / Cor. 5.2 (P = 1): an all-FP32 evaluation of one outer
    iteration stays inside the uniform-precision bound."""
    from workloads import normalize_rows
    X = normalize_rows(c1.X)
    b, s, eta = 16, 4, 0.5
    x = np.random.default_rng(4).standard_normal(256) * 0.5
    idx = R.sample_indices(42, 0, s * b, X.shape[0])
    Y, yI = X[idx], c1.y[idx].astype(np.float64)
    res = R.uniform_precision_bound(Y, x, yI, b, s, eta, R.U_FP32)
    f = np.float32
    Y32, x32 = Y.astype(f), x.astype(f)
    r = (Y32 @ x32).astype(f)
    G = (Y32 @ Y32.T).astype(f)
    d = np.zeros(s * b, f)
    for j in range(s):
        rows = slice(j * b, (j + 1) * b)
        z = r[rows] + f(eta / b) * (G[rows, :j * b] @ d[:j * b]) if j else r[rows]
        yy = yI[rows].astype(f)
        d[rows] = yy / (f(1) + np.exp(yy * z))
    x_s = x32 + f(eta / b) * (Y32.T @ d)
    err = np.linalg.norm(x_s.astype(np.float64) - res["x_exact"])
    assert err <= res["bound"]


# ------------------------------------------------------ stats and the MLP

def test_column_stats_match_numpy():
    X = np.random.default_rng(5).standard_normal((300, 7))
    X[:, 2] = 0
    X[::3, 4] = 0
    st = R.column_stats(X)
    assert np.allclose(st[:, 0], X.mean(axis=0))
    assert np.allclose(st[:, 1], X.var(axis=0))
    assert np.allclose(st[:, 2], np.count_nonzero(X, axis=0) / 300)
    assert np.allclose(st[:, 3], np.abs(X).max(axis=0))


def test_column_stats_csr_matches_dense():
    p = sparse_zipf_logreg(2000, 300, 6, nnz_mean=10.0)
    D = p.to_dense()
    a = R.column_stats_csr(p.row_ptr, p.col_idx, p.values, p.m, p.n)
    assert np.allclose(a, R.column_stats(D), rtol=1e-9, atol=1e-12)


def test_mlp_gradients_match_finite_differences():
    g = np.random.default_rng(6)
    N, Hd, P = 40, 16, 3
    F = g.standard_normal((N, 4))
    seg = np.sort(g.integers(0, P, N))
    seg[:P] = np.arange(P)
    seg = np.sort(seg)
    t_d = g.standard_normal(N)
    t_eta = g.standard_normal(P)
    W1, b1 = g.standard_normal((Hd, 4)) * 0.5, g.standard_normal(Hd) * 0.1
    W2, b2 = g.standard_normal((2, Hd)) * 0.5, g.standard_normal(2) * 0.1

    def L(W1, b1, W2, b2):
        o, _, _ = R.mlp_forward(F, W1, b1, W2, b2)
        return R.mlp_loss(o, seg, t_d, t_eta)[0]

    o, h, pre = R.mlp_forward(F, W1, b1, W2, b2)
    _, go = R.mlp_loss(o, seg, t_d, t_eta)
    grads = R.mlp_backward(F, h, pre, W2, go)
    params = [W1, b1, W2, b2]
    eps = 1e-6
    for pi, (p, gp) in enumerate(zip(params, grads)):
        flat = p.reshape(-1)
        for k in range(0, flat.size, max(1, flat.size // 11)):
            old = flat[k]
            flat[k] = old + eps
            lp = L(*params)
            flat[k] = old - eps
            lm = L(*params)
            flat[k] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - gp.reshape(-1)[k]) < 1e-6 * max(1.0, abs(fd)), (pi, k)


def test_hess_diag_matches_second_differences_of_objective():
    # H_kk is the second derivative of F_lambda along coordinate k; the
    # objective is a separate code path (stable softplus, no sigmoid).
    g = np.random.default_rng(7)
    X = g.standard_normal((200, 6))
    y = np.where(g.random(200) < 0.5, -1.0, 1.0)
    x = g.standard_normal(6) * 0.4
    lam = 1e-2
    h = R.hess_diag(X * y[:, None], x, lam)  # sign of the label cancels in s(1-s) X^2
    assert np.allclose(h, R.hess_diag(X, x, lam), rtol=1e-13)
    e = 1e-4
    for k in range(6):
        u = np.zeros(6)
        u[k] = e
        fd = (R.objective(X, y, x + u, lam) - 2 * R.objective(X, y, x, lam)
              + R.objective(X, y, x - u, lam)) / e ** 2
        assert abs(fd - h[k]) < 1e-6 * max(1.0, h[k]), k


def test_jacobi_target_unit_geometric_mean_and_scale():
    h = np.array([4.0, 1.0, 0.25, 16.0])
    t, q = R.jacobi_target(h)
    assert abs(t.sum()) < 1e-14
    # q^2 h is constant: the scaled Hessian diagonal is uniform
    assert np.allclose(q * q * h, (q * q * h)[0], rtol=1e-14)
    assert np.allclose(np.exp(t.mean()), 1.0)


def test_feature_norm_standardises_features():
    st = np.abs(np.random.default_rng(8).standard_normal((500, 4))) * [1, 10, 0.1, 3]
    mu, sd = R.feature_norm(st)
    F = R.mlp_features(st, mu, sd)
    assert np.allclose(F.mean(axis=0), 0.0, atol=1e-12)
    assert np.allclose(F.std(axis=0, ddof=1), 1.0, rtol=1e-12)
    const = np.ones((10, 4))
    assert np.all(R.feature_norm(const)[1] == 1e-6)


def test_mlp_apply_centres_and_clips():
    o = np.array([[1.0, 0.0], [3.0, np.log(4.0)], [50.0, np.log(0.25)], [-40.0, 0.0]])
    q, eta = R.mlp_apply(o)
    assert np.allclose(np.log(q) * 2, [-2.5, -0.5, 20.0, -20.0])
    assert np.isclose(eta, 1.0)


def test_adam_first_step_is_signed_lr():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    p1, _, _ = R.adam_step(p, g, np.zeros(3), np.zeros(3), 1, 0.01)
    # bias-corrected moments give m/sqrt(v) = sign(g) on the first step
    assert np.allclose(p1, p - 0.01 * np.sign(g), atol=1e-7)
