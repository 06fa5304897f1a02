"""Further pins of the FP64 oracle: known-answer vectors, closed forms and
hand-computed cases for the parts that a second implementation or a library
routine alone does not fix.

* SplitMix64 known-answer outputs of the published generator (Steele, Lea and
  Flood, OOPSLA 2014; the reference C implementation's first outputs for
  state 0 and for state 1234567).
* The FP32-input loss the golden targets come from, against the FP64 loss on
  the promoted values and against NumPy's logaddexp.
* The local error bound of the mixed-precision theorem (Sec. 5.2, eq. for the
  nine E-terms, P = 1) on hand-sized blocks whose norms, amplification factor
  and source quantities have closed forms; every slot gets its own unit
  roundoff so that a term fed the wrong slot, a wrong power of alpha, the
  Frobenius norm in place of the spectral norm, |G| in place of H_L or a
  missing jb factor changes a term by far more than the tolerance.
* Adam (Kingma and Ba, 2015) over many steps against the closed-form moment
  recursions for a constant and for an alternating gradient.
"""
import math

import numpy as np
import pytest

from oracle import reference as R


# ------------------------------------------------------- SplitMix64 vectors

# First outputs of the reference SplitMix64 generator (state += golden gamma,
# then the variant-13 mix) for the initial states 0 and 1234567.
KAT = {
    0: [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F],
    1234567: [6457827717110365317, 3203168211198807973, 9817491932198370423,
              4593380528125082431, 16408922859458223821],
}


@pytest.mark.parametrize("seed", sorted(KAT))
def test_splitmix64_known_answers(seed):
    for t, want in enumerate(KAT[seed]):
        assert R.splitmix64(seed, t) == want
        assert R._py_splitmix(seed, t) == want


def test_sample_index_is_high_half_of_product():
    # row = floor(u m / 2^64): with m = 2^32 it is the top 32 bits of u
    idx = R.sample_indices(1234567, 0, 5, 1 << 32)
    assert list(idx) == [v >> 32 for v in KAT[1234567]]
    idx = R.sample_indices(0, 0, 3, 1000)
    assert list(idx) == [(v * 1000) >> 64 for v in KAT[0]]


# --------------------------------------------------------- FP32-input loss

def test_logloss_f32_equals_promoted_f64_and_logaddexp():
    g = np.random.default_rng(11)
    m, n = 3000, 70      # m*n above the oracle's threading threshold
    X32 = (g.standard_normal((m, n)) / math.sqrt(n)).astype(np.float32)
    X32[:, 5] *= 10
    y32 = np.where(g.random(m) < 0.5, -1.0, 1.0).astype(np.float32)
    x = g.standard_normal(n) * 0.7
    a = R.logloss(X32, y32, x)
    b = R.logloss(X32.astype(np.float64), y32.astype(np.float64), x)
    # same terms; the threaded FP32-input sum adds them in another order
    assert abs(a - b) <= 1e-13 * b
    z = X32.astype(np.float64) @ x
    c = float(np.mean(np.logaddexp(0.0, -y32.astype(np.float64) * z)))
    assert abs(a - c) <= 1e-12 * c
    # x = 0: every term is log 2 (the sum of m of them rounds m times)
    assert abs(R.logloss(X32, y32, np.zeros(n)) - math.log(2.0)) <= m * 2.0 ** -52


# ------------------------------------------------ Thm. 5.1 local error bound

def _lam_max_sym2(a, b, c):
    """Largest eigenvalue of the symmetric 2x2 matrix [[a, b], [b, c]]."""
    return 0.5 * (a + c) + math.sqrt(0.25 * (a - c) ** 2 + b * b)


def _sig_max_2x2(B):
    """Largest singular value of a 2x2 matrix from the eigenvalues of B^T B."""
    (p, q), (r, t) = B
    return math.sqrt(_lam_max_sym2(p * p + r * r, p * q + r * t, q * q + t * t))


def _unit_lower_norm(c):
    """2-norm of [[I, 0], [B, I]] when B has largest singular value c:
    (c + sqrt(c^2 + 4)) / 2."""
    return 0.5 * (c + math.sqrt(c * c + 4.0))


U = dict(u_A=1.1e-3, gamma_r=2.3e-3, gamma_G=3.7e-3, u_c=5.3e-3, u_sigma=7.9e-3,
         gamma_g=1.13e-2, u_x=1.71e-2)


def _check_terms(res, want):
    assert set(res["E"]) == set(want)
    for k, v in want.items():
        assert res["E"][k] == pytest.approx(v, rel=1e-12, abs=1e-300), k


def test_local_bound_single_block_closed_form():
    # s = 1, b = 2, n = 2: no Gram block, K_s = 1, T_G = T_c = 0.
    Y = np.array([[0.6, 0.8], [0.6, -0.8]])
    x = np.array([0.5, -0.25])
    yI = np.array([1.0, -1.0])
    eta, b, s = 0.9, 2, 1
    alpha = eta / b
    res = R.local_error_bound(Y, x, yI, b, s, eta, **U)
    # hand values
    normY = math.sqrt(1.28)                 # Y^T Y = diag(0.72, 1.28); ||Y||_F = sqrt(2)
    r = np.array([0.6 * 0.5 - 0.8 * 0.25, 0.6 * 0.5 + 0.8 * 0.25])   # (0.1, 0.5)
    d = np.array([1.0 / (1.0 + math.exp(0.1)), -1.0 / (1.0 + math.exp(-0.5))])
    T_r = math.hypot(0.6 * 0.5 + 0.8 * 0.25, 0.6 * 0.5 + 0.8 * 0.25)   # |Y||x| = (0.5, 0.5)
    T_g = math.hypot(0.6 * abs(d[0]) + 0.6 * abs(d[1]), 0.8 * abs(d[0]) + 0.8 * abs(d[1]))
    g = np.array([0.6 * d[0] + 0.6 * d[1], 0.8 * d[0] - 0.8 * d[1]])
    xs = x + alpha * g
    assert res["K_s"] == pytest.approx(1.0, rel=1e-15)
    assert np.allclose(res["x_exact"], xs, rtol=1e-15, atol=1e-16)
    a1 = alpha * normY * 1.0 * 0.25
    want = dict(
        A=a1 * U["u_A"] * T_r + alpha * U["u_A"] * T_g,
        r=a1 * U["gamma_r"] * T_r,
        G=0.0,
        c=a1 * U["u_c"] * T_r,
        sigma=alpha * normY * 1.0 * 8.0 * U["u_sigma"] * 1.0 * math.sqrt(2.0),
        g=alpha * U["gamma_g"] * T_g,
        x=U["u_x"] * (math.hypot(*xs) + alpha * math.hypot(*g)),
    )
    _check_terms(res, want)
    omega = max(U["u_A"], U["gamma_r"], U["gamma_G"], R.gamma(0, U["u_c"]), U["gamma_g"],
                U["u_sigma"], U["u_x"])
    assert res["Omega"] == pytest.approx(omega, rel=1e-15)   # tau = 0: H_L = 0
    assert res["bound"] == pytest.approx((1 + 2 * omega) * sum(want.values()), rel=1e-12)


def test_local_bound_two_blocks_closed_form():
    # s = 2, b = 2, n = 2: one Gram block G_{1,0} (2x2) whose signs differ
    # from H_{1,0} = |Y_1||Y_0|^T, so |G_L| != H_L; jb = 2 in T_c.
    Y0 = np.array([[0.6, 0.8], [1.0, 0.0]])
    Y1 = np.array([[0.6, -0.8], [0.0, -0.5]])
    Y = np.vstack([Y0, Y1])
    x = np.array([0.3, 0.2])
    yI = np.array([1.0, -1.0, -1.0, 1.0])
    eta, b, s = 1.4, 2, 2
    alpha = eta / b                                   # 0.7: alpha and alpha^2 differ
    res = R.local_error_bound(Y, x, yI, b, s, eta, **U)

    # Gram block and its magnitude version, entry by entry
    G10 = np.array([[0.6 * 0.6 - 0.8 * 0.8, 0.6 * 1.0],
                    [-0.5 * 0.8, 0.0]])                # [[-0.28, 0.6], [-0.4, 0]]
    H10 = np.array([[0.6 * 0.6 + 0.8 * 0.8, 0.6 * 1.0],
                    [0.5 * 0.8, 0.0]])                 # [[1.0, 0.6], [0.4, 0]]
    # exact lambda = 0 recurrence
    r = np.array([0.6 * 0.3 + 0.8 * 0.2, 0.3, 0.6 * 0.3 - 0.8 * 0.2, -0.5 * 0.2])
    dlt = lambda z, yy: yy / (1.0 + math.exp(yy * z))
    d0 = np.array([dlt(r[0], 1.0), dlt(r[1], -1.0)])
    z1 = r[2:] + alpha * (G10 @ d0)
    d1 = np.array([dlt(z1[0], -1.0), dlt(z1[1], 1.0)])
    d = np.concatenate([d0, d1])
    # ||Y||_2 from the 2x2 Y^T Y (closed-form eigenvalue)
    YtY = Y.T @ Y
    normY = math.sqrt(_lam_max_sym2(YtY[0, 0], YtY[0, 1], YtY[1, 1]))
    assert abs(normY - math.sqrt(np.sum(Y * Y))) > 0.1        # not the Frobenius norm
    # K_s = ||(I - M)^-1|| = ||I + M||, M = alpha/4 |G_L| (M^2 = 0)
    K_s = _unit_lower_norm(0.25 * alpha * _sig_max_2x2(np.abs(G10)))
    assert res["K_s"] == pytest.approx(K_s, rel=1e-12)
    T_r = float(np.linalg.norm(np.abs(Y) @ np.abs(x)))
    T_g = float(np.linalg.norm(np.abs(Y).T @ np.abs(d)))
    T_G = float(np.linalg.norm(H10 @ np.abs(d0)))          # H_L |d| has only block 1
    T_c = 1 * b * math.sqrt(np.sum(G10 * G10)) * float(np.linalg.norm(d0))
    normH = _sig_max_2x2(H10)
    xs = x + alpha * (Y.T @ d)
    assert np.allclose(res["x_exact"], xs, rtol=1e-14, atol=1e-16)
    a1 = alpha * normY * K_s * 0.25
    want = dict(
        A=a1 * U["u_A"] * T_r + 2 * alpha * a1 * U["u_A"] * T_G + alpha * U["u_A"] * T_g,
        r=a1 * U["gamma_r"] * T_r,
        G=alpha * a1 * U["gamma_G"] * T_G,
        c=a1 * U["u_c"] * T_r + 2 * alpha * a1 * U["u_c"] * T_G + alpha * a1 * U["u_c"] * T_c,
        sigma=alpha * normY * K_s * 8.0 * U["u_sigma"] * 1.0 * math.sqrt(4.0),
        g=alpha * U["gamma_g"] * T_g,
        x=U["u_x"] * (float(np.linalg.norm(xs)) + alpha * float(np.linalg.norm(Y.T @ d))),
    )
    _check_terms(res, want)
    tau = K_s * 0.25 * alpha * (2 * U["u_A"] + U["gamma_G"]) * normH
    omega = max(U["u_A"], U["gamma_r"], U["gamma_G"], R.gamma(2, U["u_c"]), U["gamma_g"],
                U["u_sigma"], U["u_x"])
    assert res["Omega"] == pytest.approx(max(omega, tau), rel=1e-12)


def test_local_bound_terms_vanish_with_their_slot():
    # each E-term is first order in its own slot only: zeroing one slot
    # zeroes exactly its term (the shared-source rows A and c aside)
    g = np.random.default_rng(3)
    b, s, n, eta = 4, 3, 6, 0.8
    Y = g.standard_normal((s * b, n)) / math.sqrt(n)
    x = g.standard_normal(n) * 0.3
    yI = np.where(g.random(s * b) < 0.5, -1.0, 1.0)
    base = R.local_error_bound(Y, x, yI, b, s, eta, **U)
    slot_of = dict(u_A="A", gamma_r="r", gamma_G="G", u_c="c", u_sigma="sigma",
                   gamma_g="g", u_x="x")
    for slot, term in slot_of.items():
        kw = dict(U)
        kw[slot] = 0.0
        res = R.local_error_bound(Y, x, yI, b, s, eta, **kw)
        assert res["E"][term] == 0.0, slot
        for other in res["E"]:
            if other != term:
                assert res["E"][other] == pytest.approx(base["E"][other], rel=1e-12), (slot,
                                                                                       other)
        # doubling the slot doubles its term
        kw[slot] = 2 * U[slot]
        res2 = R.local_error_bound(Y, x, yI, b, s, eta, **kw)
        assert res2["E"][term] == pytest.approx(2 * base["E"][term], rel=1e-12), slot


# ------------------------------------------------------------------ Adam

def test_adam_constant_gradient_closed_form():
    # constant g: m1_t = (1 - b1^t) g, m2_t = (1 - b2^t) g^2, so every
    # bias-corrected step is lr * g / (|g| + eps)
    g = np.array([0.5, -4.0, 1e-3, 2.5])
    p0 = np.array([1.0, -2.0, 3.0, 0.0])
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    p, m1, m2 = p0.copy(), np.zeros(4), np.zeros(4)
    for t in range(1, 41):
        p, m1, m2 = R.adam_step(p, g, m1, m2, t, lr, b1, b2, eps)
        assert np.allclose(m1, (1 - b1 ** t) * g, rtol=1e-13, atol=0)
        assert np.allclose(m2, (1 - b2 ** t) * g * g, rtol=1e-13, atol=0)
    assert np.allclose(p, p0 - 40 * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-14)


def test_adam_alternating_gradient_closed_form():
    # g_t = (-1)^t g: m1_t = (1 - b1) g (-1)^t (1 - (-b1)^t) / (1 + b1),
    # m2_t = (1 - b2^t) g^2; the step of t is lr m1_t/(1-b1^t) / (|g| + eps)
    g = np.array([0.3, -1.5])
    p0 = np.array([0.2, 0.1])
    lr, b1, b2, eps = 5e-3, 0.8, 0.99, 1e-8
    p, m1, m2 = p0.copy(), np.zeros(2), np.zeros(2)
    expect_p = p0.copy()
    for t in range(1, 26):
        p, m1, m2 = R.adam_step(p, (-1) ** t * g, m1, m2, t, lr, b1, b2, eps)
        em1 = (1 - b1) * g * (-1) ** t * (1 - (-b1) ** t) / (1 + b1)
        em2 = (1 - b2 ** t) * g * g
        assert np.allclose(m1, em1, rtol=1e-12, atol=1e-15)
        assert np.allclose(m2, em2, rtol=1e-12, atol=0)
        expect_p = expect_p - lr * (em1 / (1 - b1 ** t)) / (np.abs(g) + eps)
    assert np.allclose(p, expect_p, rtol=1e-12, atol=1e-15)


# ------------------------------------------------- small remaining pieces

def test_lowp_fp32acc_factor_dominates_simulated_products():
    # BF16 inputs, FP32 accumulation (Sec. 5.2, the effective factor
    # 2 u_16 + gamma_n(u_32)): a sequential FP32 sum of products of
    # BF16-rounded FP32 inputs stays within the factor times |x|^T |y|,
    # and the factor is not loose by orders of magnitude.
    g = np.random.default_rng(21)
    n = 2048
    worst = 0.0
    for _ in range(40):
        x = g.standard_normal(n).astype(np.float32)
        y = g.standard_normal(n).astype(np.float32) + 0.5
        xb, yb = R.bf16_round(x), R.bf16_round(y)
        acc = np.float32(0.0)
        for k in range(n):
            acc = np.float32(acc + np.float32(xb[k] * yb[k]))
        exact = float(x.astype(np.float64) @ y.astype(np.float64))
        scale = float(np.abs(x.astype(np.float64)) @ np.abs(y.astype(np.float64)))
        worst = max(worst, abs(float(acc) - exact) / scale)
    f = R.lowp_fp32acc_factor(n, R.U_BF16)
    assert worst <= f
    assert worst > 1e-3 * f


def test_mlp_forward_and_loss_hand_case():
    # one hidden unit active, one cut by the ReLU
    F = np.array([[1.0, 2.0, 0.0, -1.0], [0.5, 0.0, 1.0, 1.0]])
    W1 = np.array([[1.0, 0.0, 0.0, 0.0], [0.0, -1.0, 0.0, 0.0]])
    b1 = np.array([0.5, 0.25])
    W2 = np.array([[2.0, 3.0], [-1.0, 1.0]])
    b2 = np.array([0.1, -0.2])
    o, h, pre = R.mlp_forward(F, W1, b1, W2, b2)
    assert np.array_equal(pre, [[1.5, -1.75], [1.0, 0.25]])
    assert np.array_equal(h, [[1.5, 0.0], [1.0, 0.25]])
    assert np.allclose(o, [[3.1, -1.7], [2.85, -0.95]], rtol=0, atol=1e-15)
    # two problems of one row each: loss = mean (o0 - t_d)^2 + w mean (o1 - t_eta)^2
    loss, go = R.mlp_loss(o, np.array([0, 1]), np.array([3.0, 3.0]), np.array([-1.0, -1.0]),
                          w_eta=0.5)
    want = (0.1 ** 2 + 0.15 ** 2) / 2 + 0.5 * (0.7 ** 2 + 0.05 ** 2) / 2
    assert loss == pytest.approx(want, rel=1e-13)
    assert np.allclose(go, [[0.1, 0.5 * 2 * -0.7 / 2], [-0.15, 0.5 * 2 * 0.05 / 2]], atol=1e-14)
