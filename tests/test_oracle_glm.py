"""Pins of the oracle's linear and Poisson losses (Sec. 2.1 losses, Sec. 3.1
residuals): closed forms, finite differences of the paper's loss
definitions, a linear solve that the linear recurrence must equal, recovery
of the planted solution on noise-free linear data, and the s-step
reformulation's exactness for both losses."""
import math

import numpy as np
import pytest

from oracle import reference as R
from workloads import dense_glm, sparse_zipf_glm

LOSS = {"linear": lambda z, y: 0.5 * (z - y) ** 2,          # Sec. 2.1
        "poisson": lambda z, y: math.exp(z) - y * z}


@pytest.mark.parametrize("loss", ["linear", "poisson"])
def test_residual_is_minus_loss_derivative(loss):
    h = 1e-6
    for z in (-2.0, -0.3, 0.0, 0.4, 1.7):
        for y in (0.0, 1.0, 3.0, -0.5):
            if loss == "poisson" and y < 0:
                continue
            fd = -(LOSS[loss](z + h, y) - LOSS[loss](z - h, y)) / (2 * h)
            assert abs(R.delta(z, y, loss) - fd) < 1e-7 * max(1.0, abs(fd)), (z, y)


def test_residual_closed_forms():
    assert R.delta(0.75, 2.0, "linear") == 1.25
    assert R.delta(0.0, 3.0, "poisson") == 2.0            # y - e^0
    assert abs(R.delta(math.log(3.0), 3.0, "poisson")) < 1e-15
    assert R.delta(0.0, 1.0, "logistic") == 0.5


def test_loss_values_closed_forms():
    X = np.array([[1.0, 0.0], [0.0, 2.0], [1.0, 1.0]])
    y = np.array([1.0, 4.0, 0.0])
    x = np.array([1.0, 2.0])                              # margins (1, 4, 3)
    assert R.loss_value(X, y, x, "linear") == pytest.approx((0 + 0 + 4.5) / 3, rel=1e-15)
    # Poisson at x = 0: every term is e^0 - 0 = 1
    assert R.loss_value(X, y, np.zeros(2), "poisson") == 1.0
    want = (math.e - 1.0 + math.exp(4.0) - 16.0 + math.exp(3.0)) / 3
    assert R.loss_value(X, y, x, "poisson") == pytest.approx(want, rel=1e-15)
    # FP32-input path equals the promoted FP64 one
    X32 = X.astype(np.float32)
    assert R.loss_value(X32, y.astype(np.float32), x, "poisson") == R.loss_value(
        X32.astype(np.float64), y, x, "poisson")


@pytest.mark.parametrize("loss", ["linear", "poisson"])
def test_sgd_step_is_gradient_step_finite_differences(loss):
    g = np.random.default_rng(5)
    m, n, b, eta, lam, seed = 9, 4, 4, 0.3, 0.05, 17
    X = g.standard_normal((m, n)) / 2
    y = g.poisson(1.0, m).astype(float) if loss == "poisson" else g.standard_normal(m)
    x0 = g.standard_normal(n) * 0.3
    x1 = R.sgd(X, y, x0, eta, lam, b, seed, 0, 1, loss=loss)
    I = R.sample_indices(seed, 0, b, m)

    def f(x):
        z = X[I] @ x
        return np.mean([LOSS[loss](zz, yy) for zz, yy in zip(z, y[I])]) + 0.5 * lam * x @ x

    h = 1e-6
    grad = np.array([(f(x0 + h * e) - f(x0 - h * e)) / (2 * h) for e in np.eye(n)])
    assert np.max(np.abs(x1 - (x0 - eta * grad))) < 1e-8


@pytest.mark.parametrize("loss", ["linear", "poisson"])
def test_c_core_matches_numpy_second_implementation(loss):
    p = dense_glm(600, 32, 3, loss, var=1 / 32)
    x = R.sgd(p.X, p.y, np.zeros(32), 0.2, 1e-3, 8, 9, 0, 60, loss=loss)
    xp = R.py_sgd(p.X, p.y, np.zeros(32), 0.2, 1e-3, 8, 9, 60, loss=loss)
    assert np.linalg.norm(x - xp) <= 1e-12 * np.linalg.norm(xp)


@pytest.mark.parametrize("loss", ["linear", "poisson"])
def test_s1_is_sgd_bitwise_and_s_step_equals_sgd(loss):
    p = dense_glm(2048, 64, 7, loss, var=1 / 64)
    x0 = np.zeros(64)
    a = R.sgd(p.X, p.y, x0, 0.25, 1e-4, 16, 42, 0, 64, loss=loss)
    b1 = R.casgd(p.X, p.y, x0, 0.25, 1e-4, 16, 1, 42, 0, 64, loss=loss)
    assert np.array_equal(a, b1)
    for s in (2, 4, 16):
        c = R.casgd(p.X, p.y, x0, 0.25, 1e-4, 16, s, 42, 0, 64 // s, loss=loss)
        assert np.linalg.norm(a - c) <= 1e-12 * np.linalg.norm(a), s


def test_linear_recurrence_is_a_triangular_solve():
    # delta_j = y_j - beta^j r_j - alpha sum_{i<j} beta^(j-1-i) G_{j,i} delta_i, i.e.
    # (I + alpha Gb) delta = y - B r with Gb the decay-weighted strict
    # block-lower Gram and B = diag(beta^j): a linear system.
    g = np.random.default_rng(8)
    b, s, n, eta, lam = 3, 5, 7, 0.6, 0.2
    Y = g.standard_normal((s * b, n)) / math.sqrt(n)
    r = g.standard_normal(s * b)
    yI = g.standard_normal(s * b)
    G = np.where(R.strict_block_lower_mask(b, s), Y @ Y.T, 0.0)
    d, c = R.inner_corrections(G, r, yI, b, s, eta, lam, loss="linear")
    beta, alpha = 1 - eta * lam, eta / b
    blk = np.arange(s * b) // b
    W = np.where(blk[:, None] > blk[None, :], beta ** (blk[:, None] - 1 - blk[None, :]), 0.0)
    A = np.eye(s * b) + alpha * W * G
    want = np.linalg.solve(A, yI - beta ** blk * r)
    assert np.allclose(d, want, rtol=1e-12, atol=1e-13)
    assert np.allclose(c, beta ** (s - 1 - blk) * want, rtol=1e-12, atol=1e-13)


def test_linear_sgd_recovers_planted_solution_without_noise():
    # consistent data (y = X w exactly) and no regularisation: w is the
    # unique minimiser with zero loss, and SGD converges to it linearly
    p = dense_glm(512, 16, 9, "linear", var=1 / 16, noise_var=0.0)
    y = (p.X @ p.w_true).astype(np.float64)
    x = R.casgd(p.X, y, np.zeros(16), 0.5, 0.0, 8, 4, 1, 0, 1500, loss="linear")
    assert np.linalg.norm(x - p.w_true) <= 1e-8 * np.linalg.norm(p.w_true)
    assert R.loss_value(p.X, y, x, "linear") < 1e-16


def test_poisson_sgd_decreases_loss_towards_planted():
    p = dense_glm(4096, 32, 4, "poisson", var=1 / 32)
    x = R.casgd(p.X, p.y, np.zeros(32), 0.1, 0.0, 16, 4, 2, 0, 400, loss="poisson")
    l0 = R.loss_value(p.X_test, p.y_test, np.zeros(32), "poisson")
    l1 = R.loss_value(p.X_test, p.y_test, x, "poisson")
    lw = R.loss_value(p.X_test, p.y_test, 0.5 * p.w_true, "poisson")
    assert l1 < l0 and l1 < lw + 0.05 * (l0 - lw)


@pytest.mark.parametrize("loss", ["linear", "poisson"])
def test_csr_oracle_equals_dense_oracle(loss):
    p = sparse_zipf_glm(3000, 512, 4, loss, nnz_mean=12.0)
    D = p.to_dense().astype(np.float64)
    x0 = np.zeros(p.n)
    a = R.casgd_csr(p.row_ptr, p.col_idx, p.values, p.n, p.y, x0, 1.0, 1e-3, 8, 4, 5, 0, 25,
                    loss=loss)
    b = R.casgd(D, p.y, x0, 1.0, 1e-3, 8, 4, 5, 0, 25, loss=loss)
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)
    assert abs(R.loss_value_csr(p.row_ptr, p.col_idx, p.values, p.y, a, loss)
               - R.loss_value(D, p.y, a, loss)) < 1e-13


@pytest.mark.parametrize("loss", ["logistic", "linear", "poisson"])
def test_outer_rows_equals_sampled_outer_iteration(loss):
    """The outer iteration on given rows is the sampled outer iteration with
    the sampling and gather steps taken out: bitwise equal to casgd on the
    rows that outer iteration samples, and its pieces equal outer_parts."""
    p = dense_glm(3000, 48, 21, loss, var=1 / 48)
    x = np.random.default_rng(4).standard_normal(48) * 0.1
    b, s, eta, lam, seed, h = 8, 5, 0.3, 1e-3, 5, 7
    idx = R.sample_indices(seed, h * s * b, s * b, p.X.shape[0])
    o = R.outer_rows(p.X[idx], p.y[idx], x, eta, lam, b, s, loss=loss)
    x1 = R.casgd(p.X, p.y, x, eta, lam, b, s, seed, h, 1, loss=loss)
    assert np.array_equal(o["x"], x1)
    parts = R.outer_parts(p.X, p.y, x, eta, lam, b, s, seed, h, loss=loss)
    for k in ("r", "delta", "c"):
        assert np.array_equal(o[k], parts[k])
    low = np.tril(np.ones((s * b, s * b)), -1) * (np.arange(s * b)[:, None] // b
                                                   > np.arange(s * b)[None, :] // b)
    assert np.array_equal(o["G"] * low, parts["G"] * low)
