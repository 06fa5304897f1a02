"""The error bounds of the GPU parity tests hold for an FP32 simulation of
one outer iteration and fail for a planted mistake (CPU only)."""
import numpy as np
import pytest

from oracle import reference as R
from workloads import dense_glm
from _bounds import U32, outer_bound


def _fp32_outer(Y, yI, x, eta, lam, b, s, loss, drop_far=False, acc=np.float32):
    """One outer iteration with FP32 margins, Gram and update (BLAS sgemm/sgemv)
    and corrections in `acc`; drop_far leaves out block 0 of the sums of the
    last row block (a plausible indexing mistake)."""
    Y32 = Y.astype(np.float32)
    r = (Y32 @ x.astype(np.float32)).astype(acc)
    G = (Y32 @ Y32.T).astype(acc)
    sb = s * b
    alpha, beta = acc(eta / b), acc(1 - eta * lam)
    d = np.zeros(sb, acc)
    for j in range(s):
        for q in range(b):
            t = j * b + q
            a = acc(0)
            for i in range(j):
                if drop_far and j == s - 1 and i == 0:
                    continue
                a += beta ** (j - 1 - i) * np.dot(G[t, i * b:(i + 1) * b], d[i * b:(i + 1) * b])
            z = beta ** j * r[t] + alpha * a
            yv = acc(yI[t])
            if loss == "linear":
                d[t] = yv - z
            elif loss == "poisson":
                d[t] = yv - np.exp(z)
            else:
                d[t] = yv / (acc(1) + np.exp(yv * z))
    c = (np.repeat(beta ** (s - 1 - np.arange(s)), b).astype(acc) * d).astype(np.float32)
    return (np.float32(beta ** s) * x.astype(np.float32) + np.float32(alpha) * (Y32.T @ c)).astype(
        np.float64)


@pytest.mark.parametrize("loss,eta", [("logistic", 0.5), ("linear", 0.2), ("poisson", 0.1)])
@pytest.mark.parametrize("acc", [np.float32, np.float64])
def test_fp32_simulation_within_bound_and_mistake_outside(loss, eta, acc):
    p = dense_glm(2000, 64, 3, loss, var=1 / 64)
    b, s, lam = 8, 6, 1e-3
    idx = R.sample_indices(7, 0, s * b, 2000)
    Y, yI = p.X[idx].astype(np.float32).astype(np.float64), p.y[idx]
    x = np.random.default_rng(1).standard_normal(64) * 0.3
    x = x.astype(np.float32).astype(np.float64)
    u = U32 if acc is np.float32 else 2.0 ** -53
    bound, ex = outer_bound(Y, x, yI, b, s, eta, lam, loss, u_acc=u)
    sim = _fp32_outer(Y, yI, x, eta, lam, b, s, loss, acc=acc)
    assert np.all(np.abs(sim - ex["x"]) <= bound)
    bad = _fp32_outer(Y, yI, x, eta, lam, b, s, loss, drop_far=True, acc=acc)
    assert np.any(np.abs(bad - ex["x"]) > bound)
