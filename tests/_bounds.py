"""First-order rounding-error bounds for the GPU parity tests.

Sec. 3.2: an inner product of length q accumulated with unit roundoff u is
within gamma_q(u) |a|^T |b| of the exact one, gamma_q(u) = q u / (1 - q u),
whatever the summation order. The bounds below propagate such input and
arithmetic errors through one outer iteration of Algorithm 1 (margins, Gram,
the s residual corrections, the update) to an entrywise bound on every
output, so that the GPU result of each piece is compared element by element
with the FP64 oracle at the precision the kernel actually computes in. A
factor `safety` covers the neglected second-order terms.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import reference as R

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def gamma(q: int, u: float) -> float:
    return q * u / (1.0 - q * u)


def _delta_lipschitz_and_eval(z, ez, yI, loss, u):
    """|d delta / dz| over [z - ez, z + ez] and the rounding error of one
    evaluation of the residual formula in unit roundoff u (Sec. 3.1)."""
    if loss == "linear":
        return np.ones_like(z), u * (np.abs(yI) + 2 * np.abs(z))
    if loss == "poisson":
        ez_hi = np.exp(np.minimum(z + ez, 700.0))
        return ez_hi, u * (np.abs(yI) + (4.0 + np.abs(z)) * ez_hi)
    d = yI / (1.0 + np.exp(np.minimum(yI * z, 700.0)))
    return np.full_like(z, 0.25), u * (6.0 + np.abs(z)) * np.abs(d)


def recurrence_bound(G, r, yI, delta, b, s, eta, lam, loss, e_r, e_G, u_acc, u_round=0.0):
    """Bounds on |delta~ - delta| and |c~ - c| for corrections computed in
    unit roundoff u_acc from inputs within e_r (margins) and e_G (Gram,
    entrywise) of the exact r and G, against the exact corrections delta of
    G, r, yI. Outputs are rounded to FP32 (included); u_round > 0 adds a
    rounding (possibly flipped: 2 u_round relative) of the correction sum, of
    z, of delta and of c to a format of that unit roundoff."""
    sb = s * b
    alpha, beta = eta / b, 1.0 - eta * lam
    A = np.abs(G)
    D = np.abs(delta)
    ed = np.zeros(sb)
    for j in range(s):
        rows = slice(j * b, (j + 1) * b)
        zj = beta ** j * r[rows]
        mag = beta ** j * np.abs(r[rows])
        ez = beta ** j * e_r[rows]
        if j > 0:
            cols = slice(0, j * b)
            w = np.repeat(beta ** (j - 1 - np.arange(j, dtype=np.float64)), b)
            zj = zj + alpha * (G[rows, cols] @ (w * delta[cols]))
            mag = mag + alpha * ((A[rows, cols] + e_G[rows, cols]) @ (w * (D[cols] + ed[cols])))
            ez = ez + alpha * (e_G[rows, cols] @ (w * (D[cols] + ed[cols]))
                               + A[rows, cols] @ (w * ed[cols]))
        ez = ez + gamma(j * b + 4, u_acc) * mag + 2 * u_round * (np.abs(zj) + 2 * mag)
        lip, ev = _delta_lipschitz_and_eval(zj, ez, yI[rows], loss, max(u_acc, u_round))
        ed[rows] = lip * ez + ev + 2 * u_round * (D[rows] + lip * ez)
    pw = np.repeat(beta ** (s - 1 - np.arange(s, dtype=np.float64)), b)
    c = pw * delta
    ec = pw * ed + (U32 + (s + 2) * u_acc + 2 * u_round) * (np.abs(c) + pw * ed)
    ed_out = ed + U32 * (D + ed)
    return ed_out, ec


def outer_bound(Y, x, yI, b, s, eta, lam, loss="logistic", u_acc=U64, scaled=False,
                safety=1.5, u_round=0.0):
    """Entrywise bound on |x_new~ - x_new| for one outer iteration from x,
    computed on the GPU from the exact stored rows Y (sb x n): margins and
    Gram accumulated in FP32 (row scales applied in FP32 when `scaled`),
    corrections in unit roundoff u_acc, update accumulated in FP32. Returns
    (bound, oracle pieces of R.outer_rows). u_round > 0 adds one rounding to
    a format of that unit roundoff at every slot's output (in both of two
    computations being compared: a rounding may flip by one unit in the last
    place, 2 u_round relative)."""
    sb, n = Y.shape
    ex = R.outer_rows(Y, yI, x, eta, lam, b, s, loss=loss)
    aY = np.abs(Y)
    k = 2 if scaled else 1
    e_r = 2 * gamma(n + 2 * k, U32) * (aY @ np.abs(x)) + 2 * u_round * np.abs(ex["r"])
    e_G = 2 * gamma(n + 2 * k, U32) * (aY @ aY.T) + 2 * u_round * np.abs(ex["G"])
    _, ec = recurrence_bound(ex["G"], ex["r"], np.asarray(yI, np.float64), ex["delta"], b, s,
                             eta, lam, loss, e_r, e_G, u_acc, u_round)
    alpha, beta = eta / b, 1.0 - eta * lam
    c = np.abs(ex["c"])
    g = aY.T @ (c + ec)
    bound = alpha * (aY.T @ ec) + alpha * 2 * gamma(sb + 2 + k, U32) * g \
        + 4 * U32 * np.abs(ex["x"]) + 2 * U32 * beta ** s * np.abs(x) + 1e-30 \
        + 2 * u_round * (alpha * g + np.abs(ex["x"]) + alpha * (aY.T @ ec))
    return safety * bound, ex


def assert_within(got, want, bound, what=""):
    err = np.abs(np.asarray(got, np.float64) - want)
    bad = np.nonzero(~(err <= bound))[0]
    if bad.size:
        i = bad[np.argmax(err[bad] / np.maximum(bound[bad], 1e-300))]
        raise AssertionError(f"{what}: {bad.size} entries outside the bound; worst index {i}: "
                             f"got {got[i]!r}, want {want[i]!r}, err {err[i]:.3e}, "
                             f"bound {bound[i]:.3e}")
    return float(np.max(err / bound)) if err.size else 0.0


def rec_prec_u(recur_prec: int, sb: int) -> float:
    """Unit roundoff of the corrections for a recur_prec setting (0 = automatic:
    FP64 from s*b = 512 on)."""
    if recur_prec == 64 or (recur_prec == 0 and sb >= 512):
        return U64
    return U32


__all__ = ["U32", "U64", "gamma", "recurrence_bound", "outer_bound", "assert_within",
           "rec_prec_u", "math"]
