"""Learned diagonal preconditioner for s-step SGD (not part of the paper).

A 4 -> 64 -> 2 MLP maps per-column statistics (mean, variance, fraction of
nonzeros, max |value|) to log d_k, a per-feature step scale, and (averaged over
a problem's columns) the log step size. The preconditioned method runs the
unchanged s-step kernels on X~ = X diag(sqrt(d)) and maps back x = sqrt(d) * x~;
that is SGD with the diagonal step matrix D on the data term and a decoupled
scalar L2 decay, and it keeps the s-step reformulation exact.

Training targets come from runs of the plain method:
  * log d_k = -log H_kk (centred per problem), H_kk the diagonal of the
    Hessian of the regularised logistic loss at the plain method's solution
    (a Jacobi preconditioner);
  * log (eta r2) = log of the best step size of a short sweep on the rescaled
    problem times its mean squared row norm r2: a dimensionless step, so the
    prediction does not have to learn the problem's scale (the absolute step
    is the prediction divided by r2 of the rescaled problem).

Everything numeric runs in libcasgd's kernels (column statistics, Hessian
diagonal, MLP forward/backward/Adam, quantisation, fits, losses); this module
only moves tensors and keeps the bookkeeping.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

import paper_2606_18463_amd as cg

# Step-size grid relative to the mean squared row norm r2 of the (rescaled)
# problem: eta = 2^k / r2 (column scales spread row norms over orders of
# magnitude, so an absolute grid misses the useful range).
ETA_K = range(-4, 13)


def mean_row_norm2(X) -> float:
    """mean_i ||a_i||^2 = sum_k (variance_k + mean_k^2) from the column
    statistics kernel (no host pass over X)."""
    st = cg.casgd_colstats(X).double()
    return float((st[:, 1] + st[:, 0] ** 2).sum())


def eta_grid(X):
    r2 = mean_row_norm2(X)
    return [2.0 ** k / r2 for k in ETA_K]


@dataclass
class Model:
    params: "object"      # device FP32 (450,)
    norm: "object"        # device FP32 (8,): feature means then standard deviations


@dataclass
class DeviceProblem:
    X32: "object"          # device FP32 m x n (kept to re-quantise after rescaling)
    y: "object"
    Xt32: "object"         # held-out rows, device FP32 (unpadded)
    Xt: "object"           # the same as a padded FP32 MatrixRef
    yt: "object"
    n: int
    m: int
    dtype: int


def upload(p, dtype=cg.BF16) -> DeviceProblem:
    import torch
    X32 = torch.from_numpy(np.ascontiguousarray(p.X, dtype=np.float32)).cuda()
    Xt32 = torch.from_numpy(np.ascontiguousarray(p.X_test, dtype=np.float32)).cuda()
    vals, _ = cg.casgd_quantize(Xt32, cg.F32)
    return DeviceProblem(X32, torch.from_numpy(p.y).cuda(), Xt32, cg.dense_matrix(vals, None, n=p.n),
                         torch.from_numpy(p.y_test).cuda(), p.n, p.m, dtype)


def stored(dp: DeviceProblem, q=None):
    """X, or X diag(q), in the problem's storage dtype."""
    if q is None:
        vals, sc = cg.casgd_quantize(dp.X32, dp.dtype)
    else:
        vals, sc = cg.casgd_quantize_scaled(dp.X32, q, dp.dtype)
    return cg.dense_matrix(vals, sc, n=dp.n)


def stored_test(dp: DeviceProblem, q=None):
    """The held-out rows, scaled like the training rows (FP32)."""
    if q is None:
        return dp.Xt
    vals, _ = cg.casgd_quantize_scaled(dp.Xt32, q, cg.F32)
    return cg.dense_matrix(vals, None, n=dp.n)


def unscale(x_tilde, q):
    """x = q * x~ (a 1 x n FP32 quantisation with column scale q)."""
    vals, _ = cg.casgd_quantize_scaled(x_tilde.view(1, -1), q, cg.F32)
    return vals.view(-1)[: x_tilde.numel()]


def fit(X, y, n, eta, lam, b, s, seed, n_outer, snapshot_every=0):
    """s-step fit from zero; returns (x, snapshot history or None)."""
    import torch
    x = torch.zeros(n, device="cuda")
    hist = None
    o = None
    if snapshot_every:
        k = n_outer // snapshot_every
        hist = torch.zeros(k, n, device="cuda")
        o = cg.opts(snapshot_every=snapshot_every, x_history=hist)
    ws = cg.casgd_fit(X, y, x, eta, lam, b, s, seed, 0, n_outer, opts=o)
    cg.casgd_check(ws)
    return x, hist


def best_eta(X, y, Xt, yt, n, lam, b, s, seed, n_outer, grid=None):
    """Step size of `grid` (default eta_grid(X)) with the lowest held-out loss
    after n_outer iterations."""
    grid = eta_grid(X) if grid is None else grid
    best = None
    for eta in grid:
        x, _ = fit(X, y, n, eta, lam, b, s, seed, n_outer)
        loss = float(cg.casgd_logloss(Xt, yt, x))
        if math.isfinite(loss) and (best is None or loss < best[0]):
            best = (loss, eta)
    return best[1]


def best_eta_plateau(X, y, Xt, yt, n, lam, b, s, seed, n_outer, grid, snaps: int = 16):
    """Step size of `grid` with the lowest mean held-out loss over the second
    half of an n_outer run (snapshots every n_outer / snaps outer iterations):
    constant-step SGD ends on a plateau whose height grows with the step, and
    a short run alone would favour steps that settle too high."""
    every = max(1, n_outer // snaps)
    best = None
    for eta in grid:
        try:
            losses = loss_curve(X, y, Xt, yt, n, eta, lam, b, s, seed, every * snaps, every)
        except cg.CasgdError:       # diverged (non-finite iterate)
            continue
        tail = np.asarray(losses[len(losses) // 2:], dtype=np.float64)
        if tail.size and np.all(np.isfinite(tail)):
            score = float(tail.mean())
            if best is None or score < best[0]:
                best = (score, eta)
    return best[1]


def targets(dp: DeviceProblem, lam: float, b: int, s: int, seed: int, epochs: float = 2.0):
    """(t_d per column, log (eta r2) for the rescaled problem, plain best eta).
    The plain step is the best of a short sweep (it only has to give a usable
    solution for the Hessian); the rescaled problem's step is the best for the
    plateau of an `epochs` run."""
    X = stored(dp)
    n_outer = max(2, int(epochs * dp.m / (b * s)))
    short = max(2, n_outer // 4)
    eta0 = best_eta(X, dp.y, dp.Xt, dp.yt, dp.n, lam, b, s, seed, short)
    x, _ = fit(X, dp.y, dp.n, eta0, lam, b, s, seed, n_outer)
    h = cg.casgd_hess_diag(X, x, lam)
    t_d, q = cg.casgd_jacobi_target(h)
    Xq = stored(dp, q)
    r2 = mean_row_norm2(Xq)
    eta1 = best_eta_plateau(Xq, dp.y, stored_test(dp, q), dp.yt, dp.n, lam, b, s, seed, n_outer,
                            grid=[2.0 ** k / r2 for k in ETA_K])
    return t_d, math.log(eta1 * r2), eta0


def init_params(seed: int = 0):
    """He-initialised first layer, zero biases (host RNG, uploaded once)."""
    import torch
    g = np.random.default_rng(seed)
    W1 = g.standard_normal((64, 4)) * math.sqrt(2.0 / 4)
    b1 = np.zeros(64)
    W2 = g.standard_normal((2, 64)) * math.sqrt(1.0 / 64)
    b2 = np.zeros(2)
    flat = np.concatenate([W1.ravel(), b1, W2.ravel(), b2]).astype(np.float32)
    return torch.from_numpy(flat).cuda()


def train(stats_list, t_d_list, t_eta_list, steps: int = 2000, lr: float = 3e-3,
          w_eta: float = 1.0, seed: int = 0, log_every: int = 0):
    """Full-batch Adam over the columns of all training problems.
    Returns (Model, [(step, loss)])."""
    import torch
    stats = torch.cat(stats_list, dim=0).contiguous()
    norm = cg.casgd_mlp_feature_norm(stats)
    feats = cg.casgd_mlp_features(stats, norm)
    t_d = torch.cat(t_d_list).float().contiguous()
    t_eta = torch.tensor(t_eta_list, dtype=torch.float32, device="cuda")
    counts = [st.shape[0] for st in stats_list]
    seg_off = torch.tensor(np.concatenate([[0], np.cumsum(counts)]), dtype=torch.int64,
                           device="cuda")
    P = len(stats_list)
    params = init_params(seed)
    m1 = torch.zeros_like(params)
    m2 = torch.zeros_like(params)
    hist = []
    ws = cg._mlp_ws(feats.shape[0], P)
    for t in range(1, steps + 1):
        out, pre = cg.casgd_mlp_forward(params, feats)
        loss, g = cg.casgd_mlp_loss_grad(out, seg_off, t_d, t_eta, w_eta, ws=ws)
        grad = cg.casgd_mlp_backward(params, feats, pre, g, P, ws=ws)
        cg.casgd_adam_step(params, grad, m1, m2, t, lr)
        if log_every and (t % log_every == 0 or t == 1 or t == steps):
            hist.append((t, float(loss)))
    return Model(params, norm), hist


def predict(model: Model, X):
    """(column scale q = sqrt(d), dimensionless step eta r2) for a problem from
    its column statistics."""
    st = cg.casgd_colstats(X)
    feats = cg.casgd_mlp_features(st, model.norm)
    out, _ = cg.casgd_mlp_forward(model.params, feats, want_pre=False)
    q, eta = cg.casgd_mlp_apply(out)
    return q, float(eta)


def apply(model: Model, dp: DeviceProblem):
    """The preconditioned problem: (X~ = X diag(q) in the storage dtype, the
    held-out rows scaled alike, q, absolute step size)."""
    q, eta_rel = predict(model, stored(dp))
    Xq = stored(dp, q)
    return Xq, stored_test(dp, q), q, eta_rel / mean_row_norm2(Xq)


def loss_curve(X, y, Xt, yt, n, eta, lam, b, s, seed, n_outer, every):
    """Held-out loss every `every` outer iterations (snapshots in the fit)."""
    _, hist = fit(X, y, n, eta, lam, b, s, seed, n_outer, snapshot_every=every)
    return cg.casgd_logloss(Xt, yt, hist).cpu().numpy()


def first_hit(losses, target, every):
    """Outer iterations until a loss curve first reaches `target`, or None."""
    hit = np.nonzero(np.asarray(losses) <= target)[0]
    return None if hit.size == 0 else int(hit[0] + 1) * every
