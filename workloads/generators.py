"""Seeded synthetic workload generators.

Every generator is deterministic in its seed: the random streams come from
``numpy.random.SeedSequence(seed).spawn(...)`` and large matrices are filled in
fixed-size row chunks, each from its own child stream, so the result does not
depend on how many threads fill them.

Workloads (the paper's datasets are not available; these stand in for them):

* ``dense_c1``  -- 4096 x 256 FP64, entries N(0, 1/256), planted w ~ N(0, I),
  labels sign(Xw + eps) with eps ~ N(0, 0.1) (0.1 read as a variance),
  1024 held-out rows.
* ``dense_c2``  -- 2^20 x 2048 FP32, entries N(0, 1/2048) with 205 seeded
  columns scaled x10 (uneven column norms), labels sign(Xw) then 5% random
  flips, 2^18 held-out rows.
* ``sparse_c4`` -- CSR 10^6 x 2^17, about 50 nonzeros per row whose columns
  follow a Zipf(1.1) law over a seeded rank->column permutation, log-normal
  values, rows l2-normalised, planted-w labels with N(0, 0.1) noise.
* ``uneven_problem_specs`` / ``uneven_problem`` -- the many-problem batch:
  m log-uniform in [1e4, 2e5], n log-uniform in [128, 4096], column-scale
  spread S log-uniform in [1, 1e3], column scales log-uniform in [1, S],
  entries N(0, 1/n) * scale.

* ``dense_glm`` / ``sparse_zipf_glm`` -- the same feature matrices with
  labels for the linear and Poisson losses: linear y = Xw + eps with
  eps ~ N(0, noise_var); Poisson y ~ Poisson(exp(rate_scale * Xw)), counts
  (the paper's Poisson-synth generator is not specified; rate_scale = 0.5
  keeps the rates near exp(+-1) for unit-variance margins).

``sign(0)`` is +1 throughout. Logistic labels are stored as float32 +-1,
linear and Poisson labels as float32 values.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

_CHUNK_ROWS = 16384


def _threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    n = int(env) if env and env.isdigit() else (os.cpu_count() or 1)
    return max(1, min(n, 16))


@dataclass
class DenseProblem:
    X: np.ndarray            # m x n, row-major
    y: np.ndarray            # m, float32 in {-1, +1}
    X_test: np.ndarray       # m_test x n
    y_test: np.ndarray       # m_test
    w_true: np.ndarray       # n, float64
    col_scale: np.ndarray    # n, float64 (1 where unscaled)
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.X.shape[0]

    @property
    def n(self) -> int:
        return self.X.shape[1]


@dataclass
class SparseProblem:
    row_ptr: np.ndarray      # m + 1, int64
    col_idx: np.ndarray      # nnz, int32 (sorted within each row)
    values: np.ndarray       # nnz, float32
    n: int
    y: np.ndarray            # m, float32
    test_row_ptr: np.ndarray
    test_col_idx: np.ndarray
    test_values: np.ndarray
    y_test: np.ndarray
    w_true: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.row_ptr.shape[0] - 1

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_dense(self, test: bool = False) -> np.ndarray:
        rp, ci, va = ((self.test_row_ptr, self.test_col_idx, self.test_values)
                      if test else (self.row_ptr, self.col_idx, self.values))
        m = rp.shape[0] - 1
        out = np.zeros((m, self.n), dtype=np.float32)
        rows = np.repeat(np.arange(m), np.diff(rp))
        out[rows, ci] = va
        return out


def _fill_normal(out: np.ndarray, seq: np.random.SeedSequence, std: float,
                 col_scale: np.ndarray | None) -> None:
    """Fill ``out`` (m x n) with N(0, std^2) * col_scale, chunk by chunk."""
    m = out.shape[0]
    nchunks = max(1, -(-m // _CHUNK_ROWS))
    kids = seq.spawn(nchunks)
    scale32 = None
    if col_scale is not None:
        scale32 = (col_scale * std).astype(out.dtype)

    def work(c: int) -> None:
        lo, hi = c * _CHUNK_ROWS, min(m, (c + 1) * _CHUNK_ROWS)
        g = np.random.Generator(np.random.PCG64(kids[c]))
        blk = out[lo:hi]
        if out.dtype == np.float32:
            g.standard_normal(out=blk, dtype=np.float32)
        else:
            blk[...] = g.standard_normal(blk.shape)
        if scale32 is not None:
            blk *= scale32
        else:
            blk *= out.dtype.type(std)

    if nchunks == 1:
        work(0)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, range(nchunks)))


def _margins(X: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Planted margins X w, in the storage precision of X, chunked."""
    wt = w.astype(X.dtype)
    m = X.shape[0]
    out = np.empty(m, dtype=np.float64)
    step = 1 << 16
    for lo in range(0, m, step):
        out[lo:lo + step] = X[lo:lo + step] @ wt
    return out


def _labels(margin: np.ndarray, noise_seq, noise_var: float,
            flip_seq, flip_frac: float) -> np.ndarray:
    v = margin.copy()
    if noise_var > 0:
        g = np.random.Generator(np.random.PCG64(noise_seq))
        v += g.standard_normal(v.shape[0]) * math.sqrt(noise_var)
    y = np.where(v >= 0, 1.0, -1.0).astype(np.float32)
    if flip_frac > 0:
        g = np.random.Generator(np.random.PCG64(flip_seq))
        flips = g.random(y.shape[0]) < flip_frac
        y[flips] = -y[flips]
    return y


def dense_logreg(m: int, n: int, seed: int, *, var: float, scaled_cols: int = 0,
                 col_factor: float = 1.0, col_scale: np.ndarray | None = None,
                 noise_var: float = 0.0, flip_frac: float = 0.0,
                 m_test: int | None = None, dtype=np.float64) -> DenseProblem:
    """Dense planted-w logistic-regression data (see module docstring)."""
    root = np.random.SeedSequence(seed)
    (s_w, s_cols, s_train, s_test, s_noise, s_noise_t, s_flip,
     s_flip_t) = root.spawn(8)
    w = np.random.Generator(np.random.PCG64(s_w)).standard_normal(n)
    if col_scale is None:
        col_scale = np.ones(n)
        if scaled_cols > 0:
            sel = np.random.Generator(np.random.PCG64(s_cols)).choice(
                n, size=scaled_cols, replace=False)
            col_scale[sel] = col_factor
    std = math.sqrt(var)
    m_test = m // 4 if m_test is None else m_test
    X = np.empty((m, n), dtype=dtype)
    _fill_normal(X, s_train, std, None if np.all(col_scale == 1) else col_scale)
    Xt = np.empty((m_test, n), dtype=dtype)
    _fill_normal(Xt, s_test, std, None if np.all(col_scale == 1) else col_scale)
    y = _labels(_margins(X, w), s_noise, noise_var, s_flip, flip_frac)
    yt = _labels(_margins(Xt, w), s_noise_t, noise_var, s_flip_t, flip_frac)
    meta = dict(m=m, n=n, seed=seed, var=var, scaled_cols=scaled_cols,
                col_factor=col_factor, noise_var=noise_var, flip_frac=flip_frac,
                dtype=np.dtype(dtype).name)
    return DenseProblem(X, y, Xt, yt, w, col_scale, meta)


def dense_c1(seed: int = 42) -> DenseProblem:
    """4096 x 256 FP64, N(0, 1/256), noise variance 0.1, 1024 test rows."""
    return dense_logreg(4096, 256, seed, var=1.0 / 256, noise_var=0.1,
                        m_test=1024, dtype=np.float64)


def dense_c2(seed: int = 42, m: int = 1 << 20, n: int = 2048,
             m_test: int | None = None) -> DenseProblem:
    """2^20 x 2048 FP32, N(0, 1/n), 10% of columns x10, 5% label flips.

    ``m``/``n`` may be reduced for tests; the column fraction, scale factor
    and flip fraction are kept.
    """
    k = int(round(0.1 * n))
    return dense_logreg(m, n, seed, var=1.0 / n, scaled_cols=k, col_factor=10.0,
                        flip_frac=0.05, m_test=(m // 4 if m_test is None else m_test),
                        dtype=np.float32)


def normalize_rows(X: np.ndarray) -> np.ndarray:
    """Scale every row to unit l2 norm (zero rows are left as they are)."""
    nrm = np.sqrt((X.astype(np.float64) ** 2).sum(axis=1))
    nrm[nrm == 0] = 1.0
    return (X / nrm[:, None]).astype(X.dtype)


# --------------------------------------------------------------------------
# Sparse CSR with Zipf-distributed columns
# --------------------------------------------------------------------------

def _zipf_cdf(n: int, a: float) -> np.ndarray:
    p = np.arange(1, n + 1, dtype=np.float64) ** (-a)
    c = np.cumsum(p)
    return c / c[-1]


def _sparse_rows(m: int, n: int, g: np.random.Generator, nnz_mean: float,
                 cdf: np.ndarray, perm: np.ndarray):
    """Row lengths ~ max(1, Poisson(nnz_mean)) of distinct Zipf-ranked columns.

    Each round draws exactly the missing count for every unfinished row;
    draws that repeat a column already in the row are discarded and drawn
    again next round (at most 64 rounds, after which a row keeps what it has).
    """
    target = np.maximum(1, g.poisson(nnz_mean, size=m)).astype(np.int64)
    need = target.copy()
    active = np.arange(m)
    held: list[np.ndarray] = []          # sorted key chunks, key = row*n + col
    for _ in range(64):
        if active.size == 0:
            break
        rows = np.repeat(active, need[active])
        ranks = np.minimum(np.searchsorted(cdf, g.random(rows.size), side="right"), n - 1)
        keys = rows * n + perm[ranks].astype(np.int64)
        _, first = np.unique(keys, return_index=True)
        first.sort()
        cand = keys[first]                # distinct, in draw order (rows ascending)
        fresh = np.ones(cand.size, dtype=bool)
        for h in held:
            if h.size == 0:
                continue
            pos = np.minimum(np.searchsorted(h, cand), h.size - 1)
            fresh &= h[pos] != cand
        cand = cand[fresh]
        held.append(np.sort(cand))
        need -= np.bincount(cand // n, minlength=m)
        active = np.nonzero(need > 0)[0]
    keys = np.sort(np.concatenate(held))
    rows = keys // n
    cols = (keys % n).astype(np.int32)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=row_ptr[1:])
    return row_ptr, cols


def sparse_zipf_logreg(m: int, n: int, seed: int, *, nnz_mean: float = 50.0,
                       zipf_a: float = 1.1, noise_var: float = 0.1,
                       m_test: int | None = None) -> SparseProblem:
    root = np.random.SeedSequence(seed)
    s_perm, s_w, s_train, s_test, s_noise, s_noise_t, s_val, s_val_t = root.spawn(8)
    perm = np.random.Generator(np.random.PCG64(s_perm)).permutation(n)
    w = np.random.Generator(np.random.PCG64(s_w)).standard_normal(n)
    cdf = _zipf_cdf(n, zipf_a)
    m_test = m // 4 if m_test is None else m_test

    def build(mm, s_rows, s_vals, s_nz):
        rp, ci = _sparse_rows(mm, n, np.random.Generator(np.random.PCG64(s_rows)),
                              nnz_mean, cdf, perm)
        vals = np.exp(np.random.Generator(np.random.PCG64(s_vals)).standard_normal(ci.size))
        rows = np.repeat(np.arange(mm), np.diff(rp))
        nrm = np.sqrt(np.bincount(rows, weights=vals * vals, minlength=mm))
        nrm[nrm == 0] = 1.0
        vals = (vals / nrm[rows]).astype(np.float32)
        margin = np.bincount(rows, weights=vals.astype(np.float64) * w[ci], minlength=mm)
        y = _labels(margin, s_nz, noise_var, None, 0.0)
        return rp, ci, vals, y

    rp, ci, va, y = build(m, s_train, s_val, s_noise)
    trp, tci, tva, yt = build(m_test, s_test, s_val_t, s_noise_t)
    meta = dict(m=m, n=n, seed=seed, nnz_mean=nnz_mean, zipf_a=zipf_a,
                noise_var=noise_var)
    return SparseProblem(rp, ci, va, n, y, trp, tci, tva, yt, w, meta)


def glm_labels(margin: np.ndarray, loss: str, seq, *, noise_var: float = 0.1,
               rate_scale: float = 0.5) -> np.ndarray:
    """Labels for planted margins (data generation only): logistic
    sign(margin + eps), linear margin + eps, Poisson draws with mean
    exp(rate_scale * margin); eps ~ N(0, noise_var)."""
    if loss == "logistic":
        return _labels(margin, seq, noise_var, None, 0.0)
    g = np.random.Generator(np.random.PCG64(seq))
    if loss == "linear":
        return (margin + g.standard_normal(margin.shape[0]) * math.sqrt(noise_var)).astype(
            np.float32)
    if loss == "poisson":
        return g.poisson(np.exp(rate_scale * margin)).astype(np.float32)
    raise ValueError(loss)


def dense_glm(m: int, n: int, seed: int, loss: str, *, var: float, noise_var: float = 0.1,
              rate_scale: float = 0.5, m_test: int | None = None,
              dtype=np.float64) -> DenseProblem:
    """Dense planted-w data with labels for `loss` (see glm_labels)."""
    p = dense_logreg(m, n, seed, var=var, m_test=m_test, dtype=dtype)
    s_y, s_yt = np.random.SeedSequence([seed, 11]).spawn(2)
    p.y = glm_labels(_margins(p.X, p.w_true), loss, s_y, noise_var=noise_var,
                     rate_scale=rate_scale)
    p.y_test = glm_labels(_margins(p.X_test, p.w_true), loss, s_yt, noise_var=noise_var,
                          rate_scale=rate_scale)
    p.meta.update(loss=loss, noise_var=noise_var, rate_scale=rate_scale)
    return p


def sparse_zipf_glm(m: int, n: int, seed: int, loss: str, *, nnz_mean: float = 50.0,
                    noise_var: float = 0.1, rate_scale: float = 0.5) -> SparseProblem:
    """The Zipf CSR matrix of sparse_zipf_logreg with labels for `loss`."""
    p = sparse_zipf_logreg(m, n, seed, nnz_mean=nnz_mean, noise_var=noise_var)
    s_y, s_yt = np.random.SeedSequence([seed, 13]).spawn(2)

    def margin(rp, ci, va):
        mm = rp.shape[0] - 1
        rows = np.repeat(np.arange(mm), np.diff(rp))
        return np.bincount(rows, weights=va.astype(np.float64) * p.w_true[ci], minlength=mm)

    p.y = glm_labels(margin(p.row_ptr, p.col_idx, p.values), loss, s_y,
                     noise_var=noise_var, rate_scale=rate_scale)
    p.y_test = glm_labels(margin(p.test_row_ptr, p.test_col_idx, p.test_values), loss, s_yt,
                          noise_var=noise_var, rate_scale=rate_scale)
    p.meta.update(loss=loss, rate_scale=rate_scale)
    return p


def sparse_c4(seed: int = 42, m: int = 1_000_000, n: int = 1 << 17) -> SparseProblem:
    return sparse_zipf_logreg(m, n, seed)


def lambda_path_c4(L: int = 32, lo: float = 1e-7, hi: float = 1e-2) -> np.ndarray:
    """L regularisation strengths log-spaced from ``lo`` to ``hi``."""
    return np.logspace(math.log10(lo), math.log10(hi), L)


# --------------------------------------------------------------------------
# Many uneven problems
# --------------------------------------------------------------------------

def uneven_problem_specs(count: int, seed: int, *, m_range=(1e4, 2e5),
                         n_range=(128, 4096), spread_range=(1.0, 1e3)) -> list[dict]:
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))

    def logu(lo, hi, size):
        return np.exp(g.uniform(math.log(lo), math.log(hi), size))

    ms = np.round(logu(*m_range, count)).astype(np.int64)
    ns = np.round(logu(*n_range, count)).astype(np.int64)
    ss = logu(*spread_range, count)
    seeds = g.integers(0, 2**31 - 1, size=count)
    return [dict(m=int(ms[i]), n=int(ns[i]), spread=float(ss[i]), seed=int(seeds[i]))
            for i in range(count)]


def uneven_problem(spec: dict, dtype=np.float32) -> DenseProblem:
    n = spec["n"]
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([spec["seed"], 7])))
    S = spec["spread"]
    col_scale = np.exp(g.uniform(0.0, math.log(S), n)) if S > 1 else np.ones(n)
    p = dense_logreg(spec["m"], n, spec["seed"], var=1.0 / n, col_scale=col_scale,
                     noise_var=0.1, dtype=dtype)
    p.meta.update(spread=S)
    return p
