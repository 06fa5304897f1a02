"""FP64 CPU oracle for s-step mini-batch SGD on L2-regularised generalized linear
models: logistic regression (the default), linear regression and Poisson
regression (the three losses of Sec. 2.1, residuals of Sec. 3.1).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module. It shares no code with the GPU
path (the library, its kernels and its Python binding) and imports nothing
from it.

Two layers:

* the C core (``casgd_oracle.c`` -> ``liboracle.so``): plain mini-batch SGD,
  the s-step outer iteration, its pieces, a CSR variant and the losses, for
  each of the three losses, all in IEEE double with left-to-right sums;
* NumPy FP64 code here: a second, independent pure-Python SGD for tiny
  cases, the storage formats (BF16, FP16, OCP FP8-e4m3 with per-row scales)
  written from their definitions, the local error bound of the paper's
  mixed-precision theorem (Thm. 5.1) and its uniform-precision corollary,
  column statistics, and the 2-layer MLP used for the learned
  preconditioner (forward, backward, Adam).

Paper references are to "Mixed-Precision Communication-Avoiding SGD for
Generalized Linear Models on GPUs" (Sec. 3 notation, Algorithm 1, Sec. 5).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import build as _build

_lib = None

_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double
_pd = ctypes.POINTER(ctypes.c_double)
_pf = ctypes.POINTER(ctypes.c_float)
_pi64 = ctypes.POINTER(ctypes.c_int64)
_pi32 = ctypes.POINTER(ctypes.c_int32)


def lib():
    """Load ``liboracle.so``, compiling it first if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.oracle_splitmix64.restype = _u64
        L.oracle_splitmix64.argtypes = [_u64, _u64]
        L.oracle_sample_index.restype = _i64
        L.oracle_sample_index.argtypes = [_u64, _u64, _i64]
        L.oracle_sample_indices.restype = None
        L.oracle_sample_indices.argtypes = [_u64, _u64, _i64, _i64, _pi64]
        L.oracle_delta.restype = _dbl
        L.oracle_delta.argtypes = [_dbl, _dbl]
        L.oracle_logloss.restype = _dbl
        L.oracle_logloss.argtypes = [_pd, _i64, _i64, _i64, _pd, _pd]
        L.oracle_logloss_f32.restype = _dbl
        L.oracle_logloss_f32.argtypes = [_pf, _i64, _i64, _i64, _pf, _pd]
        L.oracle_logloss_csr.restype = _dbl
        L.oracle_logloss_csr.argtypes = [_pi64, _pi32, _pd, _i64, _pd, _pd]
        L.oracle_sgd.restype = ctypes.c_int
        L.oracle_sgd.argtypes = [_pd, _i64, _i64, _i64, _pd, _pd, _dbl, _dbl, _i32,
                                 _u64, _u64, _i64]
        L.oracle_sgd_f32.restype = ctypes.c_int
        L.oracle_sgd_f32.argtypes = [_pf, _i64, _i64, _i64, _pf, _pd, _dbl, _dbl, _i32,
                                     _u64, _u64, _i64]
        L.oracle_casgd.restype = ctypes.c_int
        L.oracle_casgd.argtypes = [_pd, _i64, _i64, _i64, _pd, _pd, _dbl, _dbl, _i32,
                                   _i32, _u64, _u64, _i64]
        L.oracle_casgd_f32.restype = ctypes.c_int
        L.oracle_casgd_f32.argtypes = [_pf, _i64, _i64, _i64, _pf, _pd, _dbl, _dbl,
                                       _i32, _i32, _u64, _u64, _i64]
        L.oracle_outer_parts.restype = ctypes.c_int
        L.oracle_outer_parts.argtypes = [_pd, _i64, _i64, _i64, _pd, _pd, _dbl, _dbl,
                                         _i32, _i32, _u64, _u64, _pi64, _pd, _pd, _pd,
                                         _pd, _pd]
        L.oracle_inner_corrections.restype = ctypes.c_int
        L.oracle_inner_corrections.argtypes = [_pd, _pd, _pd, _i32, _i32, _dbl, _dbl,
                                               _pd, _pd]
        L.oracle_casgd_csr.restype = ctypes.c_int
        L.oracle_casgd_csr.argtypes = [_pi64, _pi32, _pd, _i64, _i64, _pd, _pd, _dbl,
                                       _dbl, _i32, _i32, _u64, _u64, _i64]
        L.oracle_delta_glm.restype = _dbl
        L.oracle_delta_glm.argtypes = [_dbl, _dbl, _i32]
        L.oracle_loss_glm.restype = _dbl
        L.oracle_loss_glm.argtypes = [_pd, _i64, _i64, _i64, _pd, _pd, _i32]
        L.oracle_loss_glm_f32.restype = _dbl
        L.oracle_loss_glm_f32.argtypes = [_pf, _i64, _i64, _i64, _pf, _pd, _i32]
        L.oracle_loss_glm_csr.restype = _dbl
        L.oracle_loss_glm_csr.argtypes = [_pi64, _pi32, _pd, _i64, _pd, _pd, _i32]
        L.oracle_sgd_glm.restype = ctypes.c_int
        L.oracle_sgd_glm.argtypes = [_pd, _i64, _i64, _i64, _pd, _pd, _dbl, _dbl, _i32,
                                     _u64, _u64, _i64, _i32]
        L.oracle_sgd_glm_f32.restype = ctypes.c_int
        L.oracle_sgd_glm_f32.argtypes = [_pf, _i64, _i64, _i64, _pf, _pd, _dbl, _dbl, _i32,
                                         _u64, _u64, _i64, _i32]
        L.oracle_casgd_glm.restype = ctypes.c_int
        L.oracle_casgd_glm.argtypes = [_pd, _i64, _i64, _i64, _pd, _pd, _dbl, _dbl, _i32,
                                       _i32, _u64, _u64, _i64, _i32]
        L.oracle_casgd_glm_f32.restype = ctypes.c_int
        L.oracle_casgd_glm_f32.argtypes = [_pf, _i64, _i64, _i64, _pf, _pd, _dbl, _dbl,
                                           _i32, _i32, _u64, _u64, _i64, _i32]
        L.oracle_outer_parts_glm.restype = ctypes.c_int
        L.oracle_outer_parts_glm.argtypes = [_pd, _i64, _i64, _i64, _pd, _pd, _dbl, _dbl,
                                             _i32, _i32, _u64, _u64, _pi64, _pd, _pd, _pd,
                                             _pd, _pd, _i32]
        L.oracle_outer_rows_glm.restype = ctypes.c_int
        L.oracle_outer_rows_glm.argtypes = [_pd, _i64, _pd, _pd, _dbl, _dbl, _i32, _i32, _pd,
                                            _pd, _pd, _pd, _pd, _i32]
        L.oracle_inner_corrections_glm.restype = ctypes.c_int
        L.oracle_inner_corrections_glm.argtypes = [_pd, _pd, _pd, _i32, _i32, _dbl, _dbl,
                                                   _pd, _pd, _i32]
        L.oracle_casgd_csr_glm.restype = ctypes.c_int
        L.oracle_casgd_csr_glm.argtypes = [_pi64, _pi32, _pd, _i64, _i64, _pd, _pd, _dbl,
                                           _dbl, _i32, _i32, _u64, _u64, _i64, _i32]
        L.oracle_set_threads.restype = None
        L.oracle_set_threads.argtypes = [_i32]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        _lib = L
    return _lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc: int) -> None:
    if rc != 0:
        raise RuntimeError(f"oracle call failed with code {rc}")


# Loss selector of the C core (Sec. 2.1): logistic, linear (least squares),
# Poisson.
LOSSES = {"logistic": 0, "linear": 1, "poisson": 2}


def _loss_code(loss) -> int:
    return LOSSES[loss] if isinstance(loss, str) else int(loss)


# ------------------------------------------------------------------ sampling

def splitmix64(seed: int, t: int) -> int:
    return int(lib().oracle_splitmix64(seed & (2**64 - 1), t))


def sample_indices(seed: int, t0: int, count: int, m: int) -> np.ndarray:
    """Indices of samples t0 .. t0+count-1 (Algorithm 1, sampling step)."""
    out = np.empty(count, dtype=np.int64)
    lib().oracle_sample_indices(seed & (2**64 - 1), t0, count, m, _p(out, _pi64))
    return out


def threads() -> int:
    return int(lib().oracle_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on."""
    lib().oracle_set_threads(int(n))


# ------------------------------------------------------------------ solvers

def _rows(X: np.ndarray):
    """(pointer, is_f32, ld) for a row-major FP32 or FP64 matrix."""
    if X.dtype == np.float32:
        X = np.ascontiguousarray(X)
        return X, True
    return _f64(X), False


def sgd(X, y, x0, eta: float, lam: float, b: int, seed: int, step0: int = 0,
        nsteps: int = 1, loss="logistic") -> np.ndarray:
    """Plain mini-batch SGD in delta form with L2 decay (Sec. 3.1)."""
    Xr, f32 = _rows(X)
    x = _f64(x0).copy()
    m, n = Xr.shape
    lc = _loss_code(loss)
    if f32:
        yv = np.ascontiguousarray(y, dtype=np.float32)
        _check(lib().oracle_sgd_glm_f32(_p(Xr, _pf), n, m, n, _p(yv, _pf), _p(x, _pd),
                                        eta, lam, b, seed, step0, nsteps, lc))
    else:
        yv = _f64(y)
        _check(lib().oracle_sgd_glm(_p(Xr, _pd), n, m, n, _p(yv, _pd), _p(x, _pd),
                                    eta, lam, b, seed, step0, nsteps, lc))
    return x


def casgd(X, y, x0, eta: float, lam: float, b: int, s: int, seed: int,
          outer0: int = 0, nouter: int = 1, loss="logistic") -> np.ndarray:
    """s-step SGD (Algorithm 1 with L2 decay), ``nouter`` outer iterations."""
    Xr, f32 = _rows(X)
    x = _f64(x0).copy()
    m, n = Xr.shape
    lc = _loss_code(loss)
    if f32:
        yv = np.ascontiguousarray(y, dtype=np.float32)
        _check(lib().oracle_casgd_glm_f32(_p(Xr, _pf), n, m, n, _p(yv, _pf), _p(x, _pd),
                                          eta, lam, b, s, seed, outer0, nouter, lc))
    else:
        yv = _f64(y)
        _check(lib().oracle_casgd_glm(_p(Xr, _pd), n, m, n, _p(yv, _pd), _p(x, _pd),
                                      eta, lam, b, s, seed, outer0, nouter, lc))
    return x


def outer_parts(X, y, x, eta: float, lam: float, b: int, s: int, seed: int,
                outer: int, loss="logistic") -> dict:
    """idx, yI, r, strict block-lower G, delta and c of one outer iteration."""
    Xr = _f64(X)
    yv = _f64(y)
    xv = _f64(x)
    m, n = Xr.shape
    sb = s * b
    idx = np.empty(sb, dtype=np.int64)
    yI = np.empty(sb)
    r = np.empty(sb)
    G = np.empty((sb, sb))
    d = np.empty(sb)
    c = np.empty(sb)
    _check(lib().oracle_outer_parts_glm(_p(Xr, _pd), n, m, n, _p(yv, _pd), _p(xv, _pd),
                                        eta, lam, b, s, seed, outer, _p(idx, _pi64),
                                        _p(yI, _pd), _p(r, _pd), _p(G, _pd), _p(d, _pd),
                                        _p(c, _pd), _loss_code(loss)))
    return dict(idx=idx, yI=yI, r=r, G=G, delta=d, c=c)


def outer_rows(Y, yI, x, eta: float, lam: float, b: int, s: int, loss="logistic") -> dict:
    """One outer iteration of Algorithm 1 (with decay) on the given sampled rows
    Y (s*b x n) and labels yI: r, strict block-lower G, delta, c and the new x."""
    Yr = _f64(Y)
    sb, n = Yr.shape
    assert sb == s * b
    yv, xv = _f64(yI), _f64(x)
    r, d, c = np.empty(sb), np.empty(sb), np.empty(sb)
    G = np.empty((sb, sb))
    xn = np.empty(n)
    _check(lib().oracle_outer_rows_glm(_p(Yr, _pd), n, _p(yv, _pd), _p(xv, _pd), eta, lam, b, s,
                                       _p(r, _pd), _p(G, _pd), _p(d, _pd), _p(c, _pd),
                                       _p(xn, _pd), _loss_code(loss)))
    return dict(r=r, G=G, delta=d, c=c, x=xn)


def inner_corrections(G, r, yI, b: int, s: int, eta: float, lam: float, loss="logistic"):
    """The s residual corrections of Algorithm 1 (with decay): (delta, c)."""
    Gv, rv, yv = _f64(G), _f64(r), _f64(yI)
    d = np.empty(s * b)
    c = np.empty(s * b)
    _check(lib().oracle_inner_corrections_glm(_p(Gv, _pd), _p(rv, _pd), _p(yv, _pd), b, s,
                                              eta, lam, _p(d, _pd), _p(c, _pd),
                                              _loss_code(loss)))
    return d, c


def delta(z: float, y: float, loss="logistic") -> float:
    """Residual -dL/dz of Sec. 3.1 for one sample."""
    return float(lib().oracle_delta_glm(z, y, _loss_code(loss)))


def loss_value(X, y, x, loss="logistic") -> float:
    """Mean loss m^-1 sum L(a_i^T x, y_i) of Sec. 2.1 (unregularised)."""
    xv = _f64(x)
    lc = _loss_code(loss)
    if X.dtype == np.float32:
        Xr = np.ascontiguousarray(X)
        yv = np.ascontiguousarray(y, dtype=np.float32)
        return float(lib().oracle_loss_glm_f32(_p(Xr, _pf), Xr.shape[1], Xr.shape[0],
                                               Xr.shape[1], _p(yv, _pf), _p(xv, _pd), lc))
    Xr, yv = _f64(X), _f64(y)
    return float(lib().oracle_loss_glm(_p(Xr, _pd), Xr.shape[1], Xr.shape[0], Xr.shape[1],
                                       _p(yv, _pd), _p(xv, _pd), lc))


def loss_value_csr(row_ptr, col_idx, values, y, x, loss="logistic") -> float:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    va, yv, xv = _f64(values), _f64(y), _f64(x)
    return float(lib().oracle_loss_glm_csr(_p(rp, _pi64), _p(ci, _pi32), _p(va, _pd),
                                           rp.shape[0] - 1, _p(yv, _pd), _p(xv, _pd),
                                           _loss_code(loss)))


def logloss(X, y, x) -> float:
    """Mean logistic loss m^-1 sum log(1 + exp(-y_i a_i^T x)) (Sec. 2.1)."""
    xv = _f64(x)
    if X.dtype == np.float32:
        Xr = np.ascontiguousarray(X)
        yv = np.ascontiguousarray(y, dtype=np.float32)
        return float(lib().oracle_logloss_f32(_p(Xr, _pf), Xr.shape[1], Xr.shape[0],
                                              Xr.shape[1], _p(yv, _pf), _p(xv, _pd)))
    Xr, yv = _f64(X), _f64(y)
    return float(lib().oracle_logloss(_p(Xr, _pd), Xr.shape[1], Xr.shape[0],
                                      Xr.shape[1], _p(yv, _pd), _p(xv, _pd)))


def objective(X, y, x, lam: float) -> float:
    """Training objective F_lambda(x) = logloss + (lambda/2) ||x||^2."""
    xv = _f64(x)
    return logloss(X, y, xv) + 0.5 * lam * float(xv @ xv)


def casgd_csr(row_ptr, col_idx, values, n: int, y, x0, eta: float, lam: float,
              b: int, s: int, seed: int, outer0: int = 0, nouter: int = 1,
              loss="logistic") -> np.ndarray:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    va = _f64(values)
    yv = _f64(y)
    x = _f64(x0).copy()
    _check(lib().oracle_casgd_csr_glm(_p(rp, _pi64), _p(ci, _pi32), _p(va, _pd),
                                      rp.shape[0] - 1, n, _p(yv, _pd), _p(x, _pd), eta, lam,
                                      b, s, seed, outer0, nouter, _loss_code(loss)))
    return x


def logloss_csr(row_ptr, col_idx, values, y, x) -> float:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    va, yv, xv = _f64(values), _f64(y), _f64(x)
    return float(lib().oracle_logloss_csr(_p(rp, _pi64), _p(ci, _pi32), _p(va, _pd),
                                          rp.shape[0] - 1, _p(yv, _pd), _p(xv, _pd)))


# ------------------------------------------- independent pure-Python SGD (tiny)

_M64 = 2**64 - 1


def _py_splitmix(seed: int, t: int) -> int:
    z = (seed + (t + 1) * 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def py_sample_indices(seed: int, t0: int, count: int, m: int) -> np.ndarray:
    return np.array([(_py_splitmix(seed, t0 + q) * m) >> 64 for q in range(count)],
                    dtype=np.int64)


def py_sgd(X, y, x0, eta, lam, b, seed, nsteps, loss="logistic"):
    """Second implementation of plain SGD with NumPy vector ops (tiny inputs).

    Independent of the C core: it recomputes the samples, the residual and the
    step from the definitions with NumPy's own dot products.
    """
    X = _f64(X)
    y = _f64(y)
    x = _f64(x0).copy()
    m = X.shape[0]
    lc = _loss_code(loss)
    for k in range(nsteps):
        I = py_sample_indices(seed, k * b, b, m)
        Y = X[I]
        z = Y @ x
        yi = y[I]
        if lc == 1:
            dlt = yi - z                                         # linear
        elif lc == 2:
            dlt = yi - np.exp(z)                                 # Poisson
        else:
            dlt = yi * (1.0 - 1.0 / (1.0 + np.exp(-yi * z)))     # y (1 - sigma(y z))
        x = (1.0 - eta * lam) * x + (eta / b) * (Y.T @ dlt)
    return x


# --------------------------------------------------------- storage formats

U_FP32 = 2.0 ** -24
U_BF16 = 2.0 ** -8
U_FP16 = 2.0 ** -11
U_E4M3 = 2.0 ** -4
U_FP64 = 2.0 ** -53


def bf16_round(x32: np.ndarray) -> np.ndarray:
    """Round FP32 values to BF16 (round to nearest, ties to even); FP32 result."""
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def bf16_bits(x32: np.ndarray) -> np.ndarray:
    return (bf16_round(x32).view(np.uint32) >> 16).astype(np.uint16)


def fp16_round(x32: np.ndarray) -> np.ndarray:
    return np.asarray(x32, dtype=np.float32).astype(np.float16).astype(np.float32)


def e4m3_values() -> np.ndarray:
    """Magnitudes of the 127 finite OCP FP8-e4m3 codes 0x00..0x7E (ascending).

    Bias 7, three mantissa bits; exponent field 0 is subnormal (m * 2^-9);
    0x7F is NaN and there is no infinity, so the largest value is 448.
    """
    v = np.empty(127)
    for c in range(127):
        e, mnt = c >> 3, c & 7
        v[c] = mnt * 2.0 ** -9 if e == 0 else (1.0 + mnt / 8.0) * 2.0 ** (e - 7)
    return v


_E4M3 = e4m3_values()


def e4m3_encode(v32: np.ndarray) -> np.ndarray:
    """FP32 -> e4m3 code, round to nearest (ties to even code), saturating at 448."""
    v = np.asarray(v32, dtype=np.float32).astype(np.float64)
    a = np.abs(v)
    p = np.searchsorted(_E4M3, a, side="left")
    p = np.clip(p, 1, 126)
    lo, hi = _E4M3[p - 1], _E4M3[p]
    dl, dh = a - lo, hi - a
    pick_hi = (dh < dl) | ((dh == dl) & ((p % 2) == 0))
    code = np.where(pick_hi, p, p - 1)
    code = np.where(a >= 448.0, 126, code)
    code = np.where(a == 0, 0, code)
    sign = np.signbit(v).astype(np.uint8) << 7
    return (code.astype(np.uint8) | sign).astype(np.uint8)


def e4m3_decode(codes: np.ndarray) -> np.ndarray:
    c = np.asarray(codes, dtype=np.uint8)
    mag = _E4M3[np.minimum(c & 0x7F, 126)]
    return np.where(c & 0x80, -mag, mag)


def quantize_rows_e4m3(X32: np.ndarray):
    """Per-row scaled FP8-e4m3 storage, written out from its definition.

    amax_i = max_k |X_ik| (FP32); scale_i = amax_i / 448 and
    inv_i = 448 / amax_i (both FP32 divisions); q_ik = e4m3(X_ik * inv_i)
    with the product rounded to FP32 first. An all-zero row has scale 1.
    Returns (codes uint8 m x n, scale float32 m, dequantised FP64 m x n).
    """
    X = np.ascontiguousarray(X32, dtype=np.float32)
    amax = np.abs(X).max(axis=1).astype(np.float32)
    zero = amax == 0
    safe = np.where(zero, np.float32(448.0), amax).astype(np.float32)
    scale = np.where(zero, np.float32(1.0), safe / np.float32(448.0)).astype(np.float32)
    inv = np.where(zero, np.float32(1.0), np.float32(448.0) / safe).astype(np.float32)
    v = (X * inv[:, None]).astype(np.float32)
    codes = e4m3_encode(v)
    deq = e4m3_decode(codes) * scale.astype(np.float64)[:, None]
    return codes, scale, deq


def quantize(X32: np.ndarray, fmt: str):
    """(stored representation, row scale or None, exact FP64 values)."""
    X32 = np.ascontiguousarray(X32, dtype=np.float32)
    if fmt == "f32":
        return X32, None, X32.astype(np.float64)
    if fmt == "bf16":
        r = bf16_round(X32)
        return (r.view(np.uint32) >> 16).astype(np.uint16), None, r.astype(np.float64)
    if fmt == "f16":
        h = X32.astype(np.float16)
        return h, None, h.astype(np.float64)
    if fmt == "fp8":
        codes, scale, deq = quantize_rows_e4m3(X32)
        return codes, scale, deq
    raise ValueError(fmt)


def round_to_format(v, fmt: str | None) -> np.ndarray:
    """Round FP64 values to BF16 or FP16 (round to nearest, ties to even,
    subnormals of the format included; FP16 overflows to +-inf); fmt None
    returns the values unchanged."""
    v = np.asarray(v, dtype=np.float64)
    if fmt is None:
        return v.copy()
    p, emin = {"bf16": (8, -126), "f16": (11, -14)}[fmt]
    _, e = np.frexp(v)
    q = np.maximum(e - p, emin - p + 1)              # quantum exponent at v's binade
    r = np.ldexp(np.rint(np.ldexp(v, -q)), q)
    if fmt == "f16":
        r = np.where(np.abs(r) > 65504.0, np.copysign(np.inf, r), r)
    return r


def casgd_e2e(X, y, x0, eta: float, lam: float, b: int, s: int, seed: int, outer0: int,
              nouter: int, fmt: str | None, loss="logistic", snapshots: bool = False):
    """End-to-end low-precision s-step SGD (the paper's all-BF16 / all-FP16
    recipes, Table 3): Algorithm 1 with every slot's output rounded to `fmt`
    (round_to_format), sums exact in FP64 before the rounding:
        G = fl(Y Y^T) (strict block-lower), r = fl(Y x),
        a_j = fl(sum_{i<j} beta^(j-1-i) G_{j,i} delta_i), z_j = fl(beta^j r_j + alpha a_j),
        delta_j = fl(delta(z_j, y_j)), c_j = fl(beta^(s-1-j) delta_j),
        g = fl(Y^T c), x <- fl(beta^s x + alpha g).
    X holds the exact stored values. Returns x (and the list of iterates after
    every outer iteration when snapshots)."""
    Xr = _f64(X)
    yv = _f64(y)
    x = round_to_format(_f64(x0), fmt)
    m = Xr.shape[0]
    alpha, beta = eta / b, 1.0 - eta * lam
    lc = _loss_code(loss)
    sb = s * b
    snaps = []
    for h in range(outer0, outer0 + nouter):
        idx = sample_indices(seed, h * sb, sb, m)
        Y, yI = Xr[idx], yv[idx]
        G = round_to_format(Y @ Y.T, fmt)
        r = round_to_format(Y @ x, fmt)
        d = np.zeros(sb)
        for j in range(s):
            rows = slice(j * b, (j + 1) * b)
            a = np.zeros(b)
            for i in range(j):
                a += beta ** (j - 1 - i) * (G[rows, i * b:(i + 1) * b] @ d[i * b:(i + 1) * b])
            a = round_to_format(a, fmt)
            z = round_to_format(beta ** j * r[rows] + alpha * a, fmt)
            d[rows] = round_to_format([delta(float(zz), float(yy), lc)
                                       for zz, yy in zip(z, yI[rows])], fmt)
        c = round_to_format(np.repeat(beta ** (s - 1 - np.arange(s)), b) * d, fmt)
        g = round_to_format(Y.T @ c, fmt)
        x = round_to_format(beta ** s * x + alpha * g, fmt)
        if snapshots:
            snaps.append(x.copy())
    return (x, snaps) if snapshots else x


def unit_roundoff(fmt: str) -> float:
    return {"f64": U_FP64, "f32": U_FP32, "bf16": U_BF16, "f16": U_FP16,
            "fp8": U_E4M3}[fmt]


# ------------------------------------------------- Higham factor and bounds

def gamma(q: int, u: float) -> float:
    """Deterministic inner-product factor gamma_q = q u / (1 - q u) (Sec. 3.2)."""
    qu = q * u
    if qu >= 1.0:
        return math.inf
    return qu / (1.0 - qu)


def strict_block_lower_mask(b: int, s: int) -> np.ndarray:
    blk = np.arange(s * b) // b
    return blk[:, None] > blk[None, :]


def local_error_bound(Y, x, yI, b: int, s: int, eta: float, *, u_A: float,
                      gamma_r: float, gamma_G: float, u_c: float, u_sigma: float,
                      gamma_g: float, u_x: float, C_delta: float = 8.0,
                      D_delta: float = 1.0, L_sigma: float = 0.25,
                      C_loc: float = 2.0, loss="logistic") -> dict:
    """Local forward-error bound of one outer iteration (Thm. 5.1, P = 1).

    Y (sb x n, exact rows), x and yI are the exact inputs. With one device
    the two all-reduce rows vanish. Returns the nine-term sum, Omega and the
    bound (1 + C_loc * Omega) * sum (remainder read with C_loc = 2).
    The theorem is stated for the paper's method without an L2 term, so the
    exact residual history d comes from the lambda = 0 recurrence.
    """
    Y = _f64(Y)
    x = _f64(x)
    yI = _f64(yI)
    sb = s * b
    alpha = eta / b
    G = Y @ Y.T
    mask = strict_block_lower_mask(b, s)
    GL = np.where(mask, G, 0.0)
    absY = np.abs(Y)
    HL = np.where(mask, absY @ absY.T, 0.0)
    r = Y @ x
    d, _ = inner_corrections(GL, r, yI, b, s, eta, 0.0, loss=loss)
    M = L_sigma * alpha * np.abs(GL)
    # Neumann series terminates: |G_L| is strictly block-lower, so M^s = 0.
    inv = np.eye(sb)
    P = np.eye(sb)
    for _ in range(1, s):
        P = P @ M
        inv = inv + P
    K_s = float(np.linalg.norm(inv, 2))
    normY = float(np.linalg.norm(Y, 2))
    T_g = float(np.linalg.norm(absY.T @ np.abs(d)))
    T_r = float(np.linalg.norm(absY @ np.abs(x)))
    T_G = float(np.linalg.norm(HL @ np.abs(d)))
    tc = 0.0
    for j in range(1, s):
        Gj = G[j * b:(j + 1) * b, :j * b]
        tc += (j * b * np.linalg.norm(Gj, "fro") * np.linalg.norm(d[:j * b])) ** 2
    T_c = math.sqrt(tc)
    x_s = x + alpha * (Y.T @ d)
    a1 = alpha * normY * K_s * L_sigma
    E = dict(
        A=a1 * u_A * T_r + 2 * alpha * a1 * u_A * T_G + alpha * u_A * T_g,
        r=a1 * gamma_r * T_r,
        G=alpha * a1 * gamma_G * T_G,
        c=a1 * u_c * T_r + 2 * alpha * a1 * u_c * T_G + alpha * a1 * u_c * T_c,
        sigma=alpha * normY * K_s * C_delta * u_sigma * D_delta * math.sqrt(sb),
        g=alpha * gamma_g * T_g,
        x=u_x * (float(np.linalg.norm(x_s)) + alpha * float(np.linalg.norm(Y.T @ d))),
    )
    total = sum(E.values())
    omega = max(u_A, gamma_r, gamma_G, gamma((s - 1) * b, u_c), gamma_g, u_sigma, u_x)
    tau = K_s * L_sigma * alpha * (2 * u_A + gamma_G) * float(np.linalg.norm(HL, 2))
    Omega = max(omega, tau)
    return dict(E=E, sum=total, Omega=Omega, K_s=K_s, bound=(1 + C_loc * Omega) * total,
                x_exact=x_s, norm_Y=normY, norm_HL=float(np.linalg.norm(HL, 2)), T_g=T_g,
                T_r=T_r, T_G=T_G, T_c=T_c, d=d)


def uniform_precision_bound(Y, x, yI, b, s, eta, u, **kw) -> dict:
    """Cor. 5.2: every slot at unit roundoff u, gamma_r = gamma_G = gamma_n,
    gamma_g = gamma_sb."""
    n = np.asarray(Y).shape[1]
    return local_error_bound(Y, x, yI, b, s, eta, u_A=u, gamma_r=gamma(n, u),
                             gamma_G=gamma(n, u), u_c=u, u_sigma=u,
                             gamma_g=gamma(s * b, u), u_x=u, **kw)


def lowp_fp32acc_factor(n: int, u_in: float) -> float:
    """Input-cast plus FP32-accumulate factor 2 u_in + gamma_n(u32) (Sec. 5.2)."""
    return 2 * u_in + gamma(n, U_FP32)


# ------------------------------------------------------ column statistics

def column_stats(X) -> np.ndarray:
    """Per column: mean, population variance, fraction of nonzeros, max |x|."""
    X = _f64(X)
    m = X.shape[0]
    mean = X.sum(axis=0) / m
    var = ((X - mean) ** 2).sum(axis=0) / m
    nnz = (X != 0).sum(axis=0) / m
    amax = np.abs(X).max(axis=0)
    return np.stack([mean, var, nnz, amax], axis=1)


def column_stats_csr(row_ptr, col_idx, values, m: int, n: int) -> np.ndarray:
    ci = np.asarray(col_idx, dtype=np.int64)
    v = _f64(values)
    s1 = np.bincount(ci, weights=v, minlength=n)
    s2 = np.bincount(ci, weights=v * v, minlength=n)
    cnt = np.bincount(ci, minlength=n).astype(np.float64)
    mean = s1 / m
    var = s2 / m - mean ** 2
    amax = np.zeros(n)
    np.maximum.at(amax, ci, np.abs(v))
    return np.stack([mean, var, cnt / m, amax], axis=1)


# ------------------------------------- learned preconditioner: targets and use

def hess_diag(X, x, lam: float) -> np.ndarray:
    """Diagonal of the Hessian of the mean logistic loss (Sec. 2.1) plus the L2
    term at x: m^-1 sum_i s(z_i)(1 - s(z_i)) X_ik^2 + lam, z_i = X_i . x."""
    X = _f64(X)
    z = X @ _f64(x)
    s = 1.0 / (1.0 + np.exp(-z))
    return (s * (1.0 - s)) @ (X * X) / X.shape[0] + lam


def jacobi_target(h) -> tuple:
    """(t_d, q): t_d = -log h centred to zero mean (log of a Jacobi scale with
    unit geometric mean) and the column scale q = exp(t_d / 2)."""
    t = -np.log(_f64(h))
    t = t - t.mean()
    return t, np.exp(0.5 * t)


def feature_norm(stats) -> tuple:
    """(mu, sd) of log(1 + |stat|) per statistic over all rows; sample std,
    floored at 1e-6."""
    L = np.log1p(np.abs(_f64(stats)))
    return L.mean(axis=0), np.maximum(L.std(axis=0, ddof=1), 1e-6)


def mlp_apply(o) -> tuple:
    """(q, eta) for one problem from its forward output o (N x 2):
    q = exp(clip(o0 - mean o0, -20, 20) / 2), eta = exp(mean o1)."""
    o = _f64(o)
    t = np.clip(o[:, 0] - o[:, 0].mean(), -20.0, 20.0)
    return np.exp(0.5 * t), float(np.exp(o[:, 1].mean()))


# ------------------------------------------------------- MLP (FP64 reference)

def mlp_features(stats: np.ndarray, mu: np.ndarray, sd: np.ndarray) -> np.ndarray:
    """Standardised log(1 + |stat|) features (one row per column)."""
    return (np.log1p(np.abs(_f64(stats))) - mu) / sd


def mlp_forward(F, W1, b1, W2, b2):
    """h = relu(F W1^T + b1); o = h W2^T + b2.  F: N x 4, W1: H x 4, W2: O x H."""
    pre = _f64(F) @ _f64(W1).T + _f64(b1)
    h = np.maximum(pre, 0.0)
    o = h @ _f64(W2).T + _f64(b2)
    return o, h, pre


def mlp_loss(o: np.ndarray, seg: np.ndarray, t_d: np.ndarray, t_eta: np.ndarray,
             w_eta: float = 1.0):
    """Training loss of the learned preconditioner and its gradient wrt o.

    Rows of o belong to problems given by ``seg`` (problem id per row).
    Column 0 predicts log d_k (target t_d per row); column 1 is averaged per
    problem into the log step size (target t_eta per problem).
      loss = mean_rows (o0 - t_d)^2 + w_eta * mean_problems (mean_p o1 - t_eta)^2
    """
    o = _f64(o)
    seg = np.asarray(seg, dtype=np.int64)
    P = t_eta.shape[0]
    N = o.shape[0]
    cnt = np.bincount(seg, minlength=P).astype(np.float64)
    e0 = o[:, 0] - t_d
    pm = np.bincount(seg, weights=o[:, 1], minlength=P) / cnt
    e1 = pm - t_eta
    loss = float((e0 ** 2).sum() / N + w_eta * (e1 ** 2).sum() / P)
    g = np.zeros_like(o)
    g[:, 0] = 2.0 * e0 / N
    g[:, 1] = w_eta * 2.0 * e1[seg] / (P * cnt[seg])
    return loss, g


def mlp_backward(F, h, pre, W2, g_o):
    """Gradients of a scalar loss wrt W1, b1, W2, b2 given dLoss/do."""
    F, h, pre, W2, g_o = map(_f64, (F, h, pre, W2, g_o))
    gW2 = g_o.T @ h
    gb2 = g_o.sum(axis=0)
    g_h = g_o @ W2
    g_pre = g_h * (pre > 0)
    gW1 = g_pre.T @ F
    gb1 = g_pre.sum(axis=0)
    return gW1, gb1, gW2, gb2


def adam_step(p, g, m1, m2, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) with bias correction; returns new
    (p, m1, m2). t counts from 1."""
    m1 = beta1 * m1 + (1 - beta1) * g
    m2 = beta2 * m2 + (1 - beta2) * g * g
    mh = m1 / (1 - beta1 ** t)
    vh = m2 / (1 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m1, m2
