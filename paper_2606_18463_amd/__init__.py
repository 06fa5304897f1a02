"""MI355X-native s-step (communication-avoiding) SGD for L2-regularised logistic
regression.

Python binding of libcasgd (``include/casgd.h``). Every function here only
marshals arguments: tensors are passed to the C ABI by device pointer and the
current HIP stream; all computation happens in the library's HIP kernels.
PyTorch is used for device memory and streams.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import BF16, CSR, DENSE, F16, F32, FP8E4M3  # noqa: F401
from ._lib import LOSS_LINEAR, LOSS_LOGISTIC, LOSS_POISSON, LOSSES  # noqa: F401

__all__ = [
    "CasgdError", "dense_matrix", "csr_matrix", "opts", "workspace",
    "casgd_workspace_size", "casgd_gram_workspace_size", "casgd_reset", "casgd_step", "casgd_fit",
    "casgd_check", "casgd_fit_noalloc",
    "casgd_sample_indices", "casgd_gram_margin", "casgd_recurrence", "casgd_update",
    "casgd_quantize", "casgd_logloss", "casgd_loss", "casgd_colstats", "casgd_version",
    "casgd_recurrence_workspace_size",
    "casgd_path_workspace_size", "casgd_sparse_prepare", "casgd_fit_path",
    "casgd_fit_batch", "casgd_quantize_scaled", "casgd_mlp_features", "casgd_mlp_forward",
    "casgd_mlp_loss_grad", "casgd_mlp_backward", "casgd_adam_step", "casgd_hess_diag",
    "casgd_select_precision", "MLP_PARAMS",
]

MLP_PARAMS = 450


class CasgdError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{_lib.STATUS_NAMES.get(status, status)}: {message}")


def _L():
    return _lib.load()


def _check(rc: int) -> None:
    if rc != 0:
        raise CasgdError(rc, _L().casgd_last_error().decode())


def _torch():
    import torch
    return torch


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


_DTYPES = {}


def _dtype_code(t) -> int:
    torch = _torch()
    if not _DTYPES:
        _DTYPES.update({torch.float32: F32, torch.bfloat16: BF16, torch.float16: F16,
                        torch.uint8: FP8E4M3, torch.float8_e4m3fn: FP8E4M3})
    return _DTYPES[t.dtype]


class MatrixRef:
    """A casgd_matrix plus references that keep its tensors alive."""

    def __init__(self, struct: _lib.Matrix, keep: tuple):
        self.struct = struct
        self._keep = keep

    @property
    def m(self) -> int:
        return self.struct.m

    @property
    def n(self) -> int:
        return self.struct.n

    @property
    def dtype(self) -> int:
        return self.struct.dtype

    def ref(self):
        return ctypes.byref(self.struct)


def dense_matrix(values, row_scale=None, n: int | None = None) -> MatrixRef:
    """Dense row-major X: ``values`` (m x ld device tensor; float32, bfloat16,
    float16, or uint8/float8_e4m3fn holding E4M3 codes); ``n`` <= ld valid
    columns (default ld)."""
    assert values.dim() == 2 and values.is_cuda and values.stride(1) == 1
    m, ld = values.shape[0], values.stride(0)
    s = _lib.Matrix(m=m, n=(n if n is not None else values.shape[1]), ld=ld,
                    dtype=_dtype_code(values), layout=DENSE, values=_ptr(values),
                    row_scale=_ptr(row_scale), row_ptr=None, col_idx=None, nnz=0)
    return MatrixRef(s, (values, row_scale))


def csr_matrix(row_ptr, col_idx, values, n: int) -> MatrixRef:
    """CSR X: row_ptr (int64, m+1), col_idx (int32, sorted per row), values (float32)."""
    torch = _torch()
    assert row_ptr.dtype == torch.int64 and col_idx.dtype == torch.int32
    assert values.dtype == torch.float32
    s = _lib.Matrix(m=row_ptr.numel() - 1, n=n, ld=0, dtype=F32, layout=CSR,
                    values=_ptr(values), row_scale=None, row_ptr=_ptr(row_ptr),
                    col_idx=_ptr(col_idx), nnz=values.numel())
    return MatrixRef(s, (row_ptr, col_idx, values))


def _loss_code(loss) -> int:
    return LOSSES[loss] if isinstance(loss, str) else int(loss)


def opts(recur_prec: int = 0, exec_mode: int = 0, snapshot_every: int = 0, x_history=None,
         t_history=None, spin_limit: int = 0, fused_variant: int = 0, grid_blocks: int = 0,
         phase_trace=None, rec_split: int = 0, loss=0, e2e: int = 0, gram_tile: int = 0):
    """casgd_opts; phase_trace: device int64 tensor of 8 words per traced outer iteration;
    loss: "logistic", "linear", "poisson" or its code; e2e: 0, 1 (BF16), 2 (FP16)."""
    o = _lib.Opts(recur_prec=recur_prec, exec_mode=exec_mode, snapshot_every=snapshot_every,
                  x_history=_ptr(x_history), t_history=_ptr(t_history), spin_limit=spin_limit,
                  fused_variant=fused_variant, grid_blocks=grid_blocks,
                  phase_trace=_ptr(phase_trace),
                  phase_trace_outer=0 if phase_trace is None else phase_trace.numel() // 8,
                  rec_split=rec_split, loss=_loss_code(loss), e2e=e2e, gram_tile=gram_tile)
    o._keep = (x_history, t_history, phase_trace)
    return o


def casgd_version() -> int:
    return int(_L().casgd_version())


def casgd_workspace_size(X: MatrixRef, b: int, s: int) -> int:
    out = ctypes.c_size_t(0)
    _check(_L().casgd_workspace_size(X.ref(), b, s, ctypes.byref(out)))
    return int(out.value)


def workspace(nbytes: int, device=None):
    """A zeroed, 256-byte aligned device buffer of nbytes (torch allocation)."""
    torch = _torch()
    t = torch.zeros(max(nbytes, 256) + 256, dtype=torch.uint8, device=device or "cuda")
    off = (-t.data_ptr()) % 256
    return t[off:off + max(nbytes, 256)]


def _ws(ws, need: int):
    if ws is None:
        ws = workspace(need)
    return ws, ws.numel()


def casgd_reset(ws, stream=None) -> None:
    _check(_L().casgd_reset(_ptr(ws), ws.numel(), _stream(stream)))


def casgd_check(ws, stream=None) -> None:
    _check(_L().casgd_check(_ptr(ws), ws.numel(), _stream(stream)))


def _opts_ref(o):
    return None if o is None else ctypes.byref(o)


def casgd_fit(X: MatrixRef, y, x, eta: float, lam: float, b: int, s: int, seed: int,
              outer_begin: int = 0, n_outer: int = 1, opts=None, ws=None, stream=None):
    """Outer iterations outer_begin .. outer_begin + n_outer - 1 on x (in place)."""
    ws, nb = _ws(ws, casgd_workspace_size(X, b, s))
    _check(_L().casgd_fit(X.ref(), _ptr(y), _ptr(x), eta, lam, b, s, seed, outer_begin,
                          n_outer, _opts_ref(opts), _ptr(ws), nb, _stream(stream)))
    return ws


def casgd_fit_noalloc(X: MatrixRef, y, x, eta: float, lam: float, b: int, s: int, seed: int,
                      outer_begin: int = 0, n_outer: int = 1, opts=None, status=None,
                      stream=None):
    """casgd_fit with the library's static device scratch array as workspace (no
    device allocation). status: optional device int32 tensor (1 element) that
    receives the flag status after the fit."""
    _check(_L().casgd_fit_noalloc(X.ref(), _ptr(y), _ptr(x), eta, lam, b, s, seed, outer_begin,
                                  n_outer, _opts_ref(opts), _ptr(status), _stream(stream)))
    return status


def casgd_step(X: MatrixRef, y, x, eta: float, lam: float, b: int, s: int, seed: int,
               outer_iter: int, opts=None, ws=None, stream=None):
    ws, nb = _ws(ws, casgd_workspace_size(X, b, s))
    _check(_L().casgd_step(X.ref(), _ptr(y), _ptr(x), eta, lam, b, s, seed, outer_iter,
                           _opts_ref(opts), _ptr(ws), nb, _stream(stream)))
    return ws


def casgd_path_workspace_size(X: MatrixRef, b: int, s: int, lanes: int) -> int:
    out = ctypes.c_size_t(0)
    _check(_L().casgd_path_workspace_size(X.ref(), b, s, lanes, ctypes.byref(out)))
    return int(out.value)


def casgd_sparse_prepare(X: MatrixRef, b: int, s: int, lanes: int = 1, ws=None, stream=None):
    """Prepare (and if needed allocate) a workspace for a CSR X; returns it."""
    ws, nb = _ws(ws, casgd_path_workspace_size(X, b, s, lanes))
    _check(_L().casgd_sparse_prepare(X.ref(), b, s, lanes, _ptr(ws), nb, _stream(stream)))
    return ws


def casgd_fit_path(X: MatrixRef, y, x_lanes, lambdas, eta: float, b: int, s: int, seed: int,
                   outer_begin: int = 0, n_outer: int = 1, opts=None, ws=None, stream=None):
    """Regularisation path on a CSR X: x_lanes (n x L) in place, one lane per lambda."""
    lam = (ctypes.c_double * len(lambdas))(*[float(v) for v in lambdas])
    if ws is None:
        ws = casgd_sparse_prepare(X, b, s, len(lambdas), stream=stream)
    _check(_L().casgd_fit_path(X.ref(), _ptr(y), _ptr(x_lanes), lam, len(lambdas), eta, b, s,
                               seed, outer_begin, n_outer, _opts_ref(opts), _ptr(ws), ws.numel(),
                               _stream(stream)))
    return ws


def casgd_fit_batch(problems, spin_limit: int = 0, stream=None):
    """Fit many dense problems in one launch. `problems`: list of dicts with keys
    X (MatrixRef), y, x, eta, lam, b, s, seed and optionally outer_begin,
    n_outer, ws, groups, variant, recur_prec, loss, snapshot_every, x_history,
    t_history. Returns the list of workspaces."""
    n = len(problems)
    arr = (_lib.Problem * n)()
    keep = []
    for i, q in enumerate(problems):
        X = q["X"]
        ws = q.get("ws")
        if ws is None:
            ws = workspace(casgd_workspace_size(X, q["b"], q["s"]))
        keep.append((X, ws))
        arr[i] = _lib.Problem(X=X.struct, y=_ptr(q["y"]), x=_ptr(q["x"]), eta=q["eta"],
                              lam=q["lam"], b=q["b"], s=q["s"], seed=q["seed"],
                              outer_begin=q.get("outer_begin", 0), n_outer=q.get("n_outer", 1),
                              ws=_ptr(ws), ws_bytes=ws.numel(), groups=q.get("groups", 0),
                              variant=q.get("variant", 0), recur_prec=q.get("recur_prec", 0),
                              loss=_loss_code(q.get("loss", 0)),
                              snapshot_every=q.get("snapshot_every", 0),
                              x_history=_ptr(q.get("x_history")),
                              t_history=_ptr(q.get("t_history")),
                              gram_tile=q.get("gram_tile", 0), reserved=0)
    tb = workspace(int(_L().casgd_batch_table_size(n)))
    _check(_L().casgd_fit_batch(arr, n, spin_limit, _ptr(tb), tb.numel(), _stream(stream)))
    for i, q in enumerate(problems):
        q["groups_used"] = int(arr[i].groups)
        q["variant_used"] = int(arr[i].variant)
    return [w for _, w in keep]


def casgd_sample_indices(seed: int, t0: int, count: int, m: int, out=None, stream=None):
    torch = _torch()
    out = out if out is not None else torch.empty(count, dtype=torch.int64, device="cuda")
    _check(_L().casgd_sample_indices(seed, t0, count, m, _ptr(out), _stream(stream)))
    return out


def casgd_gram_workspace_size(X: MatrixRef, b: int, s: int) -> int:
    out = ctypes.c_size_t(0)
    _check(_L().casgd_gram_workspace_size(X.ref(), b, s, ctypes.byref(out)))
    return int(out.value)


def casgd_gram_margin(X: MatrixRef, x, b: int, s: int, seed: int, outer_iter: int, G=None,
                      r=None, ws=None, stream=None, opts=None):
    """Margins and Gram of one outer iteration. The workspace (allocated here
    when None) holds the K-split Gram's exchange region."""
    torch = _torch()
    sb = s * b
    G = G if G is not None else torch.zeros(sb, sb, dtype=torch.float32, device="cuda")
    if x is not None and r is None:
        r = torch.zeros(sb, dtype=torch.float32, device="cuda")
    ws, nb = _ws(ws, casgd_gram_workspace_size(X, b, s))
    _check(_L().casgd_gram_margin(X.ref(), _ptr(x), b, s, seed, outer_iter, _ptr(G), _ptr(r),
                                  _opts_ref(opts), _ptr(ws), nb, _stream(stream)))
    return G, r


def casgd_recurrence_workspace_size(b: int, s: int) -> int:
    return int(_L().casgd_recurrence_workspace_size(b, s))


def casgd_recurrence(G, r, yI, b: int, s: int, eta: float, lam: float, prec: int = 0,
                     c=None, delta=None, loss=0, form: int = 0, ws=None, stream=None):
    """The s residual corrections from device G, r, yI; returns c. form 1: one
    workgroup; form 2: chain + helper workgroups (b in 16, 32, 64, 128); 0: auto.
    ws: the flag/exchange workspace (allocated when None); read its flags with
    casgd_check(ws)."""
    torch = _torch()
    c = c if c is not None else torch.empty(s * b, dtype=torch.float32, device="cuda")
    if ws is None:
        ws = workspace(casgd_recurrence_workspace_size(b, s))
    _check(_L().casgd_recurrence(_ptr(G), _ptr(r), _ptr(yI), b, s, eta, lam, prec,
                                 _loss_code(loss), form, _ptr(c), _ptr(delta), _ptr(ws),
                                 ws.numel(), _stream(stream)))
    return c


def casgd_update(X: MatrixRef, x, c, b: int, s: int, seed: int, outer_iter: int, eta: float,
                 lam: float, ws=None, stream=None):
    ws, nb = _ws(ws, casgd_workspace_size(X, b, s))
    _check(_L().casgd_update(X.ref(), _ptr(x), _ptr(c), b, s, seed, outer_iter, eta, lam,
                             _ptr(ws), nb, _stream(stream)))
    return x


def casgd_quantize(src, dtype: int, ld_dst: int | None = None, stream=None):
    """Convert an FP32 (m x n) device tensor to storage dtype; returns
    (stored tensor m x ld_dst, row_scale or None)."""
    torch = _torch()
    m, n = src.shape
    vec = {F32: 4, BF16: 8, F16: 8, FP8E4M3: 16}[dtype]
    ld = ld_dst or ((n + vec - 1) // vec * vec)
    tdt = {F32: torch.float32, BF16: torch.bfloat16, F16: torch.float16,
           FP8E4M3: torch.uint8}[dtype]
    dst = torch.empty(m, ld, dtype=tdt, device=src.device)
    scale = torch.empty(m, dtype=torch.float32, device=src.device) if dtype == FP8E4M3 else None
    _check(_L().casgd_quantize(_ptr(src), m, n, src.stride(0), dtype, _ptr(dst), ld, _ptr(scale),
                               _stream(stream)))
    return dst, scale


def casgd_quantize_scaled(src, col_scale, dtype: int, ld_dst: int | None = None, stream=None):
    """casgd_quantize of src * col_scale (columns scaled, e.g. by sqrt(d))."""
    torch = _torch()
    m, n = src.shape
    vec = {F32: 4, BF16: 8, F16: 8, FP8E4M3: 16}[dtype]
    ld = ld_dst or ((n + vec - 1) // vec * vec)
    tdt = {F32: torch.float32, BF16: torch.bfloat16, F16: torch.float16,
           FP8E4M3: torch.uint8}[dtype]
    dst = torch.empty(m, ld, dtype=tdt, device=src.device)
    scale = torch.empty(m, dtype=torch.float32, device=src.device) if dtype == FP8E4M3 else None
    _check(_L().casgd_quantize_scaled(_ptr(src), m, n, src.stride(0), _ptr(col_scale), dtype,
                                      _ptr(dst), ld, _ptr(scale), _stream(stream)))
    return dst, scale


def casgd_mlp_features(stats, norm, stream=None):
    torch = _torch()
    feats = torch.empty_like(stats)
    _check(_L().casgd_mlp_features(_ptr(stats), stats.shape[0], _ptr(norm), _ptr(feats),
                                   _stream(stream)))
    return feats


def casgd_mlp_feature_norm(stats, stream=None):
    """(8,) device FP32: means then standard deviations of log(1 + |stats|)."""
    torch = _torch()
    norm = torch.empty(8, dtype=torch.float32, device=stats.device)
    _check(_L().casgd_mlp_feature_norm(_ptr(stats), stats.shape[0], _ptr(norm), _stream(stream)))
    return norm


def casgd_mlp_apply(out, stream=None):
    """(q, eta) from a forward output of one problem: column scale q = sqrt(d) (N,)
    and step size eta (1,), device FP32."""
    torch = _torch()
    N = out.shape[0]
    q = torch.empty(N, dtype=torch.float32, device=out.device)
    eta = torch.empty(1, dtype=torch.float32, device=out.device)
    _check(_L().casgd_mlp_apply(_ptr(out), N, _ptr(q), _ptr(eta), _stream(stream)))
    return q, eta


def casgd_jacobi_target(hdiag, want_q: bool = True, stream=None):
    """(t_d, q or None): centred -log of a Hessian diagonal and exp(t_d / 2)."""
    torch = _torch()
    n = hdiag.numel()
    t_d = torch.empty(n, dtype=torch.float32, device=hdiag.device)
    q = torch.empty(n, dtype=torch.float32, device=hdiag.device) if want_q else None
    _check(_L().casgd_jacobi_target(_ptr(hdiag), n, _ptr(t_d), _ptr(q), _stream(stream)))
    return t_d, q


def casgd_mlp_forward(params, feats, want_pre: bool = True, stream=None):
    torch = _torch()
    N = feats.shape[0]
    out = torch.empty(N, 2, dtype=torch.float32, device=feats.device)
    pre = torch.empty(N, 64, dtype=torch.float32, device=feats.device) if want_pre else None
    _check(_L().casgd_mlp_forward(_ptr(params), _ptr(feats), N, _ptr(out), _ptr(pre),
                                  _stream(stream)))
    return out, pre


def _mlp_ws(N, P):
    return workspace(int(_L().casgd_mlp_workspace_size(N, P)))


def casgd_mlp_loss_grad(out, seg_off, t_d, t_eta, w_eta: float = 1.0, ws=None, stream=None):
    torch = _torch()
    N, P = out.shape[0], seg_off.numel() - 1
    loss = torch.empty(1, dtype=torch.float64, device=out.device)
    g = torch.empty_like(out)
    ws = ws if ws is not None else _mlp_ws(N, P)
    _check(_L().casgd_mlp_loss_grad(_ptr(out), _ptr(seg_off), P, N, _ptr(t_d), _ptr(t_eta),
                                    w_eta, _ptr(loss), _ptr(g), _ptr(ws), ws.numel(),
                                    _stream(stream)))
    return loss, g


def casgd_mlp_backward(params, feats, pre, g_out, P: int = 1, ws=None, stream=None):
    torch = _torch()
    N = feats.shape[0]
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=feats.device)
    ws = ws if ws is not None else _mlp_ws(N, P)
    _check(_L().casgd_mlp_backward(_ptr(params), _ptr(feats), _ptr(pre), _ptr(g_out), N, P,
                                   _ptr(grad), _ptr(ws), ws.numel(), _stream(stream)))
    return grad


def casgd_adam_step(params, grad, m1, m2, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8,
                    stream=None):
    _check(_L().casgd_adam_step(_ptr(params), _ptr(grad), _ptr(m1), _ptr(m2), params.numel(), t,
                                lr, beta1, beta2, eps, _stream(stream)))


def casgd_hess_diag(X: MatrixRef, x, lam: float, stream=None):
    torch = _torch()
    out = torch.empty(X.n, dtype=torch.float32, device="cuda")
    ws = workspace(int(_L().casgd_hess_diag_workspace_size(X.ref())))
    _check(_L().casgd_hess_diag(X.ref(), _ptr(x), lam, _ptr(out), _ptr(ws), ws.numel(),
                                _stream(stream)))
    return out


def casgd_logloss(X: MatrixRef, y, xs, stream=None):
    """Mean logistic loss for each row of xs (k x n) or for a single x (n)."""
    torch = _torch()
    xs2 = xs if xs.dim() == 2 else xs.view(1, -1)
    count = xs2.shape[0]
    out = torch.empty(count, dtype=torch.float64, device="cuda")
    need = int(_L().casgd_logloss_workspace_size(count))
    ws = workspace(need)
    _check(_L().casgd_logloss(X.ref(), _ptr(y), _ptr(xs2), count, xs2.stride(0), _ptr(out),
                              _ptr(ws), ws.numel(), _stream(stream)))
    return out if xs.dim() == 2 else out[0]


def casgd_loss(X: MatrixRef, y, xs, loss="logistic", stream=None):
    """Mean loss (logistic, linear or Poisson, Sec. 2.1) for each row of xs
    (k x n) or for a single x (n); FP64 results on the device."""
    torch = _torch()
    xs2 = xs if xs.dim() == 2 else xs.view(1, -1)
    count = xs2.shape[0]
    out = torch.empty(count, dtype=torch.float64, device="cuda")
    ws = workspace(int(_L().casgd_logloss_workspace_size(count)))
    _check(_L().casgd_loss(X.ref(), _ptr(y), _ptr(xs2), count, xs2.stride(0), _loss_code(loss),
                           _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))
    return out if xs.dim() == 2 else out[0]


def casgd_select_precision(X: MatrixRef, y, x, eta: float, b: int, s: int, seed: int,
                           outer_iter: int = 0, loss=0, rel_budget: float = 1e-6,
                           allowed: int = 0, stream=None) -> dict:
    """Thm. 5.1 evaluated on one sampled outer iteration (X: the FP32 master copy)
    and the cheapest (storage, correction precision) within rel_budget.
    Returns the report as a dict (slot terms keyed by name)."""
    ws = workspace(int(_L().casgd_precision_workspace_size(X.ref(), b, s)))
    rep = _lib.PrecisionReport()
    _check(_L().casgd_select_precision(X.ref(), _ptr(y), _ptr(x), eta, b, s, seed, outer_iter,
                                       _loss_code(loss), rel_budget, allowed, ctypes.byref(rep),
                                       _ptr(ws), ws.numel(), _stream(stream)))
    names = _lib.SLOT_NAMES
    cands = []
    for i in range(rep.ncand):
        c = rep.cand[i]
        cands.append(dict(dtype=c.dtype, recur_prec=c.recur_prec, valid=bool(c.valid),
                          u=dict(zip(names, list(c.u))), E=dict(zip(names, list(c.E))),
                          sum=c.sum, Omega=c.Omega, bound=c.bound, rel_bound=c.rel_bound))
    return dict(alpha=rep.alpha, norm_Y=rep.norm_Y, K_s=rep.K_s, norm_HL=rep.norm_HL,
                T_g=rep.T_g, T_r=rep.T_r, T_G=rep.T_G, T_c=rep.T_c,
                norm_x_next=rep.norm_x_next, L_sigma=rep.L_sigma, D_delta=rep.D_delta,
                coef=dict(zip(names, list(rep.coef))), candidates=cands, chosen=rep.chosen,
                dtype=rep.dtype, recur_prec=rep.recur_prec,
                meets_budget=bool(rep.meets_budget))


def casgd_colstats(X: MatrixRef, stream=None):
    torch = _torch()
    stats = torch.empty(X.n, 4, dtype=torch.float32, device="cuda")
    need = int(_L().casgd_colstats_workspace_size(X.ref()))
    ws = workspace(need)
    _check(_L().casgd_colstats(X.ref(), _ptr(stats), _ptr(ws), ws.numel(), _stream(stream)))
    return stats
