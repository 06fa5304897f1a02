"""casgd_fit_noalloc (workspace in the library's static device array) against
casgd_fit with a caller workspace, through the C ABI (on an MI355X): two
calls in a row, the second on a smaller problem, must equal the allocating
entry point bitwise (same kernels, same launch plan); the flag status comes
back through status_out; problems above the array's size are rejected."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from workloads import dense_logreg  # noqa: E402


@pytest.fixture(scope="module")
def cg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_18463_amd as cg
    cg._lib.load()
    return cg


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _call_noalloc(cg, X, y, x, eta, lam, b, s, seed, h0, H, o, status):
    lib = cg._lib.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return lib.casgd_fit_noalloc(X.ref(), y.data_ptr(), x.data_ptr(), eta, lam, b, s, seed, h0,
                                 H, None if o is None else ctypes.byref(o),
                                 None if status is None else status.data_ptr(), stream)


@pytest.mark.parametrize("kw", [dict(), dict(exec_mode=2), dict(exec_mode=1, fused_variant=2)])
def test_noalloc_equals_workspace_fit_two_calls(cg, kw):
    cases = [(4096, 256, 64, 16, 30), (1500, 72, 16, 4, 40)]   # second call: smaller
    status = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    for i, (m, n, b, s, H) in enumerate(cases):
        p = dense_logreg(m, n, 30 + i, var=1 / n, dtype=np.float32)
        X = cg.dense_matrix(_dev(p.X))
        y = _dev(p.y)
        x_ref = torch.zeros(n, device="cuda")
        ws = cg.casgd_fit(X, y, x_ref, 0.5, 1e-4, b, s, 7, 0, H, opts=cg.opts(**kw))
        cg.casgd_check(ws)
        x = torch.zeros(n, device="cuda")
        rc = _call_noalloc(cg, X, y, x, 0.5, 1e-4, b, s, 7, 0, H, cg.opts(**kw), status)
        assert rc == 0, cg._lib.load().casgd_last_error()
        torch.cuda.synchronize()
        assert int(status[0]) == 0
        assert torch.equal(x, x_ref), (i, float((x - x_ref).abs().max()))
        # resume from the returned x: again equal to the allocating path
        rc = _call_noalloc(cg, X, y, x, 0.5, 1e-4, b, s, 7, H, 5, cg.opts(**kw), None)
        assert rc == 0
        cg.casgd_fit(X, y, x_ref, 0.5, 1e-4, b, s, 7, H, 5, opts=cg.opts(**kw), ws=ws)
        torch.cuda.synchronize()
        assert torch.equal(x, x_ref)


def test_noalloc_reports_flags_and_clears_them(cg):
    p = dense_logreg(2000, 64, 3, var=1 / 64, dtype=np.float32)
    X = cg.dense_matrix(_dev(p.X * 1e18))
    y = _dev(p.y)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    x = torch.zeros(64, device="cuda")
    assert _call_noalloc(cg, X, y, x, 1e30, 0.0, 16, 4, 1, 0, 5, None, status) == 0
    torch.cuda.synchronize()
    assert int(status[0]) == -5          # CASGD_ENONFINITE
    # the next call starts from cleared flags
    X2 = cg.dense_matrix(_dev(p.X))
    x = torch.zeros(64, device="cuda")
    assert _call_noalloc(cg, X2, y, x, 0.5, 0.0, 16, 4, 1, 0, 5, None, status) == 0
    torch.cuda.synchronize()
    assert int(status[0]) == 0


def test_noalloc_rejects_problems_above_the_array(cg):
    # 2^20 x 8192 FP32 at b = 64, s = 32 needs far more than 64 MiB; the
    # check runs on the host before any device work (X is never read)
    lib = cg._lib.load()
    big = cg._lib.Matrix(m=1 << 20, n=8192, ld=8192, dtype=cg.F32, layout=cg.DENSE,
                         values=0x1000, row_scale=None, row_ptr=None, col_idx=None, nnz=0)
    rc = lib.casgd_fit_noalloc(ctypes.byref(big), 0x1000, 0x1000, 0.5, 0.0, 64, 32, 1, 0, 1,
                               None, None, None)
    assert rc == -2
    assert b"static scratch" in lib.casgd_last_error()
