"""The C ABI library loads and exports what include/casgd.h declares, and its
host-side argument checks return the documented codes (no GPU needed: every
call here fails validation before any device work)."""
import ctypes
import os

import pytest

from paper_2606_18463_amd import _lib

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH),
                                reason="libcasgd.so not built")


def test_every_declared_symbol_is_exported():
    lib = _lib.load()
    declared = _lib.header_symbols()
    assert "casgd_fit" in declared and "casgd_step" in declared
    missing = [s for s in declared if not hasattr(lib, s)]
    assert not missing, missing
    # the binding declares exactly the header's functions
    assert sorted(_lib.SIGNATURES) == declared


def test_status_strings_and_version():
    lib = _lib.load()
    assert lib.casgd_status_string(0) == b"ok"
    assert lib.casgd_status_string(-3) == b"workspace too small"
    assert lib.casgd_version() >= 100


def _dense(m=100, n=64, ld=64, dtype=_lib.F32, values=0x1000, scale=None):
    return _lib.Matrix(m=m, n=n, ld=ld, dtype=dtype, layout=_lib.DENSE, values=values,
                       row_scale=scale, row_ptr=None, col_idx=None, nnz=0)


def test_workspace_size_and_validation():
    lib = _lib.load()
    out = ctypes.c_size_t(0)
    X = _dense()
    assert lib.casgd_workspace_size(ctypes.byref(X), 16, 4, ctypes.byref(out)) == 0
    small = out.value
    assert small > 0 and small % 256 == 0
    assert lib.casgd_workspace_size(ctypes.byref(X), 64, 16, ctypes.byref(out)) == 0
    assert out.value > small
    # s*b above the limit, bad b, bad shape, misalignment, FP8 without scales
    assert lib.casgd_workspace_size(ctypes.byref(X), 64, 65, ctypes.byref(out)) == -2
    assert lib.casgd_workspace_size(ctypes.byref(X), 0, 4, ctypes.byref(out)) == -1
    bad = _dense(ld=32)
    assert lib.casgd_workspace_size(ctypes.byref(bad), 16, 4, ctypes.byref(out)) == -1
    mis = _dense(values=0x1004)
    assert lib.casgd_workspace_size(ctypes.byref(mis), 16, 4, ctypes.byref(out)) == -1
    f8 = _dense(dtype=_lib.FP8E4M3)
    assert lib.casgd_workspace_size(ctypes.byref(f8), 16, 4, ctypes.byref(out)) == -1
    assert b"row_scale" in lib.casgd_last_error()


def test_fit_argument_errors_before_device_work():
    lib = _lib.load()
    X = _dense()
    need = ctypes.c_size_t(0)
    lib.casgd_workspace_size(ctypes.byref(X), 16, 4, ctypes.byref(need))
    ws = 0x100000
    # eta <= 0
    assert lib.casgd_fit(ctypes.byref(X), 0x2000, 0x3000, 0.0, 0.0, 16, 4, 1, 0, 1, None, ws,
                         need.value, None) == -1
    # negative lambda
    assert lib.casgd_fit(ctypes.byref(X), 0x2000, 0x3000, 0.5, -1.0, 16, 4, 1, 0, 1, None, ws,
                         need.value, None) == -1
    # workspace too small / misaligned
    assert lib.casgd_fit(ctypes.byref(X), 0x2000, 0x3000, 0.5, 0.0, 16, 4, 1, 0, 1, None, ws,
                         need.value - 256, None) == -3
    assert lib.casgd_fit(ctypes.byref(X), 0x2000, 0x3000, 0.5, 0.0, 16, 4, 1, 0, 1, None,
                         ws + 8, need.value, None) == -1
    # NULL labels
    assert lib.casgd_fit(ctypes.byref(X), None, 0x3000, 0.5, 0.0, 16, 4, 1, 0, 1, None, ws,
                         need.value, None) == -1
    # bad option values
    o = _lib.Opts(recur_prec=48)
    assert lib.casgd_fit(ctypes.byref(X), 0x2000, 0x3000, 0.5, 0.0, 16, 4, 1, 0, 1,
                         ctypes.byref(o), ws, need.value, None) == -1
    o = _lib.Opts(snapshot_every=5)
    assert lib.casgd_fit(ctypes.byref(X), 0x2000, 0x3000, 0.5, 0.0, 16, 4, 1, 0, 1,
                         ctypes.byref(o), ws, need.value, None) == -1
    o = _lib.Opts(loss=3)
    assert lib.casgd_fit(ctypes.byref(X), 0x2000, 0x3000, 0.5, 0.0, 16, 4, 1, 0, 1,
                         ctypes.byref(o), ws, need.value, None) == -1
    assert b"loss" in lib.casgd_last_error()


def test_other_entry_points_validate():
    lib = _lib.load()
    assert lib.casgd_sample_indices(1, 0, 10, 0, 0x1000, None) == -1
    assert lib.casgd_recurrence(None, 0x1000, 0x1000, 16, 4, 0.5, 0.0, 0, 0, 1, 0x1000, None,
                                None, 0, None) == -1
    assert lib.casgd_recurrence(0x1000, 0x1000, 0x1000, 16, 4, 0.5, 0.0, 16, 0, 1, 0x1000, None,
                                None, 0, None) == -1
    # unknown loss, unknown form, form 2 for an unsupported b, form 2 without workspace
    assert lib.casgd_recurrence(0x1000, 0x1000, 0x1000, 16, 4, 0.5, 0.0, 0, 3, 1, 0x1000, None,
                                None, 0, None) == -1
    assert lib.casgd_recurrence(0x1000, 0x1000, 0x1000, 16, 4, 0.5, 0.0, 0, 0, 3, 0x1000, None,
                                None, 0, None) == -1
    assert lib.casgd_recurrence(0x1000, 0x1000, 0x1000, 24, 4, 0.5, 0.0, 0, 0, 2, 0x1000, None,
                                None, 0, None) == -2
    assert lib.casgd_recurrence(0x1000, 0x1000, 0x1000, 16, 4, 0.5, 0.0, 0, 0, 2, 0x1000, None,
                                None, 0, None) == -1
    need = lib.casgd_recurrence_workspace_size(64, 16)
    assert need >= 736 * 4 + 64 * 16 * 32
    assert lib.casgd_recurrence(0x1000, 0x1000, 0x1000, 64, 16, 0.5, 0.0, 0, 0, 2, 0x1000, None,
                                0x100000, need - 256, None) == -3
    assert lib.casgd_recurrence_workspace_size(64, 65) == 0
    assert lib.casgd_quantize(None, 4, 4, 4, _lib.BF16, 0x1000, 8, None, None) == -1
    assert lib.casgd_quantize(0x1000, 4, 4, 4, _lib.FP8E4M3, 0x1000, 16, None, None) == -1
    X = _dense()
    assert lib.casgd_logloss(ctypes.byref(X), 0x1000, 0x1000, 2, 64, 0x1000, None, 0,
                             None) == -1
    assert lib.casgd_logloss_workspace_size(3) == 3 * 256 * 8
    # the loss selector is validated
    assert lib.casgd_loss(ctypes.byref(X), 0x1000, 0x1000, 2, 64, 5, 0x1000, 0x1000, 4096,
                          None) == -1
