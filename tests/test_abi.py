"""The C-ABI library loads and exports every symbol include/tsk.h declares (CPU;
no compute calls)."""
import ctypes
import os
import re

import paper_1804_03859_amd.tsk as t

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tsk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tsk_[a-z0-9_]+)\s*\(", src)))


def _ensure_built():
    if not os.path.exists(t.LIB_PATH):
        from paper_1804_03859_amd import build
        build.build()


def test_header_declares_the_binding_entry_points():
    assert _declared() == sorted(t.exported_symbols())


def test_library_exports_every_declared_symbol():
    _ensure_built()
    lib = ctypes.CDLL(t.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_strings_and_invalid_handles_without_gpu():
    _ensure_built()
    lib = t.load()
    assert lib.tsk_status_str(t.TSK_EINVAL) == b"invalid argument"
    # null handles are rejected before any device work
    n = ctypes.c_int64()
    assert lib.tsk_state_dim(None, ctypes.byref(n), None, None) == t.TSK_EINVAL
    assert b"null" in lib.tsk_last_error()
    assert lib.tsk_apply(None, None, None) == t.TSK_EINVAL


def test_network_entry_points_reject_null_handles_without_gpu():
    _ensure_built()
    lib = t.load()
    n = ctypes.c_int64()
    assert lib.tsk_mlp_param_count(None, ctypes.byref(n)) == t.TSK_EINVAL
    assert lib.tsk_mlp_init(None, 0) == t.TSK_EINVAL
    assert lib.tsk_mlp_forward(None, None, 1, None) == t.TSK_EINVAL
    assert lib.tsk_mlp_train(None, None, None, 1, 1, 1e-3, None) == t.TSK_EINVAL
    assert lib.tsk_ritz_block_target(None, None, 1, None, None) == t.TSK_EINVAL
    assert lib.tsk_mlp_start(None, None, 20.0, 0.5, 0.1, 0, None, None) == t.TSK_EINVAL
    lo = (ctypes.c_double * 2)(5.0, 0.25)
    hi = (ctypes.c_double * 2)(40.0, 1.0)
    h = ctypes.c_void_p()
    # width check happens before any allocation
    assert lib.tsk_mlp_create(ctypes.byref(h), 100, lo, hi, None) == t.TSK_EINVAL
    assert b"width" in lib.tsk_last_error()
    lib.tsk_mlp_destroy(None)
