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
