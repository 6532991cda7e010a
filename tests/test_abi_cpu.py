"""CPU checks of the C ABI: the library loads and exports every function the
header declares, and the binding's signature table matches the header."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stafem.h")
LIB = os.path.join(ROOT, "paper_2605_11673_amd", "libstafem.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sta_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_core_entry_points():
    names = declared()
    for n in ("sta_build_pattern", "sta_full_rebuild", "sta_apply_edits", "sta_values_ptr"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libstafem.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signature_table_matches_header():
    import importlib.util
    spec = importlib.util.spec_from_file_location("stafem_bind", os.path.join(ROOT, "paper_2605_11673_amd", "stafem.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    assert sorted(mod.SIGNATURES) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libstafem.so not built")
def test_build_rejects_bad_input_without_gpu_work():
    """Host-checkable argument errors return before any device call."""
    import numpy as np
    lib = ctypes.CDLL(LIB)
    lib.sta_build_pattern.restype = ctypes.c_int
    lib.sta_last_error.restype = ctypes.c_char_p
    out = ctypes.c_void_p()
    x = np.zeros((4, 3))
    t = np.array([[0, 1, 2, 2]], dtype=np.int32)  # repeated vertex
    E = np.ones(1)
    m = np.ones(1, dtype=np.uint8)
    args = lambda tt, nu=0.3: (x.ctypes.data_as(ctypes.c_void_p), ctypes.c_int64(4), tt.ctypes.data_as(ctypes.c_void_p),
                               ctypes.c_int64(1), E.ctypes.data_as(ctypes.c_void_p), ctypes.c_double(nu),
                               ctypes.c_double(1.0), ctypes.c_double(0.01), m.ctypes.data_as(ctypes.c_void_p),
                               ctypes.c_void_p(None), ctypes.byref(out))
    assert lib.sta_build_pattern(*args(t)) == -4  # STA_EDEGENERATE
    assert b"repeats" in lib.sta_last_error(None)
    t2 = np.array([[0, 1, 2, 7]], dtype=np.int32)
    assert lib.sta_build_pattern(*args(t2)) == -1  # out of range
    t3 = np.array([[0, 1, 2, 3]], dtype=np.int32)
    assert lib.sta_build_pattern(*args(t3, nu=0.5)) == -1  # nu out of range
    assert out.value is None
