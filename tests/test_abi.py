"""The C ABI library loads and exports every entry point include/bamg.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bamg.h")
LIB = os.path.join(ROOT, "paper_2007_01941_amd", "libbamg.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ba_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared()
    assert "ba_lm_step" in names and "ba_plan_create" in names and "ba_lm_step_backward" in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbamg.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbamg.so not built")
def test_binding_lists_the_same_symbols():
    from paper_2007_01941_amd import _lib
    assert sorted(_lib.EXPORTED) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbamg.so not built")
def test_host_side_calls_without_gpu():
    from paper_2007_01941_amd import _lib
    o = _lib._Opts()
    assert _lib.LIB.ba_opts_default(ctypes.byref(o)) == 0
    assert o.agg_cap == 20 and o.cheb_degree == 2 and o.lanczos_steps == 5
    assert abs(o.cheb_lo - 0.3) < 1e-15 and abs(o.cheb_hi - 1.1) < 1e-15 and o.lam == 1e-4
    assert _lib.LIB.ba_opts_default(None) == -1
    assert _lib.LIB.ba_status_str(-2) == b"BA_ERR_INDEX"
    # argument validation happens before any device call
    h = ctypes.c_void_p()
    st = _lib.LIB.ba_plan_create(0, 0, 0, None, None, ctypes.byref(o), None, ctypes.byref(h))
    assert st == -1 and b"n_cam" in _lib.LIB.ba_last_error()
