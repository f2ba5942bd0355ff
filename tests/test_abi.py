"""The C ABI library loads and exports every entry point include/bamg.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("bamg.h", "bamg_selftest.h")]
LIB = os.path.join(ROOT, "paper_2007_01941_amd", "libbamg.so")


def declared():
    src = "".join(open(h).read() for h in HEADERS)
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
    assert _lib.LIB.ba_status_str(-6) == b"BA_ERR_WORKSPACE"
    h = ctypes.c_void_p()
    st = _lib.LIB.ba_plan_create(0, 0, 0, None, None, ctypes.byref(o), None, None, None, None,
                                 ctypes.byref(h))
    assert st == -1 and b"n_cam" in _lib.LIB.ba_last_error()
    # one allocation callback without the other is refused before any device call
    cb = _lib.ALLOC_FN(lambda n, ctx: None)
    st = _lib.LIB.ba_plan_create(4, 4, 8, ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.byref(o), cb, None,
                                 None, None, ctypes.byref(h))
    assert st == -1 and b"callbacks" in _lib.LIB.ba_last_error()
    # the workspace size of no plan is 0, with a message
    assert _lib.LIB.ba_workspace_bytes(None, ctypes.byref(o), 0) == 0
    assert b"plan" in _lib.LIB.ba_last_error()


def _c_layout(tmp_path, types):
    """sizeof and field offsets of header structs, from a C compiler."""
    import subprocess
    src = tmp_path / "layout.c"
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bamg.h"', "int main(void) {"]
    for t, fields in types.items():
        lines.append(f'  printf("{t} %zu\\n", sizeof({t}));')
        for f in fields:
            lines.append(f'  printf("{t}.{f} %zu\\n", offsetof({t}, {f}));')
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {k: int(v) for k, v in (l.split() for l in out.splitlines())}


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbamg.so not built")
def test_binding_structs_match_header(tmp_path):
    from paper_2007_01941_amd import _lib
    pairs = {"ba_opts": _lib._Opts, "ba_stats": _lib._Stats, "ba_lm_opts": _lib._LMOpts,
             "ba_lm_iter": _lib._LMIter, "ba_lm_summary": _lib._LMSummary}
    rename = {"lam": "lambda"}
    types = {t: [rename.get(f[0], f[0]) for f in py._fields_] for t, py in pairs.items()}
    c = _c_layout(tmp_path, types)
    for t, py in pairs.items():
        assert c[t] == ctypes.sizeof(py), t
        for f in py._fields_:
            assert c[f"{t}.{rename.get(f[0], f[0])}"] == getattr(py, f[0]).offset, (t, f[0])


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbamg.so not built")
def test_lm_host_side_without_gpu():
    from paper_2007_01941_amd import _lib
    lo = _lib._LMOpts()
    assert _lib.LIB.ba_lm_opts_default(ctypes.byref(lo)) == 0
    assert lo.max_iters == 100 and lo.radius0 == 1e4 and lo.min_relative_decrease == 1e-3
    py = _lib.LMOptions().to_c()
    for f, _ in _lib._LMOpts._fields_:
        if f.startswith("reserved"):
            continue
        assert getattr(py, f) == getattr(lo, f), f
    o = _lib._Opts()
    _lib.LIB.ba_opts_default(ctypes.byref(o))
    assert o.stop_rule == _lib.STOP_RESIDUAL and o.forcing == _lib.Options().forcing
    # null plan: rejected before any device work
    assert _lib.LIB.ba_lm_solve(None, ctypes.byref(o), ctypes.byref(lo), None, None, None, None, 0, None, None,
                                None) == -1
    assert _lib.LIB.ba_cost(None, None, None, None, None, None, 0, None, None, None) == -1
    assert o.loss == _lib.LOSS_SQUARED and o.loss_scale == _lib.Options().loss_scale == 1.0


def test_build_entry_does_not_load_the_library_first():
    """build() must work on a tree without libbamg.so: neither importing the
    entry module nor loading the build script imports the package (which loads
    the library)."""
    import subprocess
    import sys
    code = ("import sys, os, importlib.util\n"
            "import __graft_entry__\n"
            "spec = importlib.util.spec_from_file_location('_b', os.path.join('paper_2007_01941_amd', 'build.py'))\n"
            "m = importlib.util.module_from_spec(spec); spec.loader.exec_module(m)\n"
            "assert hasattr(m, 'build')\n"
            "assert 'paper_2007_01941_amd' not in sys.modules, 'package imported'\n")
    p = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert p.returncode == 0, p.stderr
