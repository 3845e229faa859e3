"""The C-ABI library loads and exports every entry point declared in
include/tdp.h (no device calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "tdp.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tdp_[A-Za-z0-9_]+)\s*\(", txt)))


def test_header_declares_core_entry_points():
    syms = declared_symbols()
    for s in ["tdp_op_create", "tdp_op_destroy", "tdp_precond_apply", "tdp_gmres_solve",
              "tdp_apply_H", "tdp_grad_m", "tdp_last_error"]:
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2006_16861_amd import tdp
    if not os.path.exists(tdp.LIB_PATH):
        pytest.fail("libtdp.so is not built (run python -m paper_2006_16861_amd.build)")
    lib = ctypes.CDLL(tdp.LIB_PATH)
    for s in declared_symbols():
        assert hasattr(lib, s), f"{s} declared in include/tdp.h but not exported"
    for s in tdp.SYMBOLS:
        assert s in declared_symbols()


def test_last_error_callable_without_device():
    from paper_2006_16861_amd import tdp
    assert tdp.last_error() == ""


def test_create_rejects_bad_arguments_before_touching_device():
    from paper_2006_16861_amd import tdp
    L = tdp.load()
    d = tdp.OpDesc()
    d.ndim = 4
    h = ctypes.c_void_p()
    assert L.tdp_op_create(ctypes.byref(d), ctypes.byref(h)) == tdp.EINVAL
    assert "ndim" in tdp.last_error()
    d.ndim = 2
    d.n[0] = d.n[1] = 8
    d.h = -1.0
    assert L.tdp_op_create(ctypes.byref(d), ctypes.byref(h)) == tdp.EINVAL
    assert L.tdp_op_destroy(None) == tdp.OK
