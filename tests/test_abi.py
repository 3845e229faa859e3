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


def _desc(ndim, n, **kw):
    from paper_2006_16861_amd import tdp
    d = tdp.OpDesc()
    d.ndim = ndim
    for a in range(3):
        d.n[a] = n[a] if a < len(n) else 1
    d.h, d.omega = 0.01, 10.0
    buf = (ctypes.c_double * 1)(1.0)          # never read: every check below fails first
    d.c = ctypes.cast(buf, ctypes.c_void_p)
    for k, v in kw.items():
        setattr(d, k, v)
    return d, buf


@pytest.mark.parametrize("ndim,n,msg", [
    (2, (262140, 2), "262139"),
    (3, (65535, 2, 2), "65534"),
    (3, (8, 262140, 2), "262139"),
    (2, (0, 8), "out of range"),
    (3, (8, 8, (1 << 20) + 1), "out of range"),
    (3, (4096, 4096, 1 << 20), "too large"),
])
def test_create_rejects_grids_beyond_the_launch_limits(ndim, n, msg):
    """Axis lengths the node-per-thread launch grids cannot cover, and grids
    beyond 2^36 nodes, are refused before any device call."""
    from paper_2006_16861_amd import tdp
    L = tdp.load()
    d, _keep = _desc(ndim, n)
    h = ctypes.c_void_p()
    assert L.tdp_op_create(ctypes.byref(d), ctypes.byref(h)) == tdp.EINVAL
    assert msg in tdp.last_error()


def test_create_rejects_bad_modes_and_tables():
    from paper_2006_16861_amd import tdp
    L = tdp.load()
    h = ctypes.c_void_p()
    cases = [({"prec": 5}, "prec"), ({"damping": 7}, "damping")]
    for kw, msg in cases:
        d, _keep = _desc(2, (8, 8), **kw)
        assert L.tdp_op_create(ctypes.byref(d), ctypes.byref(h)) == tdp.EINVAL, kw
        assert msg in tdp.last_error(), (kw, tdp.last_error())
    # App. A conditions on the cell tables (checked on the host)
    for stiff, mass, msg in [((-1.0, 0.0, 0.0), None, "not PSD"),
                             (None, (1.0, 0.0, 0.0), "2^-d"),
                             ((0.0, 0.0, 0.0), None, "zero"),
                             ((float("nan"), 0.0, 0.0), None, "non-finite")]:
        d, _keep = _desc(2, (8, 8))
        arrs = []
        for name, tab in (("stiff", stiff), ("mass", mass)):
            if tab is not None:
                arr = (ctypes.c_double * 3)(*tab)
                arrs.append(arr)
                setattr(d, name, ctypes.cast(arr, ctypes.c_void_p))
        assert L.tdp_op_create(ctypes.byref(d), ctypes.byref(h)) == tdp.EINVAL, msg
        assert msg in tdp.last_error(), (msg, tdp.last_error())


def _element_tables(d, order=3):
    """Stiffness and mass tables of the d-linear element on the unit cell by
    Gauss quadrature: entry k is the element-matrix value for two corners that
    differ in k axes (scaled by the cell volume, h = 1)."""
    import itertools
    import numpy as np
    x, w = np.polynomial.legendre.leggauss(order)
    x, w = (x + 1) / 2, w / 2
    corners = list(itertools.product((0, 1), repeat=d))

    def phi(c, p):
        return np.prod([p[a] if c[a] else 1 - p[a] for a in range(d)])

    def dphi(c, p, a):
        return np.prod([(1 if c[b] else -1) if b == a else (p[b] if c[b] else 1 - p[b])
                        for b in range(d)])

    S = np.zeros(d + 1)
    M = np.zeros(d + 1)
    b0 = corners[0]
    for g in corners:
        k = sum(1 for a in range(d) if g[a] != b0[a])
        s_ = m_ = 0.0
        for idx in itertools.product(range(order), repeat=d):
            p = [x[i] for i in idx]
            wt = np.prod([w[i] for i in idx])
            s_ += wt * sum(dphi(b0, p, a) * dphi(g, p, a) for a in range(d))
            m_ += wt * phi(b0, p) * phi(g, p)
        S[k], M[k] = s_, m_
    return S, M


def test_q1_scheme_is_the_linear_element():
    """The binding's "q1" preset equals the bilinear / trilinear element
    stiffness and mass matrices, computed here from the shape functions."""
    import numpy as np
    from paper_2006_16861_amd import tdp
    for d in (2, 3):
        S, M = _element_tables(d)
        s_pre, m_pre = tdp.SCHEMES["q1"][d]
        assert np.allclose(S, s_pre, atol=1e-14) and np.allclose(M, m_pre, atol=1e-14), d
