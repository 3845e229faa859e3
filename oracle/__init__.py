"""Plain FP64 CPU oracle of the time-domain preconditioned Helmholtz solver.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product library.  The arithmetic
lives in ``tdpo.c`` (plain C, OpenMP over nodes); this module is a ctypes shim
plus an independent sparse assembly of H used for dense/sparse LU checks.

Stencil tables.  The paper's optimised compact-stencil coefficients come from
other publications and are not given (Sec. 3.2).  The reading used here is the
classical fourth-order compact ("Mehrstellen") scheme written in the cell form
of App. A: per cell, the coupling of corners b, g is
h^-2 S[Delta(b,g)] - omega^2 m_cell M[Delta(b,g)] with Delta the number of
axes on which b and g differ.  Assembled, this gives in 2-D the stencil
h^-2 (1/6)[20, -4, -1] - k^2 (1/12)[8, 1, 0] (centre, edge, corner), in 3-D
h^-2 (1/6)[24, -2, -1, 0] - k^2 (1/12)[6, 1, 0, 0].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtdpo.so")

# cell tables indexed by Delta = 0..d (see module docstring)
STIFF_2D = (5.0 / 6.0, -1.0 / 3.0, -1.0 / 6.0)
MASS_2D = (1.0 / 6.0, 1.0 / 24.0, 0.0)
STIFF_3D = (1.0 / 2.0, -1.0 / 12.0, -1.0 / 12.0, 0.0)
MASS_3D = (1.0 / 16.0, 1.0 / 48.0, 0.0, 0.0)

OK, ENOTCONV, EINVAL, ENOMEM, ECFL = 0, 1, -1, -2, -4


def default_tables(ndim):
    return (STIFF_2D, MASS_2D) if ndim == 2 else (STIFF_3D, MASS_3D)


def build(force: bool = False) -> str:
    """Compile tdpo.c with gcc (-O2, OpenMP) into libtdpo.so."""
    src = os.path.join(HERE, "tdpo.c")
    if force or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < max(os.path.getmtime(src),
                                            os.path.getmtime(os.path.join(HERE, "tdpo.h"))):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared",
                               "-fopenmp", "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        D = ctypes.c_double
        I = ctypes.c_int
        L.tdpo_op_create.argtypes = [I, P, D, D, P, P, P, P, I, I, ctypes.POINTER(P)]
        L.tdpo_op_destroy.argtypes = [P]
        L.tdpo_op_query.argtypes = [P, P, P]
        L.tdpo_cell_slowness.argtypes = [P, P]
        L.tdpo_apply_reH.argtypes = [P, P, P]
        L.tdpo_apply_H.argtypes = [P, P, P]
        L.tdpo_apply_K.argtypes = [P, P, P]
        L.tdpo_apply_L.argtypes = [P, P, P]
        L.tdpo_damping.argtypes = [P, P]
        L.tdpo_step.argtypes = [P, P, P, P, P]
        L.tdpo_window.argtypes = [D, D]
        L.tdpo_window.restype = D
        L.tdpo_precond_apply.argtypes = [P, I, D, P, P]
        L.tdpo_gmres_solve.argtypes = [P, I, I, I, D, D, I, I, I, P, P, P, P, I]
        L.tdpo_precond_apply_complex.argtypes = [P, I, D, P, P]
        L.tdpo_grad_m.argtypes = [P, P, P, P]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what} failed with code {code}")
        self.code = code


class Op:
    """Oracle operator for H built from c, R, omega, h on an interior grid n."""

    def __init__(self, n, h, omega, c, R=None, stiff=None, mass=None, nP=0,
                 damping="diagonal"):
        L = lib()
        self.n = tuple(int(v) for v in n)
        self.ndim = len(self.n)
        self.N = int(np.prod(self.n))
        ds, dm = default_tables(self.ndim)
        self.stiff = np.ascontiguousarray(stiff if stiff is not None else ds, dtype=np.float64)
        self.mass = np.ascontiguousarray(mass if mass is not None else dm, dtype=np.float64)
        self.h, self.omega = float(h), float(omega)
        self._c = np.ascontiguousarray(c, dtype=np.float64).reshape(-1)
        self._R = None if R is None else np.ascontiguousarray(R, dtype=np.float64).reshape(-1)
        nn = np.array(self.n, dtype=np.int64)
        self._nn = nn
        if damping not in ("diagonal", "cell"):
            raise ValueError("damping must be 'diagonal' or 'cell'")
        self.damping_form = damping
        h_ = ctypes.c_void_p()
        rc = L.tdpo_op_create(self.ndim, _ptr(nn), self.h, self.omega, _ptr(self._c),
                              None if self._R is None else _ptr(self._R), _ptr(self.stiff),
                              _ptr(self.mass), int(nP), 0 if damping == "diagonal" else 1,
                              ctypes.byref(h_))
        if rc != OK:
            raise OracleError(rc, "tdpo_op_create")
        self._h = h_
        vals = np.zeros(5)
        nPv = ctypes.c_int()
        L.tdpo_op_query(self._h, _ptr(vals), ctypes.byref(nPv))
        self.omega_c, self.dt, self.alpha, self.beta, self.lam_bar = (float(v) for v in vals)
        self.nP = nPv.value

    @classmethod
    def from_problem(cls, p, **kw):
        return cls(p.n, p.h, p.omega, p.c, p.R, **kw)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().tdpo_op_destroy(self._h)
            self._h = None

    # --- operators ---
    def cell_slowness(self):
        m = np.zeros(tuple(v + 1 for v in self.n))
        lib().tdpo_cell_slowness(self._h, _ptr(m))
        return m

    def apply_reH(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(self.n)
        y = np.empty_like(x)
        lib().tdpo_apply_reH(self._h, _ptr(x), _ptr(y))
        return y

    def apply_H(self, x):
        x = np.ascontiguousarray(x, dtype=np.complex128).reshape(self.n)
        y = np.empty_like(x)
        lib().tdpo_apply_H(self._h, _ptr(x), _ptr(y))
        return y

    def apply_K(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(self.n)
        y = np.empty_like(x)
        lib().tdpo_apply_K(self._h, _ptr(x), _ptr(y))
        return y

    def apply_L(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(self.n)
        y = np.empty_like(x)
        lib().tdpo_apply_L(self._h, _ptr(x), _ptr(y))
        return y

    def damping(self):
        l = np.empty(self.n)
        lib().tdpo_damping(self._h, _ptr(l))
        return l

    def step(self, u, um, f=None):
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.n)
        um = np.ascontiguousarray(um, dtype=np.float64).reshape(self.n)
        up = np.empty_like(u)
        fp = None
        if f is not None:
            f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.n)
            fp = _ptr(f)
        lib().tdpo_step(self._h, _ptr(u), _ptr(um), fp, _ptr(up))
        return up

    def precond(self, F, T, rho=0.25, variant=0):
        F = np.ascontiguousarray(F, dtype=np.complex128).reshape(self.n)
        U = np.empty_like(F)
        fn = lib().tdpo_precond_apply_complex if variant else lib().tdpo_precond_apply
        rc = fn(self._h, int(T), float(rho), _ptr(F), _ptr(U))
        if rc != OK:
            raise OracleError(rc, "tdpo_precond_apply")
        return U

    def gmres(self, F, T, rho=0.25, tol=1e-6, restart=30, max_iters=3000, fixed_iters=0,
              x0=None, history_cap=4096, variant=0):
        F = np.ascontiguousarray(F, dtype=np.complex128).reshape(self.n)
        U = np.zeros_like(F) if x0 is None else np.ascontiguousarray(x0, dtype=np.complex128).reshape(self.n).copy()
        info = np.zeros(7)
        hist = np.zeros(history_cap)
        rc = lib().tdpo_gmres_solve(self._h, int(restart), int(max_iters), int(T), float(rho),
                                    float(tol), int(fixed_iters), int(x0 is not None),
                                    int(variant), _ptr(F), _ptr(U), _ptr(info), _ptr(hist),
                                    int(history_cap))
        if rc < 0:
            raise OracleError(rc, "tdpo_gmres_solve")
        res = {"status": rc, "iters": int(info[0]), "restarts": int(info[1]),
               "relres": float(info[2]), "relres_prec": float(info[3]),
               "history": hist[: int(info[4])].copy(), "applications": int(info[5]),
               "switched": int(info[6])}
        return U, res

    def grad_m(self, lam, U):
        lam = np.ascontiguousarray(lam, dtype=np.complex128).reshape(self.n)
        U = np.ascontiguousarray(U, dtype=np.complex128).reshape(self.n)
        g = np.empty(self.n)
        lib().tdpo_grad_m(self._h, _ptr(lam), _ptr(U), _ptr(g))
        return g


def window(s, rho):
    return lib().tdpo_window(float(s), float(rho))


def assemble_H(n, h, omega, c, R=None, stiff=None, mass=None, damping="diagonal"):
    """Independent sparse assembly of H (scipy CSR), element by element.

    Each cell (lower corner alpha, alpha_a in -1..n_a-1) adds the (2^d x 2^d)
    element matrix h^-2 S[Delta] - omega^2 m_cell M[Delta] over its interior
    corners (App. A); Im H = diag(omega R), or with damping="cell" the element
    matrices i omega r_cell M[Delta], r_cell the corner mean of R (Sec. 6)."""
    import itertools
    import scipy.sparse as sp
    n = tuple(int(v) for v in n)
    d = len(n)
    ds, dm = default_tables(d)
    S = np.asarray(stiff if stiff is not None else ds, dtype=np.float64)
    M = np.asarray(mass if mass is not None else dm, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64).reshape(n)
    slow = 1.0 / c ** 2
    # cell slowness: mean of corner slowness with indices clamped into the box
    padded = np.pad(slow, 1, mode="edge")
    m = np.zeros(tuple(v + 1 for v in n))
    corners = list(itertools.product((0, 1), repeat=d))
    for e in corners:
        sl = tuple(slice(e[a], e[a] + n[a] + 1) for a in range(d))
        m += padded[sl]
    m /= len(corners)
    r = np.zeros_like(m)
    if damping == "cell" and R is not None:
        padr = np.pad(np.asarray(R, dtype=np.float64).reshape(n), 1, mode="edge")
        for e in corners:
            r += padr[tuple(slice(e[a], e[a] + n[a] + 1) for a in range(d))]
        r /= len(corners)
    N = int(np.prod(n))
    idx = np.arange(N).reshape(n)
    pidx = np.pad(idx, 1, mode="constant", constant_values=-1)
    rows, cols, vals = [], [], []
    for eb in corners:
        for eg in corners:
            s = sum(int(eb[a] != eg[a]) for a in range(d))
            coef = S[s] / h ** 2 - omega ** 2 * m * M[s] + 1j * omega * r * M[s]
            bi = pidx[tuple(slice(eb[a], eb[a] + n[a] + 1) for a in range(d))]
            gi = pidx[tuple(slice(eg[a], eg[a] + n[a] + 1) for a in range(d))]
            ok = (bi >= 0) & (gi >= 0)
            rows.append(bi[ok])
            cols.append(gi[ok])
            vals.append(coef[ok])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals).astype(np.complex128)
    H = sp.coo_matrix((vals, (rows, cols)), shape=(N, N)).tocsr()
    if R is not None and damping == "diagonal":
        H = H + sp.diags(1j * omega * np.asarray(R, dtype=np.float64).reshape(-1))
    return H.tocsr()
