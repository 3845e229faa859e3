"""ctypes binding of libtdp (include/tdp.h): argument marshalling only.

Every array is a torch tensor on the GPU; the binding passes its data pointer
and the current torch stream to the C ABI.  There is no CPU fallback: if
libtdp.so is missing or fails to load, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtdp.so")

OK, ENOTCONV, EINVAL, ENOMEM, EHIP, ECFL = 0, 1, -1, -2, -3, -4
F64, F32 = 0, 1
# damping discretisation: "node" Im H = diag(omega R) (I_acd); "cell" Im H =
# omega sum_cells r_cell M_cell, the non-diagonal damping of Sec. 6 (I_abd)
DAMPING = {"node": 0, "cell": 1}

SYMBOLS = ("tdp_op_create", "tdp_op_destroy", "tdp_op_query", "tdp_apply_H",
           "tdp_precond_apply", "tdp_precond_apply_complex", "tdp_precond_apply_noalloc",
           "tdp_gmres_solve", "tdp_grad_m", "tdp_op_set_tuning", "tdp_op_autotune",
           "tdp_op_get_tuning", "tdp_op_force_resident_abort", "tdp_last_error",
           "tdp_batch_create", "tdp_batch_destroy",
           "tdp_batch_set_tuning", "tdp_batch_precond", "tdp_batch_solve", "tdp_batch_autotune")


# Cell tables (stiffness, mass; entry k for node pairs of a cell that differ in k
# axes, the cell form of App. A) of the discretisations the library knows by name.
#   "compact": the library default (NULL tables), the fourth-order compact scheme.
#   "fd2": the second-order scheme of Sec. 3.1 -- assembled, h^-2 times 2d on the
#          node and -1 on each axis neighbour, with a lumped (diagonal) mass; a node
#          lies in 2^d cells and an axis pair in 2^(d-1), so S = (2d/2^d, -1/2^(d-1), 0..)
#          and M = (1/2^d, 0..).
#   "q1":  bilinear / trilinear finite elements (consistent mass): every class of the
#          9- / 27-point stencil is nonzero in the mass table, so the full 27-point
#          stencil runs in 3-D.
SCHEMES = {
    "compact": {2: (None, None), 3: (None, None)},
    "fd2": {2: ((1.0, -0.5, 0.0), (0.25, 0.0, 0.0)),
            3: ((0.75, -0.25, 0.0, 0.0), (0.125, 0.0, 0.0, 0.0))},
    "q1": {2: ((2 / 3, -1 / 6, -1 / 3), (1 / 9, 1 / 18, 1 / 36)),
           3: ((1 / 3, 0.0, -1 / 12, -1 / 12), (1 / 27, 1 / 54, 1 / 108, 1 / 216))},
}


class TdpError(RuntimeError):
    def __init__(self, code, what, msg):
        super().__init__(f"{what} failed ({code}): {msg}")
        self.code = code


class OpDesc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int64 * 3), ("h", ctypes.c_double),
                ("omega", ctypes.c_double), ("c", ctypes.c_void_p), ("R", ctypes.c_void_p),
                ("stiff", ctypes.c_void_p), ("mass", ctypes.c_void_p),
                ("steps_per_period", ctypes.c_int), ("prec", ctypes.c_int),
                ("stream", ctypes.c_void_p), ("damping", ctypes.c_int)]


class OpInfo(ctypes.Structure):
    _fields_ = [("omega_c", ctypes.c_double), ("dt", ctypes.c_double),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("lam_bar", ctypes.c_double), ("n_P", ctypes.c_int), ("ndim", ctypes.c_int),
                ("N", ctypes.c_int64), ("lam_im", ctypes.c_double), ("res_aborts", ctypes.c_int)]


class GmresCfg(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int), ("max_iters", ctypes.c_int),
                ("periods_T", ctypes.c_int), ("rho", ctypes.c_double), ("tol", ctypes.c_double),
                ("x0_given", ctypes.c_int), ("fixed_iters", ctypes.c_int),
                ("variant", ctypes.c_int)]


class GmresInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int),
                ("relres_true", ctypes.c_double), ("relres_prec", ctypes.c_double),
                ("steps", ctypes.c_int64), ("ms_total", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int),
                ("history_len", ctypes.c_int), ("switched", ctypes.c_int),
                ("ms_precond", ctypes.c_double), ("ms_H", ctypes.c_double),
                ("ms_arnoldi", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int), ("tb_depth", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("tile", ctypes.c_int)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libtdp.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libtdp.so not found at {path}; run paper_2006_16861_amd.build")
    L = ctypes.CDLL(path)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.tdp_op_create.argtypes = [ctypes.POINTER(OpDesc), ctypes.POINTER(P)]
    L.tdp_op_destroy.argtypes = [P]
    L.tdp_op_query.argtypes = [P, ctypes.POINTER(OpInfo)]
    L.tdp_apply_H.argtypes = [P, P, P]
    L.tdp_precond_apply.argtypes = [P, I, D, P, P]
    L.tdp_precond_apply_complex.argtypes = [P, I, D, P, P]
    L.tdp_precond_apply_noalloc.argtypes = [P, I, D, P, P]
    L.tdp_gmres_solve.argtypes = [P, ctypes.POINTER(GmresCfg), P, P, ctypes.POINTER(GmresInfo)]
    L.tdp_grad_m.argtypes = [P, P, P, P]
    L.tdp_op_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    L.tdp_op_get_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    L.tdp_op_autotune.argtypes = [P, I, D, I, ctypes.POINTER(Tuning), P, I]
    L.tdp_batch_create.argtypes = [P, I, P, ctypes.POINTER(P)]
    L.tdp_batch_destroy.argtypes = [P]
    L.tdp_batch_set_tuning.argtypes = [P, I, I, I]
    L.tdp_batch_precond.argtypes = [P, P, D, P, P]
    L.tdp_batch_solve.argtypes = [P, ctypes.POINTER(GmresCfg), P, P, P, P]
    L.tdp_batch_autotune.argtypes = [P, P, D, P, I]
    L.tdp_op_force_resident_abort.argtypes = [P, I]
    L.tdp_last_error.restype = ctypes.c_char_p
    for name in SYMBOLS:
        L[name].restype = L[name].restype if name == "tdp_last_error" else ctypes.c_int
    _lib = L
    return L


def last_error() -> str:
    return load().tdp_last_error().decode()


def _check(rc, what):
    if rc < 0:
        raise TdpError(rc, what, last_error())
    return rc


def _stream_ptr():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, dtype, numel, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{what} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class SolveInfo:
    status: int
    iters: int
    restarts: int
    relres: float
    relres_prec: float
    steps: int
    ms_total: float
    history: list
    switched: int = 0      # 1: a rejected cycle moved the solve to the complex-linear variant
    ms_precond: float = 0.0   # GPU time of the preconditioner applications
    ms_H: float = 0.0         # ... of the H-applies
    ms_arnoldi: float = 0.0   # ... of the Gram-Schmidt kernels


class Operator:
    """H for -Lap U - omega^2/c^2 U + i omega R U = F on an interior grid `n`
    with spacing `h` (Dirichlet walls); c and R are FP64 tensors on the GPU.
    steps_per_period: 0 the smallest multiple of 4 above the CFL bound, -1
    the smallest integer >= 3 above it, or a given n_P (checked)."""

    def __init__(self, c, R, omega, h, prec=F64, steps_per_period=0, stiff=None, mass=None,
                 scheme=None, damping="node"):
        import torch
        L = load()
        self.n = tuple(int(v) for v in c.shape)
        self.ndim = len(self.n)
        if self.ndim not in (2, 3):
            raise ValueError("c must be 2-D or 3-D")
        if scheme is not None:
            if stiff is not None or mass is not None:
                raise ValueError("give either scheme or stiff/mass tables")
            if scheme not in SCHEMES:
                raise ValueError(f"unknown scheme {scheme!r}; known: {sorted(SCHEMES)}")
            stiff, mass = SCHEMES[scheme][self.ndim]
        self.N = int(c.numel())
        desc = OpDesc()
        desc.ndim = self.ndim
        for a in range(3):
            desc.n[a] = self.n[a] if a < self.ndim else 1
        desc.h = float(h)
        desc.omega = float(omega)
        desc.c = _dev_ptr(c, torch.float64, self.N, "c")
        desc.R = None if R is None else _dev_ptr(R, torch.float64, self.N, "R")
        self._tables = []
        for name, tab in (("stiff", stiff), ("mass", mass)):
            if tab is None:
                setattr(desc, name, None)
            else:
                arr = (ctypes.c_double * (self.ndim + 1))(*[float(v) for v in tab])
                self._tables.append(arr)
                setattr(desc, name, ctypes.cast(arr, ctypes.c_void_p))
        desc.steps_per_period = int(steps_per_period)
        desc.prec = int(prec)
        if damping not in DAMPING:
            raise ValueError(f"damping must be one of {sorted(DAMPING)}")
        desc.damping = DAMPING[damping]
        self.damping = damping
        desc.stream = _stream_ptr()
        self.prec = int(prec)
        h_ = ctypes.c_void_p()
        _check(L.tdp_op_create(ctypes.byref(desc), ctypes.byref(h_)), "tdp_op_create")
        self._h = h_
        self._destroy = L.tdp_op_destroy
        info = OpInfo()
        _check(L.tdp_op_query(self._h, ctypes.byref(info)), "tdp_op_query")
        self.omega_c, self.dt, self.alpha, self.beta = info.omega_c, info.dt, info.alpha, info.beta
        self.lam_bar, self.nP = info.lam_bar, info.n_P
        self.lam_im = info.lam_im

    def close(self):
        if getattr(self, "_h", None):
            self._destroy(self._h)
            self._h = None

    __del__ = close

    def _cplx(self, t, what):
        import torch
        return _dev_ptr(t, torch.complex128, self.N, what)

    def apply_H(self, x, out=None):
        import torch
        out = torch.empty_like(x) if out is None else out
        _check(load().tdp_apply_H(self._h, self._cplx(x, "x"), self._cplx(out, "y")),
               "tdp_apply_H")
        return out

    def precond(self, F, T, rho=0.25, out=None, variant=0):
        """Table 1 (variant 0) or Definition 4 (variant 1) preconditioner."""
        import torch
        out = torch.empty_like(F) if out is None else out
        fn = load().tdp_precond_apply_complex if variant else load().tdp_precond_apply
        _check(fn(self._h, int(T), float(rho), self._cplx(F, "F"), self._cplx(out, "U")),
               "tdp_precond_apply")
        return out

    def precond_noalloc(self, F, T, rho=0.25, out=None):
        """Table 1 preconditioner through the allocation-free entry point (the
        recurrence fields live in the library's static device array)."""
        import torch
        out = torch.empty_like(F) if out is None else out
        _check(load().tdp_precond_apply_noalloc(self._h, int(T), float(rho), self._cplx(F, "F"),
                                                self._cplx(out, "U")),
               "tdp_precond_apply_noalloc")
        return out

    def solve(self, F, T, rho=0.25, tol=1e-6, restart=30, max_iters=3000, fixed_iters=0,
              x0=None, history_cap=4096, variant=0):
        import torch
        U = torch.zeros_like(F) if x0 is None else x0.clone()
        cfg = GmresCfg(int(restart), int(max_iters), int(T), float(rho), float(tol),
                       int(x0 is not None), int(fixed_iters), int(variant))
        hist = (ctypes.c_double * max(1, history_cap))()
        info = GmresInfo()
        info.history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
        info.history_cap = int(history_cap)
        rc = _check(load().tdp_gmres_solve(self._h, ctypes.byref(cfg), self._cplx(F, "F"),
                                           self._cplx(U, "U"), ctypes.byref(info)),
                    "tdp_gmres_solve")
        return U, SolveInfo(rc, info.iters, info.restarts, info.relres_true, info.relres_prec,
                            info.steps, info.ms_total, list(hist[: info.history_len]),
                            info.switched, info.ms_precond, info.ms_H, info.ms_arnoldi)

    def grad_m(self, lam, U, out=None):
        import torch
        out = torch.empty(self.n, dtype=torch.float64, device=U.device) if out is None else out
        _check(load().tdp_grad_m(self._h, self._cplx(lam, "lam"), self._cplx(U, "U"),
                                 _dev_ptr(out, torch.float64, self.N, "grad")), "tdp_grad_m")
        return out

    def set_tuning(self, kernel=0, tb_depth=0, use_graph=1, tile=0):
        t = Tuning(int(kernel), int(tb_depth), int(use_graph), int(tile))
        _check(load().tdp_op_set_tuning(self._h, ctypes.byref(t)), "tdp_op_set_tuning")

    def autotune(self, T=4, rho=0.25, variant=0):
        """Time the sweep variants and keep the fastest; returns (best, table)
        with table rows (kernel, tb_depth, tile, us_per_step)."""
        cap = 256
        tab = (ctypes.c_double * (4 * cap))()
        best = Tuning()
        n = _check(load().tdp_op_autotune(self._h, int(T), float(rho), int(variant),
                                          ctypes.byref(best), ctypes.cast(tab, ctypes.c_void_p),
                                          cap), "tdp_op_autotune")
        rows = [tuple(tab[4 * i: 4 * i + 4]) for i in range(min(n, cap))]
        return ({"kernel": best.kernel, "tb_depth": best.tb_depth, "use_graph": best.use_graph,
                 "tile": best.tile}, rows)

    def get_tuning(self):
        t = Tuning()
        _check(load().tdp_op_get_tuning(self._h, ctypes.byref(t)), "tdp_op_get_tuning")
        return {"kernel": t.kernel, "tb_depth": t.tb_depth, "use_graph": t.use_graph,
                "tile": t.tile}

    @property
    def resident_aborts(self):
        """Resident-tile launches redone with the blocked sweep."""
        info = OpInfo()
        _check(load().tdp_op_query(self._h, ctypes.byref(info)), "tdp_op_query")
        return info.res_aborts

    def force_resident_abort(self, on=True):
        """Test hook: every resident-tile launch gives up its first wait."""
        _check(load().tdp_op_force_resident_abort(self._h, int(bool(on))),
               "tdp_op_force_resident_abort")


def operator_from_problem(p, device="cuda", **kw):
    """Operator for an inputs.Problem (copies c and R to the device)."""
    import torch
    c = torch.as_tensor(p.c, dtype=torch.float64, device=device).contiguous()
    R = torch.as_tensor(p.R, dtype=torch.float64, device=device).contiguous()
    op = Operator(c, R, p.omega, p.h, **kw)
    op._keep = (c, R)
    return op


class Batch:
    """Batched form over operators `ops` with nrhs[i] right-hand sides each.
    Fields are ordered (op 0 rhs 0..), (op 1 rhs 0..), ..."""

    def __init__(self, ops, nrhs):
        L = load()
        self.ops = list(ops)
        self.nrhs = [int(v) for v in nrhs]
        arr = (ctypes.c_void_p * len(self.ops))(*[o._h.value for o in self.ops])
        nr = (ctypes.c_int * len(self.ops))(*self.nrhs)
        h_ = ctypes.c_void_p()
        _check(L.tdp_batch_create(ctypes.cast(arr, ctypes.c_void_p), len(self.ops),
                                  ctypes.cast(nr, ctypes.c_void_p), ctypes.byref(h_)),
               "tdp_batch_create")
        self._h = h_
        self._destroy = L.tdp_batch_destroy
        self.field_op = [i for i, r in enumerate(self.nrhs) for _ in range(r)]

    def close(self):
        if getattr(self, "_h", None):
            self._destroy(self._h)
            self._h = None

    __del__ = close

    def set_tuning(self, depth, tile, medium_tile=0):
        """Steps per launch, single-field tile and shared-medium tile (-1: none)."""
        _check(load().tdp_batch_set_tuning(self._h, int(depth), int(tile), int(medium_tile)),
               "tdp_batch_set_tuning")

    def autotune(self, T, rho=0.25):
        """Time the batched sweep variants, keep the fastest; returns rows
        (depth, tile, medium_tile, ms per application)."""
        cap = 128
        tab = (ctypes.c_double * (4 * cap))()
        Tv = (ctypes.c_int * len(self.ops))(*[int(t) for t in T])
        n = _check(load().tdp_batch_autotune(self._h, ctypes.cast(Tv, ctypes.c_void_p), float(rho),
                                             ctypes.cast(tab, ctypes.c_void_p), cap),
                   "tdp_batch_autotune")
        return [tuple(tab[4 * i: 4 * i + 4]) for i in range(min(n, cap))]

    def _ptrs(self, tensors, what):
        import torch
        if len(tensors) != len(self.field_op):
            raise ValueError(f"{what}: expected {len(self.field_op)} tensors")
        for t, q in zip(tensors, self.field_op):
            _dev_ptr(t, torch.complex128, self.ops[q].N, what)
        return (ctypes.c_void_p * len(tensors))(*[t.data_ptr() for t in tensors])

    def precond(self, Fs, T, rho=0.25):
        import torch
        Us = [torch.empty_like(F) for F in Fs]
        Tv = (ctypes.c_int * len(self.ops))(*[int(t) for t in T])
        _check(load().tdp_batch_precond(self._h, ctypes.cast(Tv, ctypes.c_void_p), float(rho),
                                        ctypes.cast(self._ptrs(Fs, "F"), ctypes.c_void_p),
                                        ctypes.cast(self._ptrs(Us, "U"), ctypes.c_void_p)),
               "tdp_batch_precond")
        return Us

    def solve(self, Fs, T, rho=0.25, tol=1e-6, restart=30, max_iters=3000, fixed_iters=0,
              history_cap=512):
        import torch
        Us = [torch.zeros_like(F) for F in Fs]
        Tv = (ctypes.c_int * len(self.ops))(*[int(t) for t in T])
        cfg = GmresCfg(int(restart), int(max_iters), 1, float(rho), float(tol), 0,
                       int(fixed_iters), 0)
        n = len(Fs)
        infos = (GmresInfo * n)()
        hists = [(ctypes.c_double * history_cap)() for _ in range(n)]
        for i in range(n):
            infos[i].history = ctypes.cast(hists[i], ctypes.POINTER(ctypes.c_double))
            infos[i].history_cap = history_cap
        rc = _check(load().tdp_batch_solve(self._h, ctypes.byref(cfg),
                                           ctypes.cast(Tv, ctypes.c_void_p),
                                           ctypes.cast(self._ptrs(Fs, "F"), ctypes.c_void_p),
                                           ctypes.cast(self._ptrs(Us, "U"), ctypes.c_void_p),
                                           ctypes.cast(infos, ctypes.c_void_p)),
                    "tdp_batch_solve")
        out = [SolveInfo(0 if infos[i].relres_true <= tol or fixed_iters else 1, infos[i].iters,
                         infos[i].restarts, infos[i].relres_true, infos[i].relres_prec,
                         infos[i].steps, infos[i].ms_total,
                         list(hists[i][: infos[i].history_len])) for i in range(n)]
        return Us, out, rc
