"""GPU parity: the HIP library (through the C ABI) against the CPU oracle on
the same seeded inputs.  FP64 bar: relative L2 error <= 1e-10."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2006_16861_amd import inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    return torch


def note(msg):
    print(f"[case] {msg}", file=sys.stderr, flush=True)


def dev(a, dtype=None):
    torch = _torch()
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def make_ops(p, prec=0, **kw):
    from paper_2006_16861_amd import tdp
    return tdp.operator_from_problem(p, prec=prec, **kw), oracle.Op.from_problem(p)


CASES = [
    ("const2d-64", lambda: inputs.const2d()),
    ("rand2d-37x150", lambda: inputs.random_medium((37, 150), seed=1, width=4)),
    ("rand2d-1x9", lambda: inputs.random_medium((1, 9), seed=2, width=0)),
    ("rand3d-9x11x70", lambda: inputs.random_medium((9, 11, 70), seed=3, width=2)),
    ("rand3d-3x1x5", lambda: inputs.random_medium((3, 1, 5), seed=4, width=0)),
]


@pytest.mark.parametrize("name,mk", CASES)
def test_parameters_match(name, mk):
    p = mk()
    note(f"params {name}")
    g, o = make_ops(p)
    assert g.nP == o.nP
    for a, b in [(g.omega_c, o.omega_c), (g.dt, o.dt), (g.alpha, o.alpha), (g.beta, o.beta),
                 (g.lam_bar, o.lam_bar)]:
        assert abs(a - b) <= 1e-13 * abs(b)


@pytest.mark.parametrize("name,mk", CASES)
def test_apply_H(name, mk):
    p = mk()
    note(f"apply_H {name}")
    g, o = make_ops(p)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
    y = host(g.apply_H(dev(x)))
    assert rel(y, o.apply_H(x)) <= 1e-13


@pytest.mark.parametrize("graph", [0, 1])
@pytest.mark.parametrize("name,mk", CASES)
def test_precond_f64(name, mk, graph):
    p = mk()
    note(f"precond f64 {name} graph={graph}")
    g, o = make_ops(p)
    g.set_tuning(kernel=1, use_graph=graph)
    T = min(p.periods, 4)
    U = host(g.precond(dev(p.F), T, 0.25))
    err = rel(U, o.precond(p.F, T, 0.25))
    note(f"  rel err {err:.3e}")
    assert err <= TOL64


def test_precond_rho_variants():
    p = inputs.random_medium((20, 33), seed=9, width=3)
    g, o = make_ops(p)
    for rho in [0.0, 0.1, 0.5, 1.0]:
        note(f"precond rho={rho}")
        U = host(g.precond(dev(p.F), 3, rho))
        assert rel(U, o.precond(p.F, 3, rho)) <= TOL64


def test_gmres_fixed_iterations_match_oracle():
    p = inputs.const2d()
    note("gmres fixed 12 its, restart 5, const2d-64")
    g, o = make_ops(p)
    Ug, ig = g.solve(dev(p.F), T=p.periods, restart=5, fixed_iters=12)
    Uo, io = o.gmres(p.F, T=p.periods, restart=5, fixed_iters=12)
    assert ig.iters == io["iters"] == 12 and ig.restarts == io["restarts"]
    assert rel(host(Ug), Uo) <= TOL64
    assert np.allclose(ig.history, io["history"], rtol=1e-8, atol=0)


@pytest.mark.parametrize("name,mk", [CASES[0], CASES[1], CASES[3]])
def test_gmres_converges_like_oracle(name, mk):
    p = mk()
    note(f"gmres tol 1e-6 {name}")
    g, o = make_ops(p)
    T = p.periods
    Ug, ig = g.solve(dev(p.F), T=T, tol=1e-6)
    Uo, io = o.gmres(p.F, T=T, tol=1e-6)
    assert ig.status == 0 and ig.relres <= 1e-6
    U = host(Ug)
    # true residual recomputed with the oracle's H
    r = rel(o.apply_H(U), p.F)
    assert r <= 1e-6 * (1 + 1e-9)
    if ig.iters == io["iters"]:
        assert rel(U, Uo) <= TOL64
    else:   # the stop can flip at the threshold: both are then valid iterates
        note(f"  iteration counts differ: gpu {ig.iters} oracle {io['iters']}")
        assert rel(U, Uo) <= 1e-4


def test_grad_matches_oracle():
    p = inputs.random_medium((6, 7, 9), seed=12, width=1)
    note("grad_m 6x7x9")
    g, o = make_ops(p)
    rng = np.random.default_rng(1)
    lam = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
    U = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
    gr = host(g.grad_m(dev(lam), dev(U)))
    assert rel(gr, o.grad_m(lam, U)) <= 1e-13
    p = inputs.random_medium((13, 1), seed=13, width=0)
    g, o = make_ops(p)
    lam = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
    U = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
    assert rel(host(g.grad_m(dev(lam), dev(U))), o.grad_m(lam, U)) <= 1e-13


def test_zero_rhs_and_errors():
    from paper_2006_16861_amd import tdp
    torch = _torch()
    p = inputs.const2d(n=16, width=3)
    note("zero rhs / error paths")
    g, _ = make_ops(p)
    U, info = g.solve(torch.zeros(p.n, dtype=torch.complex128, device="cuda"), T=2)
    assert info.status == 0 and not host(U).any()
    c = dev(p.c.copy())
    c[3, 3] = -1.0
    with pytest.raises(tdp.TdpError) as ei:
        tdp.Operator(c, dev(p.R), p.omega, p.h)
    assert ei.value.code == tdp.EINVAL
    with pytest.raises(tdp.TdpError) as ei:
        tdp.Operator(dev(p.c), dev(p.R), p.omega, p.h, steps_per_period=4)
    assert ei.value.code == tdp.ECFL
    with pytest.raises(tdp.TdpError):
        g.precond(dev(p.F), 0)
    with pytest.raises(tdp.TdpError) as ei:          # N_s beyond 2^24
        g.precond(dev(p.F), (1 << 24) // g.nP + 1)
    assert ei.value.code == tdp.EINVAL and "2^24" in str(ei.value)
    _, info = g.solve(dev(p.F), T=1, tol=1e-12, max_iters=1)
    assert info.status == tdp.ENOTCONV and info.iters == 1
    Fbad = p.F.copy()
    Fbad[4, 5] = np.nan
    with pytest.raises(tdp.TdpError) as ei:        # refused at once, not iterated
        g.solve(dev(Fbad), T=2, tol=1e-6)
    assert ei.value.code == tdp.EINVAL and "NaN" in str(ei.value)
    U0 = np.zeros(p.n, complex)
    U0[2, 2] = np.inf
    with pytest.raises(tdp.TdpError) as ei:
        g.solve(dev(p.F), T=2, tol=1e-6, x0=dev(U0))
    assert ei.value.code == tdp.EINVAL
    # complex arrays 8 bytes off a 16-byte boundary are refused before any
    # work (the kernels move complex128 values as 16-byte vectors)
    import ctypes
    L = tdp.load()
    buf = torch.zeros(2 * g.N + 2, dtype=torch.float64, device="cuda")
    out = torch.zeros(p.n, dtype=torch.complex128, device="cuda")
    odd = ctypes.c_void_p(buf.data_ptr() + 8)
    good = ctypes.c_void_p(out.data_ptr())
    assert L.tdp_precond_apply(g._h, 2, ctypes.c_double(0.25), odd, good) == tdp.EINVAL
    assert L.tdp_apply_H(g._h, good, odd) == tdp.EINVAL
    assert "16-byte" in tdp.last_error()
    assert not out.abs().sum().item()


def test_precond_f32_close_to_oracle():
    p = inputs.const2d()
    note("precond f32 const2d-64")
    g, o = make_ops(p, prec=1)
    U = host(g.precond(dev(p.F), p.periods, 0.25))
    err = rel(U, o.precond(p.F, p.periods, 0.25))
    note(f"  f32 rel err {err:.3e}")
    assert err <= 1e-4


def test_gmres_f32_reaches_tolerance():
    p = inputs.random_medium((40, 52), seed=14, width=4)
    note("gmres f32 40x52")
    g, o = make_ops(p, prec=1)
    Ug, ig = g.solve(dev(p.F), T=p.periods, tol=1e-6)
    assert ig.status == 0
    U = host(Ug)
    assert rel(o.apply_H(U), p.F) <= 1e-6 * (1 + 1e-9)
    Uo, _ = o.gmres(p.F, T=p.periods, tol=1e-10)
    note(f"  f32-path error vs oracle(1e-10): {rel(U, Uo):.3e}")
    assert rel(U, Uo) <= 1e-3


# ---------------------------------------------------------------- Definition 4 variant
@pytest.mark.parametrize("name,mk", [CASES[0], CASES[1], CASES[3], CASES[4]])
def test_precond_complex_variant(name, mk):
    """Definition 4 as one complex pass (kernel 1) and as two real passes of
    the blocked (2-D) or streamed (3-D) kernels, against the oracle's complex
    recurrence."""
    from paper_2006_16861_amd import tdp
    p = mk()
    note(f"precond complex variant {name}")
    g, o = make_ops(p)
    T = min(p.periods, 4)
    Uo = o.precond(p.F, T, 0.25, variant=1)
    kernels = [(1, 0, 0), (0, 0, 0)] + ([(2, 8, 5), (2, 4, 1), (2, 3, 7), (2, 8, 9), (2, 8, 14)]
                                        if len(p.n) == 2 else
                                        [(3, 8, 0), (3, 16, 2), (4, 7, 1)])
    for kern, depth, tile in kernels:
        for graph in (0, 1):
            g.set_tuning(kernel=kern, tb_depth=depth, tile=tile, use_graph=graph)
            U = host(g.precond(dev(p.F), T, 0.25, variant=1))
            assert rel(U, Uo) <= TOL64, (kern, depth, tile, graph)
    g32 = tdp.operator_from_problem(p, prec=tdp.F32)
    assert rel(host(g32.precond(dev(p.F), T, 0.25, variant=1)), Uo) <= 1e-4


def test_gmres_complex_variant_fixed_and_converged():
    p = inputs.random_medium((30, 41), seed=15, width=3)
    note("gmres complex variant 30x41")
    g, o = make_ops(p)
    Ug, ig = g.solve(dev(p.F), T=p.periods, restart=4, fixed_iters=9, variant=1)
    Uo, io = o.gmres(p.F, T=p.periods, restart=4, fixed_iters=9, variant=1)
    assert rel(host(Ug), Uo) <= TOL64
    Ug, ig = g.solve(dev(p.F), T=p.periods, tol=1e-8, variant=1)
    Uo, io = o.gmres(p.F, T=p.periods, tol=1e-8, variant=1)
    assert ig.status == 0 and rel(o.apply_H(host(Ug)), p.F) <= 1e-8 * (1 + 1e-9)
    assert ig.iters == io["iters"] and rel(host(Ug), Uo) <= TOL64


def test_gmres_applications_match_oracle():
    """Same stopping and restart decisions: same iteration / application counts."""
    p = inputs.smooth2d(96, width=8)
    note("gmres application count smooth2d-96")
    g, o = make_ops(p)
    Ug, ig = g.solve(dev(p.F), T=p.periods, tol=1e-6)
    Uo, io = o.gmres(p.F, T=p.periods, tol=1e-6)
    assert ig.iters == io["iters"] and ig.restarts == io["restarts"]
    assert ig.steps == io["applications"] * p.periods * o.nP
    assert rel(host(Ug), Uo) <= TOL64


# ---------------------------------------------------------------- full-size workloads
def test_full_size_2d_one_period_and_H():
    """1024^2 smooth medium (the benchmark workload): one period of the
    recurrence over every tile and the ragged edges, in the configuration the
    autotuner picks for the benchmark and in the blocked depth-8 32 x 64 tile it
    has picked on every run so far, and the H-apply, against the oracle."""
    p = inputs.smooth2d(1024)
    note("full-size smooth2d-1024: P F with T=1, H-apply")
    g, o = make_ops(p)
    F = dev(p.F)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
    assert rel(host(g.apply_H(dev(x))), o.apply_H(x)) <= 1e-13
    UoF, Uox = o.precond(p.F, 1, 0.25), o.precond(x, 1, 0.25)
    best, _ = g.autotune(T=4)
    note(f"  autotuned {best}")
    for tun in (best, {"kernel": 2, "tb_depth": 8, "tile": 5, "use_graph": 1}):
        g.set_tuning(**tun)
        assert rel(host(g.precond(F, 1, 0.25)), UoF) <= TOL64, tun
        assert rel(host(g.precond(dev(x), 1, 0.25)), Uox) <= TOL64, tun


def test_full_size_2d_solve_residual_checked_by_oracle():
    p = inputs.smooth2d(1024)
    note("full-size smooth2d-1024 solve to 1e-6")
    g, o = make_ops(p)
    Ug, ig = g.solve(dev(p.F), T=p.periods, tol=1e-6)
    assert ig.status == 0
    r = rel(o.apply_H(host(Ug)), p.F)
    note(f"  iters {ig.iters} restarts {ig.restarts} oracle-checked relres {r:.3e}")
    assert r <= 1e-6 * (1 + 1e-9)


def test_full_size_3d_one_period():
    p = inputs.layered3d(256)
    note("full-size layered3d-256: P F with T=1, H-apply")
    g, o = make_ops(p)
    assert g.nP == o.nP
    F = dev(p.F)
    U = host(g.precond(F, 1, 0.25))
    Uo = o.precond(p.F, 1, 0.25)
    assert rel(U, Uo) <= TOL64
    for shape, zc in ((1, 32), (0, 64), (2, 16)):
        g.set_tuning(kernel=4, tb_depth=zc, tile=shape)
        U4 = host(g.precond(F, 1, 0.25))
        assert rel(U4, Uo) <= TOL64 and rel(U4, U) <= 1e-13
    # FP32 fields in the timed configurations (one-step chunk 32, two-step
    # 66 x 31 blocks), against the same oracle period at the FP32 bar
    from paper_2006_16861_amd import tdp
    g32 = tdp.operator_from_problem(p, prec=tdp.F32)
    for kern, zc, shape in ((3, 32, 0), (4, 8, 2)):
        g32.set_tuning(kernel=kern, tb_depth=zc, tile=shape)
        assert rel(host(g32.precond(F, 1, 0.25)), Uo) <= 1e-4, (kern, shape)
    del g32
    g.set_tuning(kernel=0)
    rng = np.random.default_rng(4)
    x = (rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n))
    assert rel(host(g.apply_H(dev(x))), o.apply_H(x)) <= 1e-13


def test_full_size_3d_f32_solve_residual_checked_by_oracle():
    """The precision form's solve (layered3d-256, FP32 fields, FP64 GMRES,
    n_P = 10, tol 1e-6): its true residual, recomputed by the oracle's FP64 H,
    meets the tolerance, and the solution agrees with the FP64 GPU solve to
    the level the tolerance allows."""
    from paper_2006_16861_amd import tdp
    p = inputs.layered3d(256)
    note("full-size layered3d-256 FP32 solve to 1e-6, residual by the oracle")
    F = dev(p.F)
    U = {}
    for prec in (tdp.F32, tdp.F64):
        g = tdp.operator_from_problem(p, prec=prec, steps_per_period=-1)
        Ug, ig = g.solve(F, T=p.periods, tol=1e-6)
        assert ig.status == 0
        U[prec] = host(Ug)
        del g, Ug
    o = oracle.Op.from_problem(p, nP=10)
    r = rel(o.apply_H(U[tdp.F32]), p.F)
    note(f"  oracle-checked relres {r:.3e}")
    assert r <= 1e-6 * (1 + 1e-9)
    assert rel(U[tdp.F32], U[tdp.F64]) <= 1e-5


def test_full_size_3d_precision_form_configuration():
    """layered3d-256 as the precision form runs it: n_P = 10 (the smallest
    integer above the CFL bound, Im U from the 2x2 solve), autotuned sweeps in
    FP64 and FP32, one period against the oracle."""
    from paper_2006_16861_amd import tdp
    p = inputs.layered3d(256)
    note("full-size layered3d-256 at n_P = 10: FP64 and FP32, autotuned")
    F = dev(p.F)
    Uo = None
    for prec, tol in ((tdp.F64, TOL64), (tdp.F32, 1e-4)):
        g = tdp.operator_from_problem(p, prec=prec, steps_per_period=-1)
        assert g.nP == 10
        if Uo is None:
            Uo = oracle.Op.from_problem(p, nP=g.nP).precond(p.F, 1, 0.25)
        best, _ = g.autotune(T=4)
        note(f"  prec {prec} autotuned {best}")
        assert rel(host(g.precond(F, 1, 0.25)), Uo) <= tol
        del g


# ---------------------------------------------------------------- temporally blocked sweep
TB_CASES = [
    ("const2d-64", lambda: inputs.const2d()),
    ("rand2d-37x150", lambda: inputs.random_medium((37, 150), seed=1, width=4)),
    ("rand2d-130x61", lambda: inputs.random_medium((130, 61), seed=17, width=5)),
    ("rand2d-1x9", lambda: inputs.random_medium((1, 9), seed=2, width=0)),
]


# deepest depth each tile is run at here (4 x depth <= its rows)
TILE_MAX_DEPTH = {3: 4, 5: 4, 7: 4, 9: 8, 10: 8, 11: 4, 14: 10, 15: 12}


@pytest.mark.parametrize("tile", [0, 1, 3, 4, 5, 6, 7, 9, 10, 11, 14, 15])
@pytest.mark.parametrize("depth", [1, 3, 4, 5, 8, 12, 16])
@pytest.mark.parametrize("name,mk", TB_CASES)
def test_precond_blocked_f64(name, mk, depth, tile):
    p = mk()
    depth = min(depth, TILE_MAX_DEPTH.get(tile, 16))
    note(f"precond blocked f64 {name} depth={depth} tile={tile}")
    g, o = make_ops(p)
    g.set_tuning(kernel=2, tb_depth=depth, tile=tile, use_graph=1)
    T = min(p.periods, 3)
    U = host(g.precond(dev(p.F), T, 0.25))
    err = rel(U, o.precond(p.F, T, 0.25))
    assert err <= TOL64, err
    g.set_tuning(kernel=1, use_graph=0)
    U1 = host(g.precond(dev(p.F), T, 0.25))
    assert rel(U, U1) <= 1e-13


@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15])
def test_precond_blocked_f32(tile):
    p = inputs.random_medium((150, 200), seed=18, width=6)
    note(f"precond blocked f32 150x200 tile={tile}")
    g, o = make_ops(p, prec=1)
    g.set_tuning(kernel=2, tb_depth=4, tile=tile)
    U = host(g.precond(dev(p.F), 3, 0.25))
    g.set_tuning(kernel=1)
    U1 = host(g.precond(dev(p.F), 3, 0.25))
    Uo = o.precond(p.F, 3, 0.25)
    assert rel(U, Uo) <= 1e-4 and rel(U1, Uo) <= 1e-4
    assert rel(U, U1) <= 1e-5


def test_gmres_blocked_full_size_matches_one_step():
    p = inputs.smooth2d(1024)
    note("gmres blocked vs one-step at 1024^2 (fixed 3 its)")
    from paper_2006_16861_amd import tdp
    g = tdp.operator_from_problem(p)
    F = dev(p.F)
    g.set_tuning(kernel=1)
    U1, _ = g.solve(F, T=p.periods, fixed_iters=3)
    g.set_tuning(kernel=2, tb_depth=4, tile=0)
    U2, _ = g.solve(F, T=p.periods, fixed_iters=3)
    assert rel(host(U2), host(U1)) <= 1e-11


def test_autotune_picks_a_variant_and_stays_exact():
    p = inputs.random_medium((200, 180), seed=19, width=6)
    note("autotune 200x180")
    g, o = make_ops(p)
    best, table = g.autotune(T=2)
    assert len(table) >= 2 and best["kernel"] in (1, 2, 5)
    assert min(r[3] for r in table) > 0
    U = host(g.precond(dev(p.F), 3, 0.25))
    assert rel(U, o.precond(p.F, 3, 0.25)) <= TOL64


# ---------------------------------------------------------------- 3-D streamed sweep, general tables
Q1_2D = ((2 / 3, -1 / 6, -1 / 3), (1 / 9, 1 / 18, 1 / 36))
Q1_3D = ((1 / 3, 0.0, -1 / 12, -1 / 12), (1 / 27, 1 / 54, 1 / 108, 1 / 216))


@pytest.mark.parametrize("kern", [3, 4])
@pytest.mark.parametrize("shape,zc", [(0, 16), (1, 7), (2, 32), (1, 64), (0, 1)])
@pytest.mark.parametrize("n", [(9, 11, 70), (17, 5, 130), (40, 23, 9), (1, 1, 3)])
def test_precond_3d_streamed_f64(n, shape, zc, kern):
    p = inputs.random_medium(n, seed=21, width=2)
    note(f"precond 3d streamed kernel {kern} {n} shape={shape} zc={zc}")
    g, o = make_ops(p)
    g.set_tuning(kernel=kern, tb_depth=zc, tile=shape)
    U = host(g.precond(dev(p.F), 2, 0.25))
    assert rel(U, o.precond(p.F, 2, 0.25)) <= TOL64
    g.set_tuning(kernel=1)
    assert rel(host(g.precond(dev(p.F), 2, 0.25)), U) <= 1e-13


def test_precond_3d_two_step_many_column_blocks():
    """The two-step sweep on a grid of 11 x 12 column blocks with ragged last
    blocks along both in-plane axes, split into runs along axis 0 (one run
    per block with shortest run 8; several with 1), every shape, FP64 and
    FP32: against the oracle and the one-step kernel."""
    p = inputs.random_medium((20, 150, 700), seed=24, width=3)
    note("precond 3d two-step 20x150x700")
    g, o = make_ops(p)
    Uo = o.precond(p.F, 2, 0.25)
    g.set_tuning(kernel=1)
    U1 = host(g.precond(dev(p.F), 2, 0.25))
    for shape in (0, 1, 2):
        for zc in (8, 1):
            g.set_tuning(kernel=4, tb_depth=zc, tile=shape)
            U = host(g.precond(dev(p.F), 2, 0.25))
            assert rel(U, Uo) <= TOL64 and rel(U, U1) <= 1e-13, (shape, zc)
    g32, _ = make_ops(p, prec=1)
    for shape in (1, 2):
        g32.set_tuning(kernel=4, tb_depth=8, tile=shape)
        assert rel(host(g32.precond(dev(p.F), 2, 0.25)), Uo) <= 1e-4, shape


@pytest.mark.parametrize("kern,shape", [(3, 1), (4, 0), (4, 1), (4, 2)])
def test_precond_3d_streamed_f32(kern, shape):
    p = inputs.random_medium((24, 30, 70), seed=22, width=3)
    note(f"precond 3d streamed f32 kernel {kern} shape {shape}")
    g, o = make_ops(p, prec=1)
    g.set_tuning(kernel=kern, tb_depth=16, tile=shape)
    U = host(g.precond(dev(p.F), 2, 0.25))
    assert rel(U, o.precond(p.F, 2, 0.25)) <= 1e-4


@pytest.mark.parametrize("ndim", [2, 3])
def test_general_cell_tables(ndim):
    """Trilinear / bilinear finite-element cell tables: every stencil class
    nonzero, so the general kernels (all 9 / 27 points, all mass classes) run."""
    from paper_2006_16861_amd import tdp
    n = (45, 77) if ndim == 2 else (11, 13, 66)
    stiff, mass = Q1_2D if ndim == 2 else Q1_3D
    p = inputs.random_medium(n, seed=23, width=2)
    note(f"general tables {ndim}-D")
    o = oracle.Op(p.n, p.h, p.omega, p.c, p.R, stiff=stiff, mass=mass)
    g = tdp.Operator(dev(p.c), dev(p.R), p.omega, p.h, stiff=stiff, mass=mass)
    assert g.nP == o.nP and abs(g.lam_bar - o.lam_bar) <= 1e-12 * o.lam_bar
    rng = np.random.default_rng(2)
    x = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
    assert rel(host(g.apply_H(dev(x))), o.apply_H(x)) <= 1e-13
    kernels = [(1, 0, 0), (2, 4, 0), (2, 3, 3), (2, 4, 4), (2, 3, 7), (2, 5, 9), (2, 3, 10),
               (2, 4, 11), (2, 6, 14)] if ndim == 2 else \
        [(1, 0, 0), (3, 16, 1), (4, 16, 1), (4, 9, 0)]
    Uo = o.precond(p.F, 2, 0.25)
    for kern, depth, tile in kernels:
        g.set_tuning(kernel=kern, tb_depth=depth, tile=tile)
        assert rel(host(g.precond(dev(p.F), 2, 0.25)), Uo) <= TOL64
    grad_l = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
    assert rel(host(g.grad_m(dev(grad_l), dev(x))), o.grad_m(grad_l, x)) <= 1e-13


# ---------------------------------------------------------------- second-order scheme (Sec. 3.1)
# the cell tables of the 5- / 7-point stencil with lumped mass, stated here
# independently of the binding's named preset
FD2_TABLES = {2: ((1.0, -0.5, 0.0), (0.25, 0.0, 0.0)),
              3: ((0.75, -0.25, 0.0, 0.0), (0.125, 0.0, 0.0, 0.0))}


@pytest.mark.parametrize("n", [(70, 131), (13, 17, 70)])
def test_fd2_scheme_every_kernel(n):
    """The binding's "fd2" scheme against the oracle with the Sec. 3.1 tables:
    parameters, H, every sweep kernel, fixed-iteration GMRES."""
    from paper_2006_16861_amd import tdp
    ndim = len(n)
    p = inputs.random_medium(n, seed=31, width=3)
    note(f"fd2 scheme {n}")
    stiff, mass = FD2_TABLES[ndim]
    o = oracle.Op(p.n, p.h, p.omega, p.c, p.R, stiff=stiff, mass=mass)
    g = tdp.Operator(dev(p.c), dev(p.R), p.omega, p.h, scheme="fd2")
    assert g.nP == o.nP and abs(g.lam_bar - o.lam_bar) <= 1e-12 * o.lam_bar
    assert abs(g.lam_bar - (4 * ndim / p.h ** 2 + g.omega_c ** 2)) <= 1e-9 * g.lam_bar
    rng = np.random.default_rng(5)
    x = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
    assert rel(host(g.apply_H(dev(x))), o.apply_H(x)) <= 1e-13
    kernels = [(1, 0, 0), (2, 8, 4), (2, 6, 5), (2, 3, 1), (2, 4, 3), (2, 8, 9), (2, 7, 10),
               (2, 8, 14), (2, 9, 15)] \
        if ndim == 2 else \
        [(1, 0, 0), (3, 16, 1), (3, 32, 2), (3, 7, 0), (4, 16, 1), (4, 32, 2), (4, 7, 0)]
    Uo = o.precond(p.F, 2, 0.25)
    for kern, depth, tile in kernels:
        g.set_tuning(kernel=kern, tb_depth=depth, tile=tile)
        assert rel(host(g.precond(dev(p.F), 2, 0.25)), Uo) <= TOL64, (kern, depth, tile)
    g.set_tuning(kernel=0)
    Ug, ig = g.solve(dev(p.F), T=p.periods, restart=6, fixed_iters=10)
    Uo, io = o.gmres(p.F, T=p.periods, restart=6, fixed_iters=10)
    assert ig.iters == io["iters"] == 10
    assert rel(host(Ug), Uo) <= TOL64


def test_fd2_solve_matches_lu_of_the_written_matrix():
    """Converged GPU solve with the "fd2" scheme on a constant medium against
    sparse LU of Sec. 3.1's matrix assembled here from its formula."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    from paper_2006_16861_amd import tdp
    n = (96, 80)
    h = 1.0 / 97
    omega = 2 * math.pi / (10 * h)
    c = np.ones(n)
    R = np.zeros(n)
    w = 12
    for a in range(2):
        i = np.arange(n[a])
        dlt = np.maximum(0, w - np.minimum(i, n[a] - 1 - i)) / w
        shp = [1, 1]
        shp[a] = n[a]
        R = np.maximum(R, 2 * omega * dlt.reshape(shp) ** 2)
    F = np.zeros(n, complex)
    F[40, 33] = 1.0
    note("fd2 solve vs LU of the written 5-point matrix")
    g = tdp.Operator(dev(c), dev(R), omega, h, scheme="fd2")
    Ug, ig = g.solve(dev(F), T=10, tol=1e-11)
    assert ig.status == 0
    N = n[0] * n[1]
    idx = np.arange(N).reshape(n)
    A = sp.lil_matrix((N, N), dtype=complex)
    for i in range(n[0]):
        for j in range(n[1]):
            b = idx[i, j]
            A[b, b] = 4 / h ** 2 - omega ** 2 + 1j * omega * R[i, j]
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                if 0 <= i + di < n[0] and 0 <= j + dj < n[1]:
                    A[b, idx[i + di, j + dj]] = -1 / h ** 2
    U = spla.spsolve(A.tocsc(), F.reshape(-1)).reshape(n)
    assert rel(host(Ug), U) <= 1e-6


@pytest.mark.parametrize("model,T", [(64, 5), (96, 5), (64, 10)])
def test_gmres_short_T_matches_oracle(model, T):
    """Short T: cycles of the real-linear Table 1 map that would raise the true
    residual are rejected and the solve continues with Definition 4; the GPU
    takes the same decisions as the oracle and converges."""
    from paper_2006_16861_amd import tdp
    p = inputs.disc2d(model, width=16)
    note(f"gmres short T disc2d-{model} T={T}")
    g, o = make_ops(p)
    Ug, ig = g.solve(dev(p.F), T=T, tol=1e-6, max_iters=600)
    Uo, io = o.gmres(p.F, T=T, tol=1e-6, max_iters=600)
    assert ig.status == io["status"] == 0
    assert ig.switched == io["switched"] == (1 if T == 5 else 0)
    assert rel(o.apply_H(host(Ug)), p.F) <= 1e-6 * (1 + 1e-9)
    if ig.iters == io["iters"]:
        assert rel(host(Ug), Uo) <= 1e-8


def test_graph_cache_beyond_its_cap():
    """More (T, rho) pairs than the per-op cache of captured loops holds: the
    cache is emptied and rebuilt, results stay identical to the oracle."""
    p = inputs.random_medium((37, 150), seed=41, width=4)
    note("graph cache: 24 captured loops on one op")
    g, o = make_ops(p)
    F = dev(p.F)
    first = host(g.precond(F, 1, 0.25))
    assert rel(first, o.precond(p.F, 1, 0.25)) <= TOL64
    for T in range(2, 14):
        for rho in (0.25, 0.5):
            U = host(g.precond(F, T, rho))
            if T in (7, 13):
                assert rel(U, o.precond(p.F, T, rho)) <= TOL64
    assert rel(host(g.precond(F, 1, 0.25)), first) <= 1e-15


@pytest.mark.parametrize("n", [(70, 131), (13, 17, 70)])
def test_general_steps_per_period_every_kernel(n):
    """n_P not a multiple of 4 (Sec. 2.3's 2x2 extraction of Im U):
    steps_per_period = -1 picks the smallest integer above the CFL bound,
    and every sweep kernel, with and without graph capture, in FP64 and FP32,
    matches the oracle run with the same n_P; so does fixed-iteration GMRES."""
    from paper_2006_16861_amd import tdp
    p = inputs.random_medium(n, seed=33, width=3)
    note(f"general n_P {n}")
    g = tdp.Operator(dev(p.c), dev(p.R), p.omega, p.h, steps_per_period=-1)
    assert g.nP % 4 != 0
    with pytest.raises(oracle.OracleError):
        oracle.Op.from_problem(p, nP=g.nP - 1)
    kernels = [(1, 0, 0), (2, 8, 4), (2, 6, 5), (2, 3, 1), (2, 8, 9), (2, 5, 11), (2, 8, 14),
               (2, 10, 15)] if len(n) == 2 else \
        [(1, 0, 0), (3, 16, 1), (3, 7, 0), (4, 16, 1), (4, 7, 2)]
    for nP in (g.nP, g.nP + 1, g.nP + 3):
        if nP % 4 == 0:
            continue
        o = oracle.Op.from_problem(p, nP=nP)
        gn = g if nP == g.nP else tdp.Operator(dev(p.c), dev(p.R), p.omega, p.h, steps_per_period=nP)
        assert gn.nP == o.nP == nP and abs(gn.dt - o.dt) <= 1e-14 * o.dt
        for T in (2, 3):
            Uo = o.precond(p.F, T, 0.25)
            for kern, depth, tile in kernels:
                for graph in (1, 0):
                    gn.set_tuning(kernel=kern, tb_depth=depth, tile=tile, use_graph=graph)
                    U = host(gn.precond(dev(p.F), T, 0.25))
                    assert rel(U, Uo) <= TOL64, (nP, T, kern, depth, tile, graph)
            gn.set_tuning(kernel=0)
            Uc = host(gn.precond(dev(p.F), T, 0.25, variant=1))
            assert rel(Uc, o.precond(p.F, T, 0.25, variant=1)) <= TOL64
    g32 = tdp.Operator(dev(p.c), dev(p.R), p.omega, p.h, steps_per_period=-1, prec=tdp.F32)
    assert g32.nP == g.nP
    o = oracle.Op.from_problem(p, nP=g.nP)
    assert rel(host(g32.precond(dev(p.F), 2, 0.25)), o.precond(p.F, 2, 0.25)) <= 1e-4
    Ug, ig = g.solve(dev(p.F), T=p.periods, restart=6, fixed_iters=10)
    Uo, io = o.gmres(p.F, T=p.periods, restart=6, fixed_iters=10)
    assert ig.iters == io["iters"] == 10
    assert rel(host(Ug), Uo) <= TOL64




@pytest.mark.parametrize("n,mode", [((40, 33), (3, 5)), ((12, 9, 17), (2, 1, 4))])
def test_gmres_complex_variant_one_iteration_on_eigenvector(n, mode):
    """Def. 4 on a sine mode of a constant medium with uniform damping: GMRES is
    exact after one iteration on the GPU as in the oracle (U = F / lambda)."""
    from paper_2006_16861_amd import tdp
    h = 1.0 / (max(n) + 1)
    omega = inputs.omega_for_ppw(1.1, h, 8.0)
    c = np.full(n, 1.1)
    R = np.full(n, 0.3 * omega)
    grids = np.meshgrid(*[np.sin(math.pi * pa * (np.arange(na) + 1) / (na + 1))
                          for na, pa in zip(n, mode)], indexing="ij")
    F = np.prod(grids, axis=0) * (0.6 - 0.8j)
    note(f"one-iteration GMRES on a sine mode {n}")
    g = tdp.Operator(dev(c), dev(R), omega, h)
    o = oracle.Op(n, h, omega, c, R)
    Ug, ig = g.solve(dev(F), T=3, tol=1e-12, variant=1)
    Uo, io = o.gmres(F, T=3, tol=1e-12, variant=1)
    assert ig.status == 0 and ig.iters == io["iters"] == 1
    assert rel(host(Ug), Uo) <= TOL64
    assert rel(o.apply_H(host(Ug)), F) <= 1e-11


@pytest.mark.parametrize("n,kernels", [
    ((262139, 2), [(1, 0, 0), (2, 8, 5), (2, 4, 4), (2, 8, 9), (2, 8, 14)]),
    ((65534, 2, 3), [(1, 0, 0), (3, 32, 1), (4, 16, 0)]),
])
def test_maximum_axis_lengths(n, kernels):
    """The longest axes the launch grids allow (2-D n[0] = 262139, 3-D
    n[0] = 65534): parameters, H, every sweep kernel and Def. 4 match the
    oracle; one more node along that axis is refused with TDP_EINVAL."""
    from paper_2006_16861_amd import tdp
    torch = _torch()
    p = inputs.random_medium(n, seed=35, width=1)
    note(f"maximum axis lengths {n}")
    g, o = make_ops(p)
    assert g.nP == o.nP and abs(g.omega_c - o.omega_c) <= 1e-14 * o.omega_c
    rng = np.random.default_rng(6)
    x = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
    assert rel(host(g.apply_H(dev(x))), o.apply_H(x)) <= 1e-13
    Uo = o.precond(p.F, 1, 0.25)
    for kern, depth, tile in kernels:
        g.set_tuning(kernel=kern, tb_depth=depth, tile=tile)
        assert rel(host(g.precond(dev(p.F), 1, 0.25)), Uo) <= TOL64, (kern, depth, tile)
    g.set_tuning(kernel=0)
    assert rel(host(g.precond(dev(p.F), 1, 0.25, variant=1)),
               o.precond(p.F, 1, 0.25, variant=1)) <= TOL64
    big = (n[0] + 1,) + n[1:]
    c = torch.ones(big, dtype=torch.float64, device="cuda")
    with pytest.raises(tdp.TdpError) as ei:
        tdp.Operator(c, None, 10.0, 1.0 / (max(big) + 1))
    assert ei.value.code == tdp.EINVAL


def test_long_loop_issued_without_capture():
    """More than 2^17 launches in one application: the loop is issued directly
    instead of being captured into a graph, and still matches the oracle."""
    p = inputs.const2d(n=16, width=3)
    g, o = make_ops(p)
    T = (1 << 17) // g.nP + 1
    note(f"long loop: T = {T}, {T * g.nP} one-step launches")
    g.set_tuning(kernel=1, use_graph=1)
    U = host(g.precond(dev(p.F), T, 0.25))
    assert rel(U, o.precond(p.F, T, 0.25)) <= TOL64


def test_two_ops_on_two_streams_from_two_threads():
    """Two operators bound to two torch streams, driven from two host threads
    at once (preconditioner and fixed-iteration GMRES): no state is shared, and
    each result matches the oracle; an error on one thread is reported on that
    thread only."""
    import threading
    from paper_2006_16861_amd import tdp
    torch = _torch()
    probs = [inputs.random_medium((37, 150), seed=51, width=4),
             inputs.random_medium((9, 11, 70), seed=52, width=2)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    ops = []
    for p, st in zip(probs, streams):
        with torch.cuda.stream(st):
            ops.append(tdp.operator_from_problem(p))
    torch.cuda.synchronize()
    note("two ops, two streams, two threads")
    out, errs = [None, None], [None, None]

    def work(k):
        try:
            with torch.cuda.stream(streams[k]):
                F = dev(probs[k].F)
                U1 = host(ops[k].precond(F, 2, 0.25))
                Ug, ig = ops[k].solve(F, T=probs[k].periods, restart=5, fixed_iters=8)
                if k == 1:
                    with pytest.raises(tdp.TdpError):
                        ops[k].precond(F, 0)
                    errs[k] = tdp.last_error()
                out[k] = (U1, host(Ug))
        except Exception as e:          # reported below on the main thread
            errs[k] = e

    th = [threading.Thread(target=work, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not isinstance(errs[0], Exception) and errs[0] is None, errs[0]
    assert isinstance(errs[1], str) and "periods_T" in errs[1], errs[1]
    for k, p in enumerate(probs):
        o = oracle.Op.from_problem(p)
        assert rel(out[k][0], o.precond(p.F, 2, 0.25)) <= TOL64
        Uo, _ = o.gmres(p.F, T=p.periods, restart=5, fixed_iters=8)
        assert rel(out[k][1], Uo) <= TOL64


def test_gmres_phase_time_and_cycle_log():
    """The report's preconditioner time is positive and below the wall time;
    with TDP_LOG=1 a solve prints one line per cycle and a summary."""
    import os
    import subprocess
    p = inputs.const2d()
    g, _ = make_ops(p)
    _, info = g.solve(dev(p.F), T=p.periods, tol=1e-8)
    assert 0.0 < info.ms_precond <= info.ms_total
    assert 0.0 < info.ms_H and 0.0 < info.ms_arnoldi
    assert info.ms_precond + info.ms_H + info.ms_arnoldi <= info.ms_total
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import torch\n"
            "from paper_2006_16861_amd import tdp, inputs\n"
            "p = inputs.const2d()\n"
            "op = tdp.operator_from_problem(p)\n"
            "U, info = op.solve(torch.as_tensor(p.F, device='cuda'), T=p.periods, tol=1e-8, restart=4)\n"
            "print(info.restarts)\n") % os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, TDP_LOG="1"))
    assert r.returncode == 0, r.stderr[-2000:]
    cycles = [l for l in r.stderr.splitlines() if l.startswith("tdp gmres: cycle")]
    assert len(cycles) == int(r.stdout.strip().splitlines()[-1]) and len(cycles) >= 2
    assert any(l.startswith("tdp gmres: done after") for l in r.stderr.splitlines())


def test_onestep_2d_beyond_the_mall():
    """The one-step 2-D sweep on a grid whose step working set exceeds the
    MALL (non-temporal streams, RY rows per thread), with ragged edges on both
    axes: one period against the oracle element-wise, FP64 and FP32."""
    from paper_2006_16861_amd import tdp
    p = inputs.random_medium((3001, 2999), seed=41, width=8)
    note("one-step 2-D 3001 x 2999 (beyond the MALL)")
    g, o = make_ops(p)
    g.set_tuning(kernel=1)
    Uo = o.precond(p.F, 1, 0.25)
    assert rel(host(g.precond(dev(p.F), 1, 0.25)), Uo) <= TOL64
    g32 = tdp.operator_from_problem(p, prec=tdp.F32)
    g32.set_tuning(kernel=1)
    assert rel(host(g32.precond(dev(p.F), 1, 0.25)), Uo) <= 1e-4
