"""GPU parity of the Sec. 6 path: cell damping Im H = omega sum_cells r_cell M_cell,
I_abd (Def. 6) and S_T^abd (Def. 7), through the C ABI against the oracle
(FP64 bar 1e-10), plus LU for a converged solve and the error paths."""
import sys

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from paper_2006_16861_amd import inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
Q1 = {2: ((2 / 3, -1 / 6, -1 / 3), (1 / 9, 1 / 18, 1 / 36)),
      3: ((1 / 3, 0.0, -1 / 12, -1 / 12), (1 / 27, 1 / 54, 1 / 108, 1 / 216))}


def note(msg):
    print(f"[case] {msg}", file=sys.stderr, flush=True)


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def problem(n, seed, rscale=2.0):
    p = inputs.random_medium(n, seed=seed, width=3, r_scale=rscale)
    rng = np.random.default_rng(seed + 11)
    R = p.R + rng.uniform(0.0, 0.2 * p.omega, p.n)
    return p, R


def ops(p, R, tables=None):
    from paper_2006_16861_amd import tdp
    kw = {} if tables is None else {"stiff": tables[0], "mass": tables[1]}
    g = tdp.Operator(dev(p.c), dev(R), p.omega, p.h, damping="cell", **kw)
    o = oracle.Op(p.n, p.h, p.omega, p.c, R, damping="cell", **kw)
    return g, o


CASES = [((37, 150), None), ((64, 64), None), ((1, 9), None), ((45, 77), "q1"),
         ((9, 11, 70), None), ((3, 1, 5), None), ((11, 13, 20), "q1")]


@pytest.mark.parametrize("n,tab", CASES)
def test_abd_parameters_H_and_precond(n, tab):
    p, R = problem(n, 3)
    note(f"abd {n} tables={tab}")
    g, o = ops(p, R, Q1[len(n)] if tab else None)
    assert g.nP == o.nP
    for a, b in ((g.omega_c, o.omega_c), (g.dt, o.dt), (g.alpha, o.alpha), (g.beta, o.beta),
                 (g.lam_bar, o.lam_bar)):
        assert abs(a - b) <= 1e-12 * abs(b)
    rng = np.random.default_rng(4)
    x = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
    assert rel(host(g.apply_H(dev(x))), o.apply_H(x)) <= 1e-13
    for T, rho in ((2, 0.25), (3, 0.0), (1, 0.75)):
        Uo = o.precond(p.F, T, rho, variant=1)
        assert rel(host(g.precond(dev(p.F), T, rho, variant=1)), Uo) <= TOL64
    g.set_tuning(kernel=1, use_graph=0)
    assert rel(host(g.precond(dev(p.F), 2, 0.25, variant=1)), o.precond(p.F, 2, 0.25, variant=1)) <= TOL64


def test_abd_gmres_fixed_and_converged():
    p, R = problem((40, 52), 5)
    note("abd gmres")
    g, o = ops(p, R)
    Ug, ig = g.solve(dev(p.F), T=p.periods, restart=5, fixed_iters=9)
    Uo, io = o.gmres(p.F, T=p.periods, restart=5, fixed_iters=9)
    assert ig.iters == io["iters"] == 9
    assert rel(host(Ug), Uo) <= TOL64
    H = oracle.assemble_H(p.n, p.h, p.omega, p.c, R, damping="cell")
    U = spla.spsolve(H.tocsc(), p.F.reshape(-1)).reshape(p.n)
    Ug, ig = g.solve(dev(p.F), T=p.periods, tol=1e-11)
    assert ig.status == 0
    assert rel(host(Ug), U) <= 1e-8
    assert rel(o.apply_H(host(Ug)), p.F) <= 1e-11 * (1 + 1e-9)


def test_abd_gradient_and_error_paths():
    import torch
    from paper_2006_16861_amd import tdp
    p, R = problem((30, 41), 6)
    note("abd grad + errors")
    g, o = ops(p, R)
    rng = np.random.default_rng(7)
    lam = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
    U = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
    assert rel(host(g.grad_m(dev(lam), dev(U))), o.grad_m(lam, U)) <= 1e-13
    with pytest.raises(tdp.TdpError):
        g.precond(dev(p.F), 2, 0.25, variant=0)        # Table 1 is the I_acd algorithm
    with pytest.raises(tdp.TdpError):
        tdp.Batch([g], [1])
    with pytest.raises(tdp.TdpError):                  # n_P below the I_abd bound
        tdp.Operator(dev(p.c), dev(R), p.omega, p.h, damping="cell", steps_per_period=g.nP - 4)
    ok = tdp.Operator(dev(p.c), dev(R), p.omega, p.h, damping="cell", steps_per_period=g.nP + 8)
    assert ok.nP == g.nP + 8
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", [(37, 150), (9, 11, 70)])
def test_abd_f32_fields(n):
    """FP32 recurrence fields with the cell damping (the precision form of the
    Sec. 6 path): S_T^abd close to the FP64 oracle, and GMRES, which keeps H and
    the residuals in FP64, reaches 1e-8 checked by the oracle's H."""
    from paper_2006_16861_amd import tdp
    p, R = problem(n, 8)
    note(f"abd f32 {n}")
    g = tdp.Operator(dev(p.c), dev(R), p.omega, p.h, damping="cell", prec=tdp.F32)
    o = oracle.Op(p.n, p.h, p.omega, p.c, R, damping="cell")
    assert g.nP == o.nP
    for graph in (1, 0):
        g.set_tuning(kernel=0, use_graph=graph)
        U = host(g.precond(dev(p.F), 2, 0.25, variant=1))
        assert rel(U, o.precond(p.F, 2, 0.25, variant=1)) <= 1e-4
    Ug, ig = g.solve(dev(p.F), T=p.periods, tol=1e-8)
    assert ig.status == 0
    assert rel(o.apply_H(host(Ug)), p.F) <= 1e-8 * (1 + 1e-9)


ABD_GRIDS = [(37, 150), (130, 77), (1, 9), (5, 200), (64, 64)]


@pytest.mark.parametrize("n", ABD_GRIDS)
def test_abd_blocked_tiles_and_depths(n):
    """The blocked I_abd kernel (both real parts, k steps per launch) on every
    FP64 tile shape it takes, depths 1..8 (odd, and not dividing N_s), graph
    on and off, against the oracle's S_T^abd; grids of one row, ragged, and
    spanning several tiles."""
    p, R = problem(n, 12)
    g, o = ops(p, R)
    for T, rho in ((2, 0.25), (1, 0.75)):
        Uo = o.precond(p.F, T, rho, variant=1)
        for tile in (5, 7):
            for depth in (1, 3, 8):
                for graph in (1, 0):
                    note(f"abd blocked {n} T={T} tile={tile} depth={depth} graph={graph}")
                    g.set_tuning(kernel=2, tb_depth=depth, tile=tile, use_graph=graph)
                    assert rel(host(g.precond(dev(p.F), T, rho, variant=1)), Uo) <= TOL64


def test_abd_blocked_fallbacks_and_f32_tiles():
    """Tiles the blocked I_abd kernel does not take, and mass tables with corner
    entries, run the one-step kernel (same result); FP32 fields on every FP32
    tile shape stay within FP32 accuracy of the FP64 oracle."""
    from paper_2006_16861_amd import tdp
    p, R = problem((70, 130), 13)
    g, o = ops(p, R)
    Uo = o.precond(p.F, 2, 0.25, variant=1)
    for tile in (0, 4, 6):
        note(f"abd blocked fallback tile={tile}")
        g.set_tuning(kernel=2, tb_depth=4, tile=tile, use_graph=1)
        assert rel(host(g.precond(dev(p.F), 2, 0.25, variant=1)), Uo) <= TOL64
    gq, oq = ops(p, R, Q1[2])
    note("abd blocked fallback corner mass")
    gq.set_tuning(kernel=2, tb_depth=4, tile=7, use_graph=1)
    assert rel(host(gq.precond(dev(p.F), 2, 0.25, variant=1)),
               oq.precond(p.F, 2, 0.25, variant=1)) <= TOL64
    g32 = tdp.Operator(dev(p.c), dev(R), p.omega, p.h, damping="cell", prec=tdp.F32)
    for tile in (4, 5, 6, 7):
        note(f"abd blocked f32 tile={tile}")
        g32.set_tuning(kernel=2, tb_depth=6, tile=tile, use_graph=1)
        assert rel(host(g32.precond(dev(p.F), 2, 0.25, variant=1)), Uo) <= 1e-4


def test_abd_autotune_picks_a_candidate():
    """The autotuner's table for the cell damping lists the one-step kernel and
    the blocked tiles, and the op keeps a listed candidate that still matches
    the oracle."""
    p, R = problem((96, 160), 14)
    g, o = ops(p, R)
    note("abd autotune")
    best, rows = g.autotune(T=1)
    kinds = {(int(r[0]), int(r[2])) for r in rows}
    assert (1, 0) in kinds and (2, 5) in kinds and (2, 7) in kinds
    assert (best["kernel"], best["tile"]) in kinds
    assert rel(host(g.precond(dev(p.F), 2, 0.25, variant=1)),
               o.precond(p.F, 2, 0.25, variant=1)) <= TOL64


def test_abd_blocked_degenerate_damping():
    """Degenerate cell damping: R = 0 everywhere (B vanishes, only the
    constant centre term of the damping stencil is left) and R nonzero on a
    single node; the blocked I_abd against the oracle."""
    p, R = problem((50, 90), 21)
    for name, RR in (("zero", np.zeros_like(R)), ("one node", np.where(np.arange(R.size).reshape(R.shape) == 2000, 3.0 * p.omega, 0.0))):
        g, o = ops(p, RR)
        Uo = o.precond(p.F, 2, 0.25, variant=1)
        for tile in (5, 7):
            note(f"abd blocked degenerate damping {name} tile={tile}")
            g.set_tuning(kernel=2, tb_depth=8, tile=tile)
            assert rel(host(g.precond(dev(p.F), 2, 0.25, variant=1)), Uo) <= TOL64


def test_abd_blocked_full_size_one_period():
    """The benchmarked cell-damping workload (smooth2d-1024 with the cell
    damping of Sec. 6): one period of S_T^abd on the blocked I_abd kernel
    (tile 7 and tile 5 at depth 8, and the one-step complex kernel) against
    the oracle element-wise; FP32 fields against it at the FP32 bar."""
    from paper_2006_16861_amd import tdp
    p = inputs.smooth2d(1024)
    note("abd full size 1024^2, one period")
    g = tdp.Operator(dev(p.c), dev(p.R), p.omega, p.h, damping="cell")
    o = oracle.Op(p.n, p.h, p.omega, p.c, p.R, damping="cell")
    assert g.nP == o.nP
    Uo = o.precond(p.F, 1, 0.25, variant=1)
    F = dev(p.F)
    for kern, depth, tile in ((0, 0, 0), (2, 8, 7), (2, 8, 5), (1, 0, 0)):
        g.set_tuning(kernel=kern, tb_depth=depth, tile=tile)
        err = rel(host(g.precond(F, 1, 0.25, variant=1)), Uo)
        note(f"  kernel {kern} depth {depth} tile {tile}: {err:.2e}")
        assert err <= TOL64, (kern, depth, tile)
    g32 = tdp.Operator(dev(p.c), dev(p.R), p.omega, p.h, damping="cell", prec=tdp.F32)
    assert rel(host(g32.precond(F, 1, 0.25, variant=1)), Uo) <= 1e-4
