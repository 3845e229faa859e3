"""GPU parity of the resident-tile 2-D sweep (tuning kernel 5): every tile
stays on one compute unit for a run of steps and swaps k-wide halo bands with
its neighbours through global memory every k steps.  Against the oracle on
the same seeded inputs at the FP64 bar (relative L2 error <= 1e-10), and
against the one-step kernel to rounding: multi-tile grids with ragged edges
and single tile rows or columns, every exchange depth, runs longer than one
launch, the samples of Table 1 when n_P is not a multiple of 4 (blocks end at
the sample step), the complex form as two real passes, the 5-point scheme,
fixed-iteration GMRES, the benchmark grid, FP32 fields, and the fall-back
where the kernel does not apply."""
import sys

import numpy as np
import pytest

import oracle
from paper_2006_16861_amd import inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def note(msg):
    print(f"[case] {msg}", file=sys.stderr, flush=True)


def dev(a):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def make_ops(p, prec=0, **kw):
    from paper_2006_16861_amd import tdp
    return tdp.operator_from_problem(p, prec=prec, **kw), oracle.Op.from_problem(p)


# tiles at exchange depth 4 (56 x 80 exact nodes each): 5 x 4, 3 x 1, 2 x 2,
# 1 x 1, 1 x 3, 4 x 1
GRIDS = [
    ("rand2d-300x250", lambda: inputs.random_medium((300, 250), seed=41, width=6)),
    ("rand2d-37x150", lambda: inputs.random_medium((37, 150), seed=1, width=4)),
    ("rand2d-130x61", lambda: inputs.random_medium((130, 61), seed=17, width=5)),
    ("rand2d-1x9", lambda: inputs.random_medium((1, 9), seed=2, width=0)),
    ("rand2d-200x5", lambda: inputs.random_medium((200, 5), seed=42, width=1)),
    ("rand2d-5x200", lambda: inputs.random_medium((5, 200), seed=43, width=1)),
]


@pytest.mark.parametrize("k", [2, 4, 6, 8])
@pytest.mark.parametrize("name,mk", GRIDS)
def test_resident_matches_oracle(name, mk, k):
    p = mk()
    note(f"resident {name} k={k}")
    g, o = make_ops(p)
    T = min(p.periods, 3)
    Uo = o.precond(p.F, T, 0.25)
    for graph in (1, 0):
        g.set_tuning(kernel=5, tb_depth=k, use_graph=graph)
        U = host(g.precond(dev(p.F), T, 0.25))
        assert rel(U, Uo) <= TOL64, graph
    g.set_tuning(kernel=1, use_graph=0)
    assert rel(U, host(g.precond(dev(p.F), T, 0.25))) <= 1e-13


@pytest.mark.parametrize("k", [2, 4, 6, 8])
@pytest.mark.parametrize("name,mk", [GRIDS[0], GRIDS[2], GRIDS[4]])
def test_resident_f32(name, mk, k):
    """FP32 fields (112 x 64 tiles): against the oracle at the FP32 bar and
    against the FP32 one-step kernel to rounding."""
    p = mk()
    note(f"resident f32 {name} k={k}")
    g, o = make_ops(p, prec=1)
    T = min(p.periods, 3)
    g.set_tuning(kernel=5, tb_depth=k)
    U = host(g.precond(dev(p.F), T, 0.25))
    assert rel(U, o.precond(p.F, T, 0.25)) <= 1e-4
    g.set_tuning(kernel=1)
    assert rel(U, host(g.precond(dev(p.F), T, 0.25))) <= 1e-5


def test_resident_runs_longer_than_one_launch():
    """N_s = 1080 steps: two launches (1024 + 56), the field handed over
    between them through the ping-pong pair."""
    p = inputs.random_medium((150, 130), seed=44, width=5)
    note("resident 150x130, T=90")
    g, o = make_ops(p)
    assert g.nP == 12
    g.set_tuning(kernel=5, tb_depth=4)
    U = host(g.precond(dev(p.F), 90, 0.1))
    assert rel(U, o.precond(p.F, 90, 0.1)) <= TOL64


def test_resident_general_steps_per_period_and_complex_form():
    """n_P not a multiple of 4: the sample u_{N_s - q} falls inside a block of
    k steps, which then ends there (odd block lengths, the level arrays swap
    roles); Def. 4 as two real passes."""
    from paper_2006_16861_amd import tdp
    p = inputs.random_medium((170, 140), seed=45, width=4)
    g = tdp.Operator(dev(p.c), dev(p.R), p.omega, p.h, steps_per_period=-1)
    assert g.nP % 4 != 0
    for nP in (g.nP, g.nP + 1, g.nP + 3):
        if nP % 4 == 0:
            continue
        o = oracle.Op.from_problem(p, nP=nP)
        gn = g if nP == g.nP else tdp.Operator(dev(p.c), dev(p.R), p.omega, p.h,
                                              steps_per_period=nP)
        for T in (2, 3):
            Uo = o.precond(p.F, T, 0.25)
            Uoc = o.precond(p.F, T, 0.25, variant=1)
            for k in (4, 6, 8):
                note(f"resident n_P={nP} T={T} k={k}")
                gn.set_tuning(kernel=5, tb_depth=k)
                assert rel(host(gn.precond(dev(p.F), T, 0.25)), Uo) <= TOL64, (nP, T, k)
                Uc = host(gn.precond(dev(p.F), T, 0.25, variant=1))
                assert rel(Uc, Uoc) <= TOL64, (nP, T, k)


FD2_2D = ((1.0, -0.5, 0.0), (0.25, 0.0, 0.0))


def test_resident_five_point_scheme():
    """The "fd2" scheme (no corner stiffness: the 5-point instantiation)."""
    from paper_2006_16861_amd import tdp
    p = inputs.random_medium((190, 150), seed=46, width=3)
    note("resident fd2 190x150")
    stiff, mass = FD2_2D
    o = oracle.Op(p.n, p.h, p.omega, p.c, p.R, stiff=stiff, mass=mass)
    g = tdp.Operator(dev(p.c), dev(p.R), p.omega, p.h, scheme="fd2")
    Uo = o.precond(p.F, 2, 0.25)
    for k in (2, 4, 8):
        g.set_tuning(kernel=5, tb_depth=k)
        assert rel(host(g.precond(dev(p.F), 2, 0.25)), Uo) <= TOL64, k


def test_resident_gmres_fixed_iterations_match_oracle():
    p = inputs.random_medium((160, 120), seed=47, width=5)
    note("resident gmres 160x120, 10 fixed iterations")
    g, o = make_ops(p)
    g.set_tuning(kernel=5, tb_depth=4)
    Ug, ig = g.solve(dev(p.F), T=p.periods, restart=6, fixed_iters=10)
    Uo, io = o.gmres(p.F, T=p.periods, restart=6, fixed_iters=10)
    assert ig.iters == io["iters"] == 10
    assert rel(host(Ug), Uo) <= TOL64


def test_resident_full_size_one_period_and_gmres():
    """The benchmark grid (smooth2d-1024: 247 tiles at depth 4, one per
    compute unit): one period against the oracle, and three fixed GMRES
    iterations against the blocked sweep."""
    p = inputs.smooth2d(1024)
    note("resident smooth2d-1024: P F with T=1; gmres 3 its vs kernel 2")
    g, o = make_ops(p)
    F = dev(p.F)
    Uo = o.precond(p.F, 1, 0.25)
    for k in (2, 4):
        g.set_tuning(kernel=5, tb_depth=k)
        assert rel(host(g.precond(F, 1, 0.25)), Uo) <= TOL64, k
    g.set_tuning(kernel=5, tb_depth=4)
    U5, i5 = g.solve(F, T=p.periods, fixed_iters=3)
    g.set_tuning(kernel=2, tb_depth=8, tile=5)
    U2, i2 = g.solve(F, T=p.periods, fixed_iters=3)
    assert i5.iters == i2.iters == 3
    assert rel(host(U5), host(U2)) <= 1e-11


def test_resident_falls_back_where_it_does_not_apply():
    """3-D, corner mass terms, and grids with more tiles than compute units:
    kernel 5 runs the automatic choice."""
    from paper_2006_16861_amd import tdp
    p3 = inputs.random_medium((9, 11, 70), seed=3, width=2)
    g, o = make_ops(p3)
    g.set_tuning(kernel=5, tb_depth=4)
    assert rel(host(g.precond(dev(p3.F), 2, 0.25)), o.precond(p3.F, 2, 0.25)) <= TOL64
    pb = inputs.random_medium((1400, 1200), seed=49, width=8)   # 18 x 22 tiles at depth 4
    gb, ob = make_ops(pb)
    gb.set_tuning(kernel=5, tb_depth=4)
    assert rel(host(gb.precond(dev(pb.F), 1, 0.25)), ob.precond(pb.F, 1, 0.25)) <= TOL64
    p = inputs.random_medium((150, 200), seed=18, width=6)
    stiff, mass = (2 / 3, -1 / 6, -1 / 3), (1 / 9, 1 / 18, 1 / 36)   # trilinear element tables
    oq = oracle.Op(p.n, p.h, p.omega, p.c, p.R, stiff=stiff, mass=mass)
    gq = tdp.Operator(dev(p.c), dev(p.R), p.omega, p.h, scheme="q1")
    gq.set_tuning(kernel=5, tb_depth=4)
    assert rel(host(gq.precond(dev(p.F), 2, 0.25)), oq.precond(p.F, 2, 0.25)) <= TOL64


def test_resident_abort_is_redone_with_the_blocked_sweep():
    """Recovery path, forced from the host: every wait of the resident launch
    looks for a flag value no tile writes and gives up after a few polls (all
    kernels still exit normally); the application is redone with the blocked
    sweep, counted, and the op's tuning goes back to auto."""
    p = inputs.random_medium((170, 140), seed=48, width=4)
    note("resident forced abort 170x140")
    g, o = make_ops(p)
    Uo = o.precond(p.F, 2, 0.25)
    g.set_tuning(kernel=5, tb_depth=4)
    assert rel(host(g.precond(dev(p.F), 2, 0.25)), Uo) <= TOL64
    assert g.resident_aborts == 0
    g.force_resident_abort(True)
    assert rel(host(g.precond(dev(p.F), 2, 0.25)), Uo) <= TOL64
    assert g.resident_aborts == 1 and g.get_tuning()["kernel"] == 0
    g.set_tuning(kernel=5, tb_depth=4)
    Ug, ig = g.solve(dev(p.F), T=p.periods, restart=6, fixed_iters=4)
    Uog, io = o.gmres(p.F, T=p.periods, restart=6, fixed_iters=4)
    assert ig.iters == io["iters"] == 4 and rel(host(Ug), Uog) <= TOL64
    assert g.resident_aborts == 2
    g.force_resident_abort(False)
    g.set_tuning(kernel=5, tb_depth=4)
    assert rel(host(g.precond(dev(p.F), 2, 0.25)), Uo) <= TOL64
    assert g.resident_aborts == 2
