"""Batched form: many right-hand sides per medium and uneven problems in one
batched preconditioner launch sequence, GMRES in lockstep.  Every field must
match its own single solve and the oracle."""
import sys

import numpy as np
import pytest

import oracle
from paper_2006_16861_amd import inputs

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[case] {msg}", file=sys.stderr, flush=True)


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def small_batch(prec=0):
    from paper_2006_16861_amd import tdp
    probs = [inputs.random_medium((37, 150), seed=1, width=4), inputs.const2d(),
             inputs.random_medium((90, 70), seed=5, width=6, cmin=1.0, cmax=3.0)]
    nrhs = [3, 1, 2]
    ops = [tdp.operator_from_problem(p, prec=prec) for p in probs]
    rng = np.random.default_rng(7)
    Fs = []
    for p, r in zip(probs, nrhs):
        for k in range(r):
            Fs.append(rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n) if k else p.F)
    return probs, nrhs, ops, Fs


@pytest.mark.parametrize("depth,tile", [(8, 1), (4, 0), (3, 3), (8, 4), (4, 5), (3, 7)])
def test_batch_precond_matches_single_and_oracle(depth, tile):
    from paper_2006_16861_amd import tdp
    probs, nrhs, ops, Fs = small_batch()
    note(f"batch precond depth={depth} tile={tile}")
    b = tdp.Batch(ops, nrhs)
    b.set_tuning(depth, tile)
    T = [3, 2, 4]
    Us = b.precond([dev(F) for F in Fs], T)
    q = 0
    for i, (p, r) in enumerate(zip(probs, nrhs)):
        o = oracle.Op.from_problem(p)
        for k in range(r):
            got = Us[q].cpu().numpy()
            single = ops[i].precond(dev(Fs[q]), T[i]).cpu().numpy()
            assert rel(got, single) <= 1e-13
            assert rel(got, o.precond(Fs[q], T[i])) <= 1e-10
            q += 1


def test_batch_gmres_fixed_and_converged_match_oracle():
    from paper_2006_16861_amd import tdp
    probs, nrhs, ops, Fs = small_batch()
    note("batch gmres fixed / converged")
    b = tdp.Batch(ops, nrhs)
    T = [p.periods for p in probs]
    Us, infos, rc = b.solve([dev(F) for F in Fs], T, restart=4, fixed_iters=7)
    q = 0
    for i, (p, r) in enumerate(zip(probs, nrhs)):
        o = oracle.Op.from_problem(p)
        for k in range(r):
            Uo, io = o.gmres(Fs[q], T[i], restart=4, fixed_iters=7)
            assert infos[q].iters == 7 and infos[q].restarts == io["restarts"]
            assert rel(Us[q].cpu().numpy(), Uo) <= 1e-10
            q += 1
    Us, infos, rc = b.solve([dev(F) for F in Fs], T, tol=1e-8)
    assert rc == 0
    q = 0
    for i, (p, r) in enumerate(zip(probs, nrhs)):
        o = oracle.Op.from_problem(p)
        for k in range(r):
            Uo, io = o.gmres(Fs[q], T[i], tol=1e-8)
            U = Us[q].cpu().numpy()
            assert infos[q].iters == io["iters"] and infos[q].restarts == io["restarts"]
            assert rel(o.apply_H(U), Fs[q]) <= 1e-8 * (1 + 1e-9)
            assert rel(U, Uo) <= 1e-10
            q += 1


def test_batch_f32_reaches_tolerance():
    from paper_2006_16861_amd import tdp
    probs, nrhs, ops, Fs = small_batch(prec=1)
    note("batch f32 to 1e-6")
    b = tdp.Batch(ops, nrhs)
    T = [p.periods for p in probs]
    Us, infos, rc = b.solve([dev(F) for F in Fs], T, tol=1e-6)
    assert rc == 0
    q = 0
    for i, (p, r) in enumerate(zip(probs, nrhs)):
        o = oracle.Op.from_problem(p)
        for k in range(r):
            assert rel(o.apply_H(Us[q].cpu().numpy()), Fs[q]) <= 1e-6 * (1 + 1e-9)
            q += 1


def test_batch_full_config_sampled():
    """64 right-hand sides on the 512^2 medium plus 32 uneven problems
    (128..768 per side), FP32 fields, all to 1e-6; the true residual of a
    sample of fields is recomputed by the oracle."""
    from paper_2006_16861_amd import tdp
    note("batch full config (64 RHS 512^2 + 32 uneven), f32")
    base = inputs.smooth2d(512, seed=4, src_seed=5)
    srcs = inputs.random_sources(base.n, 64, seed=5, margin=32)
    uneven = inputs.uneven_problems()
    probs = [base] + uneven
    nrhs = [64] + [1] * len(uneven)
    ops = [tdp.operator_from_problem(p, prec=1) for p in probs]
    b = tdp.Batch(ops, nrhs)
    Fs = [dev(srcs[k]) for k in range(64)] + [dev(p.F) for p in uneven]
    Us, infos, rc = b.solve(Fs, [p.periods for p in probs], tol=1e-6)
    assert rc == 0
    assert all(inf.relres <= 1e-6 for inf in infos)
    for q in [0, 17, 63, 64, 80, 95]:
        p = base if q < 64 else uneven[q - 64]
        F = srcs[q] if q < 64 else p.F
        o = oracle.Op.from_problem(p)
        r = rel(o.apply_H(Us[q].cpu().numpy()), F)
        note(f"  field {q}: iters {infos[q].iters} oracle-checked relres {r:.3e}")
        assert r <= 1e-6 * (1 + 1e-9)


def test_batch_autotune_keeps_results_exact():
    from paper_2006_16861_amd import tdp
    probs, nrhs, ops, Fs = small_batch()
    note("batch autotune")
    b = tdp.Batch(ops, nrhs)
    table = b.autotune([2, 2, 2])
    assert len(table) >= 10 and min(r[3] for r in table) > 0
    assert {int(r[2]) for r in table} >= {-1, 0, 1, 2}      # shared-medium tiles and none
    T = [3, 2, 4]
    Us = b.precond([dev(F) for F in Fs], T)
    q = 0
    for i, (p, r) in enumerate(zip(probs, nrhs)):
        o = oracle.Op.from_problem(p)
        for k in range(r):
            assert rel(Us[q].cpu().numpy(), o.precond(Fs[q], T[i])) <= 1e-10
            q += 1


def test_batch_with_general_steps_per_period():
    """Fields whose n_P is not a multiple of 4 (n_P = 10 and 11, next to a
    field with the default n_P = 12) in one batch: each matches the oracle run
    with its n_P, for the batched preconditioner and fixed-iteration GMRES."""
    from paper_2006_16861_amd import tdp
    probs = [inputs.random_medium((40, 50), seed=34, width=3),
             inputs.random_medium((37, 150), seed=1, width=4), inputs.const2d()]
    spp = [-1, 11, 0]
    ops = [tdp.operator_from_problem(p, steps_per_period=v) for p, v in zip(probs, spp)]
    assert [o.nP for o in ops] == [10, 11, 12]
    note("batch with n_P = 10, 11, 12")
    b = tdp.Batch(ops, [1, 2, 1])
    rng = np.random.default_rng(8)
    Fs = [probs[0].F, probs[1].F, rng.standard_normal(probs[1].n) + 1j * rng.standard_normal(probs[1].n),
          probs[2].F]
    fo = [0, 1, 1, 2]
    orc = [oracle.Op.from_problem(p, nP=o.nP) for p, o in zip(probs, ops)]
    for depth, tile in ((8, 4), (4, 5)):
        b.set_tuning(depth, tile)
        T = [3, 2, 4]
        Us = b.precond([dev(F) for F in Fs], T)
        for q, F in enumerate(Fs):
            i = fo[q]
            assert rel(Us[q].cpu().numpy(), orc[i].precond(F, T[i])) <= 1e-10, (q, depth, tile)
    T = [p.periods for p in probs]
    Us, infos, rc = b.solve([dev(F) for F in Fs], T, restart=4, fixed_iters=6)
    for q, F in enumerate(Fs):
        i = fo[q]
        Uo, io = orc[i].gmres(F, T[i], restart=4, fixed_iters=6)
        assert infos[q].iters == 6
        assert rel(Us[q].cpu().numpy(), Uo) <= 1e-10, q


def test_batch_argument_errors():
    from paper_2006_16861_amd import tdp
    probs, nrhs, ops, Fs = small_batch()
    b = tdp.Batch(ops, nrhs)
    F = [dev(F) for F in Fs]
    b.set_tuning(8, 4)
    # T < 1; N_s beyond 2^24; a captured application beyond 2^17 launches of 8 steps
    for T in ([0, 1, 1], [1, (1 << 24) // ops[1].nP + 1, 1], [1, (8 << 17) // ops[1].nP + 1, 1]):
        with pytest.raises(tdp.TdpError) as ei:
            b.precond(F, T)
        assert ei.value.code == tdp.EINVAL
        with pytest.raises(tdp.TdpError):
            b.solve(F, T, fixed_iters=1)
        with pytest.raises(tdp.TdpError):
            b.autotune(T)
    Fbad = [f.clone() for f in F]
    Fbad[2][3, 3] = float("nan")
    with pytest.raises(tdp.TdpError) as ei:         # refused at once, not iterated
        b.solve(Fbad, [2, 2, 2], tol=1e-6)
    assert ei.value.code == tdp.EINVAL and "NaN" in str(ei.value)


def test_batch_f32_tall_tile():
    """The FP32-only 128 x 64 tile with per-node coefficients (tile 8) in the
    batched sweep matches the oracle and the one-step FP32 path; FP64 batches
    refuse it."""
    from paper_2006_16861_amd import tdp
    probs, nrhs, ops, Fs = small_batch(prec=1)
    note("batch f32 tile 8")
    b = tdp.Batch(ops, nrhs)
    T = [3, 2, 4]
    for depth, mt in ((8, 0), (12, 1)):
        b.set_tuning(depth, 8, mt)
        Us = b.precond([dev(F) for F in Fs], T)
        q = 0
        for i, (p, r) in enumerate(zip(probs, nrhs)):
            o = oracle.Op.from_problem(p)
            ops[i].set_tuning(kernel=1)
            for k in range(r):
                got = Us[q].cpu().numpy()
                assert rel(got, o.precond(Fs[q], T[i])) <= 1e-4
                assert rel(got, ops[i].precond(dev(Fs[q]), T[i]).cpu().numpy()) <= 1e-5
                q += 1
    probs64, nrhs64, ops64, _ = small_batch()
    b64 = tdp.Batch(ops64, nrhs64)
    with pytest.raises(tdp.TdpError):
        b64.set_tuning(8, 8)
    with pytest.raises(tdp.TdpError):          # 4 x 12 rows exceed the 32-row shared tile
        b64.set_tuning(12, 4, 0)
    with pytest.raises(tdp.TdpError):
        b64.set_tuning(8, 4, 3)


def medium_batch(prec, nshared=7):
    """One medium with `nshared` right-hand sides (slabs of every shared tile
    end ragged) next to a second medium with one."""
    from paper_2006_16861_amd import tdp
    probs = [inputs.random_medium((75, 140), seed=11, width=5),
             inputs.random_medium((50, 61), seed=12, width=3)]
    nrhs = [nshared, 1]
    ops = [tdp.operator_from_problem(p, prec=prec) for p in probs]
    rng = np.random.default_rng(13)
    Fs = [rng.standard_normal(probs[0].n) + 1j * rng.standard_normal(probs[0].n)
          for _ in range(nshared)] + [probs[1].F]
    return probs, nrhs, ops, Fs


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("mtile", [0, 1, 2])
def test_shared_medium_tile_matches_oracle_and_per_field_tiles(prec, mtile):
    """Shared-medium tile: every right-hand side of the medium matches the
    oracle (FP64 fields: <= 1e-10; FP32 fields: <= 1e-4 against the FP64
    oracle) and the per-field tile with the same arithmetic (tile 5), at two
    depths, including the slab that ends short."""
    from paper_2006_16861_amd import tdp
    probs, nrhs, ops, Fs = medium_batch(prec)
    b = tdp.Batch(ops, nrhs)
    T = [3, 2]
    orc = [oracle.Op.from_problem(p) for p in probs]
    fo = [0] * nrhs[0] + [1]
    for depth in (8, 5):
        note(f"shared-medium tile {mtile} prec={prec} depth={depth}")
        b.set_tuning(depth, 5, -1)
        ref = [U.cpu().numpy() for U in b.precond([dev(F) for F in Fs], T)]
        b.set_tuning(depth, 5, mtile)
        Us = b.precond([dev(F) for F in Fs], T)
        for q, F in enumerate(Fs):
            got = Us[q].cpu().numpy()
            assert np.isfinite(got).all()
            assert rel(got, ref[q]) <= (1e-13 if prec == 0 else 1e-6), (q, depth)
            assert rel(got, orc[fo[q]].precond(F, T[fo[q]])) <= (1e-10 if prec == 0 else 1e-4), (q, depth)


def test_shared_medium_gmres_lockstep_matches_oracle():
    """GMRES in lockstep over the shared-medium tile: fixed iterations agree
    with the oracle element-wise, and tolerance mode takes each field's own
    decisions (same iterations and restarts as the oracle).  The right-hand
    sides converge after different numbers of iterations, so the slabs of
    live fields change between applications."""
    from paper_2006_16861_amd import tdp
    probs, nrhs, ops, Fs = medium_batch(0, nshared=5)
    # one zero right-hand side (done before the first application) and one
    # smooth one next to the random ones
    ny, nx = probs[0].n
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    Fs[2] = np.sin(np.pi * (iy + 1) / (ny + 1)) * np.sin(np.pi * (ix + 1) / (nx + 1)) + 0j
    Fs[3] = np.zeros(probs[0].n, dtype=np.complex128)
    b = tdp.Batch(ops, nrhs)
    b.set_tuning(8, 5, 0)
    T = [p.periods for p in probs]
    fo = [0] * nrhs[0] + [1]
    orc = [oracle.Op.from_problem(p) for p in probs]
    note("shared-medium gmres fixed")
    Us, infos, rc = b.solve([dev(F) for F in Fs], T, restart=4, fixed_iters=6)
    for q, F in enumerate(Fs):
        Uo, io = orc[fo[q]].gmres(F, T[fo[q]], restart=4, fixed_iters=6)
        if q == 3:
            assert not Us[q].cpu().numpy().any()
            continue
        assert infos[q].iters == 6 and rel(Us[q].cpu().numpy(), Uo) <= 1e-10, q
    note("shared-medium gmres tol 1e-8")
    Us, infos, rc = b.solve([dev(F) for F in Fs], T, tol=1e-8)
    assert rc == 0
    its = []
    for q, F in enumerate(Fs):
        Uo, io = orc[fo[q]].gmres(F, T[fo[q]], tol=1e-8)
        U = Us[q].cpu().numpy()
        its.append(infos[q].iters)
        if q == 3:
            assert not U.any()
            continue
        assert infos[q].iters == io["iters"] and infos[q].restarts == io["restarts"], q
        assert rel(orc[fo[q]].apply_H(U), F) <= 1e-8 * (1 + 1e-9)
        assert rel(U, Uo) <= 1e-10
    assert its[3] == 0 and len(set(its[:nrhs[0]])) > 1   # slabs of the live fields only


def test_batch_full_size_application_elementwise():
    """One batched application of the benchmarked configuration (64 right-hand
    sides on the 512^2 medium through the shared-medium tile, 32 uneven
    problems, FP32 fields) against the FP64 oracle element-wise on two of the
    64 fields and on the largest uneven field, and against the same fields
    run alone through the single-field FP32 path."""
    from paper_2006_16861_amd import tdp
    note("batch full-size application, f32")
    base = inputs.smooth2d(512, seed=4, src_seed=5)
    srcs = inputs.random_sources(base.n, 64, seed=5, margin=32)
    uneven = inputs.uneven_problems()
    probs = [base] + uneven
    nrhs = [64] + [1] * len(uneven)
    ops = [tdp.operator_from_problem(p, prec=1) for p in probs]
    b = tdp.Batch(ops, nrhs)
    T = [p.periods for p in probs]
    Fs = [dev(srcs[k]) for k in range(64)] + [dev(p.F) for p in uneven]
    Us = b.precond(Fs, T)
    big = max(range(len(uneven)), key=lambda i: uneven[i].N)
    for q in (5, 63, 64 + big):
        p = base if q < 64 else uneven[q - 64]
        F = srcs[q] if q < 64 else p.F
        i = 0 if q < 64 else q - 63
        got = Us[q].cpu().numpy()
        single = ops[i].precond(Fs[q], T[i]).cpu().numpy()
        ref = oracle.Op.from_problem(p).precond(F, T[i])
        e_single, e_orc = rel(got, single), rel(got, ref)
        note(f"  field {q} n={p.n}: vs single FP32 {e_single:.2e}, vs FP64 oracle {e_orc:.2e}")
        assert e_single <= 1e-6
        assert e_orc <= 1e-4


def test_batch_rejected_table1_cycle_ends_its_field():
    """Reading R19 in the batched form, which runs Table 1 only: a cycle that
    lowers no true residual ends its field with ENOTCONV and the iterate of
    least true residual (the single solve switches to Def. 4 on the same
    problem and converges); the other field of the batch is unaffected."""
    from paper_2006_16861_amd import tdp
    pd, pc = inputs.disc2d(64, width=16), inputs.const2d()
    note("batch with a rejected Table 1 cycle: disc2d-64 T=5 + const2d")
    ops = [tdp.operator_from_problem(pd), tdp.operator_from_problem(pc)]
    Ug, ig = ops[0].solve(dev(pd.F), T=5, tol=1e-6, max_iters=600)
    assert ig.status == 0 and ig.switched == 1
    b = tdp.Batch(ops, [1, 1])
    Us, infos, rc = b.solve([dev(pd.F), dev(pc.F)], [5, pc.periods], tol=1e-6, max_iters=600)
    assert rc == tdp.ENOTCONV
    r0 = rel(oracle.Op.from_problem(pd).apply_H(Us[0].cpu().numpy()), pd.F)
    assert infos[0].status == 1 and np.isfinite(r0) and r0 < 1.0
    assert abs(infos[0].relres - r0) <= 1e-6 * r0
    r1 = rel(oracle.Op.from_problem(pc).apply_H(Us[1].cpu().numpy()), pc.F)
    assert infos[1].status == 0 and r1 <= 1e-6 * (1 + 1e-9)


def test_batch_field_results_do_not_depend_on_the_other_fields():
    """Lockstep GMRES runs each per-field step (CGS2, the true residual, the
    H-apply) as one launch sequence over all live fields, with each field's
    own reductions: a field solved in a batch of six ends bit for bit where it
    ends solved alone (every field on its own tile), in tolerance mode and in
    fixed-iteration mode."""
    import torch
    from paper_2006_16861_amd import tdp
    probs, nrhs, ops, Fs = small_batch()
    T = [p.periods for p in probs]
    big = tdp.Batch(ops, nrhs)
    big.set_tuning(8, 5, -1)
    for op_i, mode in [(0, "tol"), (0, "fixed"), (2, "tol")]:
        field = {0: 1, 2: 5}[op_i]
        note(f"batch independence: field {field} ({mode})")
        kw = dict(tol=1e-8) if mode == "tol" else dict(restart=4, fixed_iters=7)
        Us, infos, rc = big.solve([dev(F) for F in Fs], T, **kw)
        one = tdp.Batch([ops[op_i]], [1])
        one.set_tuning(8, 5, -1)
        U1, info1, rc1 = one.solve([dev(Fs[field])], [T[op_i]], **kw)
        assert rc1 == rc == 0
        assert info1[0].iters == infos[field].iters
        assert info1[0].restarts == infos[field].restarts
        assert torch.equal(U1[0], Us[field]), (field, mode)
        one.close()
    big.close()
