"""Benchmark: Helmholtz solves/s at 1e-6 true relative residual, and the
recurrence sweep's GB/s against the MI355X HBM roofline.

Workload (default): 2-D smooth random medium 1024 x 1024, h = 1/1025,
c in [1.5, 4.5] (seeded Gaussian-filtered field, sigma = 20 cells), omega for
10 points per minimum wavelength, 32-cell quadratic damping layer, point
source at a seeded node, compact 9-point stencil, FP64 fields, preconditioner
T = 103 periods, rho = 0.25, GMRES(30) to a true relative residual of 1e-6.

One timed step = one complete solve (F resident in HBM -> U resident in HBM),
operator setup excluded.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, published
WORDS_PER_NODE_STEP = 7          # u_j, u_{j-1}, u_{j+1}, m, damping, Re F, Im F
# a launch of k steps must read u_j, u_{j-1}, m, the damping factor and F
# (2 words) and write u_{j+k}, u_{j+k-1}: 8 words per node, whatever k
WORDS_PER_NODE_LAUNCH = 8
RES_MAX_STEPS = 1024          # steps of one resident-tile launch (kernel 5)
# published MI355X vector peaks (TFLOP/s); the FP32 figure needs packed FP32
# instructions, which this build does not emit (non-packed FP32 issues at the
# FP64 rate)
ALU_PEAK = {8: 78.6, 4: 157.3}
ALU_PEAK_UNPACKED_F32 = 78.6


def flops_per_node_step(ndim, stencil_points):
    """Floating-point operations of one node update: one FMA (2 flops) per
    stencil point, two for the forcing (Re F, Im F) and one for the u_{j-1}
    term."""
    return 2 * stencil_points + 6


def roofline_block(kernel, launch_us, alg_bytes, alg_flops, word, traffic=None,
                   effective_bytes=None, note=None, effective_label="7word"):
    """Roofline of one launch of a kernel: the algorithmic bytes it must move
    (its inputs read once, its outputs written once) and its useful flops,
    each over the launch time, against the HBM peak and the vector ALU peak.
    frac is the larger of the two fractions (<= 1 by construction); bound names
    that roof, or "latency" when neither reaches half of its peak.
    effective_bytes, if given, is a per-step word model over the launch's
    steps (no reuse across steps; 7 words per node-step for the node damping,
    named by effective_label), reported separately: temporal blocking takes it
    above the HBM peak."""
    t = launch_us * 1e-6
    gbps = alg_bytes / t / 1e9
    tflops = alg_flops / t / 1e12
    f_hbm = gbps / HBM_PEAK_GBS
    f_alu = tflops / ALU_PEAK[word]
    roof = "hbm" if f_hbm >= f_alu else "alu"
    frac = max(f_hbm, f_alu)
    out = {"bound": roof if frac >= 0.5 else "latency", "roof": roof,
           "achieved": gbps if roof == "hbm" else tflops,
           "peak": HBM_PEAK_GBS if roof == "hbm" else ALU_PEAK[word],
           "unit": "GB/s" if roof == "hbm" else "TFLOP/s", "frac": frac,
           "traffic": traffic, "kernel": kernel, "avg_launch_us": launch_us,
           "algorithmic_bytes_per_launch": alg_bytes, "hbm_frac": f_hbm,
           "alu": {"flops_per_launch": alg_flops, "achieved_TFLOPs": tflops,
                   "peak_TFLOPs": ALU_PEAK[word], "frac": f_alu}}
    if word == 4:
        out["alu"]["peak_TFLOPs_unpacked"] = ALU_PEAK_UNPACKED_F32
    if traffic:
        out["traffic_GBps"] = traffic / t / 1e9
        out["traffic_frac"] = traffic / t / 1e9 / HBM_PEAK_GBS
    if effective_bytes:
        out[f"effective_GBps_{effective_label}"] = effective_bytes / t / 1e9
        out[f"effective_frac_{effective_label}"] = effective_bytes / t / 1e9 / HBM_PEAK_GBS
    if note:
        out["note"] = note
    return out


def measured_traffic(workload, prec, variant, tun, damping="node", scheme="compact"):
    """HBM bytes per launch of the dominant kernel, from the rocprofv3
    FETCH_SIZE / WRITE_SIZE runs recorded in profiles/traffic.json (scaled by
    the copy-kernel calibration); None when that kernel configuration was not
    measured."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    key = f"{workload}|{prec}|v{variant}|k{tun['kernel']}|d{tun['tb_depth']}|t{tun['tile']}"
    if damping != "node":
        key += f"|{damping}"
    if scheme != "compact":
        key += f"|{scheme}"
    rec = json.load(open(path)).get(key)
    return None if rec is None else rec["bytes_per_launch"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_problem(name):
    from paper_2006_16861_amd import inputs
    if name == "smooth2d-1024":
        return inputs.smooth2d(1024)
    if name == "const2d-64":
        return inputs.const2d()
    if name == "layered3d-256":
        return inputs.layered3d(256)
    if name.startswith("smooth2d-"):
        return inputs.smooth2d(int(name.split("-")[1]))
    raise SystemExit(f"unknown workload {name}")


def sweep_timing(op, F, T, rho, reps, stream, variant=0):
    """Average duration of one recurrence-step launch, from HIP events on the
    stream the sweep kernels are launched on, over `reps` preconditioner
    applications (each N_s = T n_P launches plus two staging copies)."""
    import torch
    U = torch.empty_like(F)
    op.precond(F, T, rho, out=U, variant=variant)          # capture / warm
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        op.precond(F, T, rho, out=U, variant=variant)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return ms, ms / (T * op.nP)


_ONE_THREAD = """
import json, sys, time
sys.path.insert(0, sys.argv[1])
import bench, oracle
p = bench.make_problem(sys.argv[2])
op = oracle.Op.from_problem(p)
t = time.perf_counter()
op.precond(p.F, 1, float(sys.argv[3]))
print(json.dumps({"ms_per_step": (time.perf_counter() - t) / op.nP * 1e3}))
"""


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_one_thread(workload, rho):
    """Oracle steps on one host thread (a separate process with
    OMP_NUM_THREADS=1): one period of recurrence steps on the full grid."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _ONE_THREAD, ROOT, workload, str(rho)],
                       capture_output=True, text=True, env=env, timeout=300)
    if r.returncode != 0:
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])["ms_per_step"]


def cpu_baseline(p, T, rho, napply, target_s=12.0, workload=None, handoff=None):
    """The oracle (plain C, OpenMP) on the host cores: time one H-apply and a
    bounded number of recurrence steps, scale to napply preconditioner
    applications (+ H-applies) per solve.  Also one period of steps on a
    single thread, for the per-core rate."""
    import numpy as np
    import oracle
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    op = oracle.Op.from_problem(p)
    t = time.perf_counter()
    op.apply_H(p.F)
    tH = time.perf_counter() - t
    t = time.perf_counter()
    op.precond(p.F, 1, rho)
    t1 = time.perf_counter() - t
    per_step = t1 / op.nP
    Ts = max(1, min(T, int(target_s / (per_step * op.nP))))
    t = time.perf_counter()
    op.precond(p.F, Ts, rho)
    tT = time.perf_counter() - t
    per_step = tT / (Ts * op.nP)
    t_solve = napply * (per_step * T * op.nP + tH)
    out = {"value": 1.0 / t_solve, "unit": "solves/s", "cores": cores, "kind": "oracle",
           "sample": f"{Ts * op.nP} recurrence steps + 1 H-apply on the full grid "
                     f"({per_step * 1e3:.2f} ms/step), scaled to {napply} preconditioner "
                     f"applications of {T * op.nP} steps per solve",
           "cpu_model": cpu_model(), "ms_per_step": per_step * 1e3}
    if workload is not None:
        one = cpu_one_thread(workload, rho)
        if one is not None:
            out["one_thread_ms_per_step"] = one
            # the H-applies (< 1% of a solve) left out
            out["one_thread_solves_per_s_steps_only"] = 1.0 / (napply * one * 1e-3 * T * op.nP)
    if handoff:
        out["legs"] = cpu_baseline_legs(oracle, handoff, rho)
    return out


def cpu_baseline_legs(oracle, handoff, rho):
    """Part of the CPU baseline leg (called from cpu_baseline, which passes
    the oracle module): the oracle on the configurations beyond the headline: one recurrence
    period and one H-apply on the full grid, extrapolated to the GPU run's
    preconditioner applications (labelled "extrapolated"); for the precision
    form also the oracle's check of the GPU results: its one-period S_T F
    against both GPU paths', and the true residual of both GPU solutions under
    the oracle's H."""
    legs = {}

    def period(p, nP, T):
        op = oracle.Op.from_problem(p, nP=nP) if nP else oracle.Op.from_problem(p)
        t = time.perf_counter()
        pf = op.precond(p.F, 1, rho)
        t_period = time.perf_counter() - t
        t = time.perf_counter()
        op.apply_H(p.F)
        t_h = time.perf_counter() - t
        return op, pf, t_period / op.nP, t_h

    if "precision" in handoff:
        h = handoff["precision"]
        p = h["problem"]
        op, pf, t_step, t_h = period(p, h["n_P"], p.periods)
        t_solve = h["napply"] * (t_step * p.periods * h["n_P"] + t_h)
        nrm = float(np.linalg.norm(p.F))
        chk = {"pf1_rel_error_vs_oracle": {k: float(np.linalg.norm(v - pf) / np.linalg.norm(pf))
                                           for k, v in h["PF1"].items()},
               "true_relres_under_oracle_H": {k: float(np.linalg.norm(op.apply_H(v) - p.F) / nrm)
                                              for k, v in h["U"].items()}}
        legs["precision"] = {"workload": "layered3d-256", "kind": "oracle", "extrapolated": True,
                             "ms_per_step": t_step * 1e3, "H_ms": t_h * 1e3,
                             "solves_per_s": 1.0 / t_solve,
                             "sample": f"{h['n_P']} recurrence steps + 1 H-apply on the full "
                                       f"grid, scaled to {h['napply']} applications of "
                                       f"{p.periods * h['n_P']} steps",
                             "oracle_check": chk}
        log(f"cpu leg precision: {t_step * 1e3:.0f} ms/step; check {chk}")
    if "batched" in handoff:
        h = handoff["batched"]
        p = h["problem"]
        op, _, t_step, t_h = period(p, 0, p.periods)
        # per field: its applications x (T n_P steps + one H-apply), at the
        # sampled per-node rate for the other grid sizes
        t_node_step, t_node_h = t_step / p.N, t_h / p.N
        t_all = sum(na * N * (T * nP * t_node_step + t_node_h)
                    for na, N, T, nP in h["fields"])
        legs["batched"] = {"workload": "64 rhs on smooth2d-512 + 32 uneven", "kind": "oracle",
                           "extrapolated": True, "ms_per_step_512": t_step * 1e3,
                           "solves_per_s": len(h["fields"]) / t_all,
                           "sample": "one period + 1 H-apply on the 512^2 grid, scaled per node "
                                     "to every field's applications"}
    if "adjoint" in handoff:
        h = handoff["adjoint"]
        p = h["problem"]
        op, _, t_step, t_h = period(p, h["n_P"], p.periods)
        t_grad = h["napply_per_gradient"] * (t_step * p.periods * h["n_P"] + t_h)
        legs["adjoint"] = {"workload": "smooth3d-128", "kind": "oracle", "extrapolated": True,
                           "ms_per_step": t_step * 1e3, "gradients_per_s": 1.0 / t_grad,
                           "sample": f"{h['n_P']} recurrence steps + 1 H-apply, scaled to "
                                     f"{h['napply_per_gradient']} applications per gradient"}
    return legs


def stream_probe(nbytes=2 << 30, reps=5):
    """Practical HBM ceiling on this device: best of `reps` plain device copies
    (read + write nbytes) and triads c = a + b (2 reads + 1 write), timed with
    events; reported next to the 8 TB/s specification."""
    import torch
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    c = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = {"copy": 0.0, "triad": 0.0}
    for _ in range(reps):
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best["copy"] = max(best["copy"], 2 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9)
        e0.record()
        torch.add(a, b, out=c)
        e1.record()
        torch.cuda.synchronize()
        best["triad"] = max(best["triad"], 3 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del a, b, c
    torch.cuda.empty_cache()
    return best


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t


def form_precision(rho):
    """Precision form on the 3-D layered medium (256^3, 8 ppw, T = 32, n_P = 10:
    the smallest integer above the CFL bound 9.58, with Im U from the 2x2
    solve of Sec. 2.3, against 12 for a multiple of 4): FP32
    recurrence fields inside FP64 GMRES (whose restarts recompute the true
    residual in FP64: the outer refinement), against the FP64 path.  Returns
    the result and what the CPU baseline leg checks against the oracle: both
    solutions and both paths' one-period preconditioner application."""
    import torch
    from paper_2006_16861_amd import inputs, tdp
    p = inputs.layered3d(256)
    F = torch.as_tensor(p.F, device="cuda")
    res = {"workload": "layered3d-256", "n": list(p.n), "periods_T": p.periods}
    U, PF1 = {}, {}
    for name, prec in (("f64", tdp.F64), ("f32", tdp.F32)):
        op = tdp.operator_from_problem(p, prec=prec, steps_per_period=-1)
        best, table = op.autotune(T=4, rho=rho)
        op.solve(F, T=p.periods, rho=rho, tol=1e-6)                 # warm (graphs)
        (Uq, info), dt = _timed(lambda: op.solve(F, T=p.periods, rho=rho, tol=1e-6))
        _, step_ms = sweep_timing(op, F, p.periods, rho, 1, torch.cuda.current_stream())
        us_step = step_ms * 1e3
        r = float(torch.linalg.norm(F - op.apply_H(Uq)) / torch.linalg.norm(F))
        U[name] = Uq.cpu().numpy()
        PF1[name] = op.precond(F, 1, rho).cpu().numpy()
        word = 8 if prec == tdp.F64 else 4
        tun = op.get_tuning()
        tname = 'double' if word == 8 else 'float'
        kname = (f"k_sweep3d_stream<{tname}> shape={tun['tile']} z-chunk={tun['tb_depth']}"
                 if tun["kernel"] == 3 else
                 f"k_sweep3d_stream2<{tname}> shape={tun['tile']} (two steps per launch)"
                 if tun["kernel"] == 4 else f"kernel {tun['kernel']}")
        spl = {4: 2}.get(tun["kernel"], 1)
        words_launch = WORDS_PER_NODE_LAUNCH if spl > 1 else WORDS_PER_NODE_STEP
        key = f"layered3d-256|{name}|v0|k{tun['kernel']}|d{tun['tb_depth']}|t{tun['tile']}"
        traffic = _traffic(key)
        res[name] = {"solves_per_s": 1.0 / dt, "seconds": dt, "iters": info.iters, "n_P": op.nP,
                     "precond_applications": info.steps // (p.periods * op.nP),
                     "switched": int(info.switched),
                     "true_relres_fp64": r, "tuning": best, "sweep_us_per_step": us_step,
                     "roofline": roofline_block(kname, us_step * spl,
                                                p.N * word * words_launch,
                                                flops_per_node_step(3, 19) * p.N * spl, word,
                                                traffic=traffic)}
        log(f"form precision {name}: {dt:.3f} s, iters {info.iters}, relres {r:.2e}")
        del op
    res["f32_rel_error_vs_f64_gpu_solution"] = float(
        np.linalg.norm(U["f32"] - U["f64"]) / np.linalg.norm(U["f64"]))
    res["speedup_f32_vs_f64"] = res["f32"]["solves_per_s"] / res["f64"]["solves_per_s"]
    handoff = {"problem": p, "U": U, "PF1": PF1, "rho": rho, "n_P": res["f64"]["n_P"],
               "napply": res["f64"]["precond_applications"]}
    return res, handoff


def _traffic(key):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(key)
    return None if rec is None else rec["bytes_per_launch"]


def profile_batched(args):
    """Profiling mode of the batched form's shared-medium sweep: the 64
    right-hand sides of form_batched on their 512^2 medium, at a fixed tuning,
    after the same 256 MiB calibration copy as --profile-sweeps."""
    import torch
    from paper_2006_16861_amd import inputs, tdp
    base = inputs.smooth2d(512, seed=4, src_seed=5)
    srcs = inputs.random_sources(base.n, 64, seed=5, margin=32)
    op = tdp.operator_from_problem(base, prec=tdp.F32)
    Fs = [torch.as_tensor(srcs[k], device="cuda") for k in range(64)]
    b = tdp.Batch([op], [64])
    depth = args.tb_depth or 8
    b.set_tuning(depth, args.tile, args.medium_tile)
    src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)                       # plain copy: 256 MiB read + 256 MiB written
    b.precond(Fs, [base.periods], args.rho)                             # warm (graph)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.profile_batched):
        b.precond(Fs, [base.periods], args.rho)
    torch.cuda.synchronize()
    apply_ms = (time.perf_counter() - t) * 1e3 / args.profile_batched
    launches = -(-base.periods * op.nP // depth)
    print(json.dumps({"mode": "profile_batched", "fields": 64, "N": base.N,
                      "tuning": {"depth": depth, "tile": args.tile, "medium_tile": args.medium_tile},
                      "launches_per_apply": launches, "apply_ms": apply_ms,
                      "us_per_launch": apply_ms * 1e3 / launches}), flush=True)
    b.close()


def form_batched(rho):
    """Batched form: 64 right-hand sides (seeded unit sources) on one 512^2
    smooth medium plus 32 independent problems of sizes 128..768 per side,
    FP32 fields / FP64 GMRES, all in one batched launch sequence.  Also the 64
    right-hand sides alone, on the shared-medium tile and on per-field tiles,
    against the plain single-solve FP32 and FP64 paths on a sample of the
    same fields."""
    import torch
    from paper_2006_16861_amd import inputs, tdp
    base = inputs.smooth2d(512, seed=4, src_seed=5)
    srcs = inputs.random_sources(base.n, 64, seed=5, margin=32)
    uneven = inputs.uneven_problems()
    probs = [base] + uneven
    nrhs = [64] + [1] * len(uneven)
    T = [p.periods for p in probs]
    ops = [tdp.operator_from_problem(p, prec=tdp.F32) for p in probs]
    Fs = [torch.as_tensor(srcs[k], device="cuda") for k in range(64)] + \
         [torch.as_tensor(p.F, device="cuda") for p in uneven]
    field_N = [base.N] * 64 + [p.N for p in uneven]

    def timed_solve(b, fs, field_n, Tb):
        b.solve(fs, Tb, rho=rho, tol=1e-6)                               # warm (graphs)
        (out, dt) = _timed(lambda: b.solve(fs, Tb, rho=rho, tol=1e-6))
        Us, infos, rc = out
        steps = sum(i.steps * n for i, n in zip(infos, field_n))
        return {"solves_per_s": len(fs) / dt, "seconds": dt, "status": rc,
                "worst_relres": max(i.relres for i in infos),
                "node_steps_per_s": steps / dt, "fields": len(fs),
                "iters_max": max(i.iters for i in infos)}, infos

    b = tdp.Batch(ops, nrhs)
    t = time.perf_counter()
    table = b.autotune([max(1, t_ // 8) for t_ in T], rho=rho)
    best = min(table, key=lambda r: r[3])
    log(f"form batched: autotune {len(table)} variants in {time.perf_counter() - t:.2f} s, "
        f"best depth {int(best[0])} tile {int(best[1])} shared tile {int(best[2])}")
    b.set_tuning(int(best[0]), int(best[1]), int(best[2]))
    res = {"workload": "64 rhs on smooth2d-512 + 32 uneven 128..768", "fields": len(Fs),
           "tuning": {"depth": int(best[0]), "tile": int(best[1]), "medium_tile": int(best[2])},
           "total_nodes": sum(field_N)}
    r_all, infos_all = timed_solve(b, Fs, field_N, T)
    res.update(r_all)
    fo = [0] * 64 + list(range(1, len(probs)))
    handoff = {"problem": base, "fields": [(i.steps // (T[fo[q]] * ops[fo[q]].nP), field_N[q],
                                            T[fo[q]], ops[fo[q]].nP)
                                           for q, i in enumerate(infos_all)]}
    log(f"form batched: {len(Fs)} solves in {res['seconds']:.3f} s, worst relres {res['worst_relres']:.2e}")
    b.close()

    # the 64 right-hand sides of one medium alone: shared-medium tile against
    # per-field tiles, and the kernel launch time of one batched application
    b64 = tdp.Batch([ops[0]], [64])
    tab64 = b64.autotune([max(1, T[0] // 8)], rho=rho)
    # best of each kind (every field on its own tile: medium_tile -1)
    shared = min((r for r in tab64 if r[2] >= 0), key=lambda r: r[3])
    single = min((r for r in tab64 if r[2] < 0), key=lambda r: r[3])
    sub = {}
    for name, r in (("shared_medium_tile", shared), ("per_field_tiles", single)):
        b64.set_tuning(int(r[0]), int(r[1]), int(r[2]))
        sub[name] = timed_solve(b64, Fs[:64], field_N[:64], T[:1])[0]
        sub[name]["tuning"] = {"depth": int(r[0]), "tile": int(r[1]), "medium_tile": int(r[2])}
    b64.set_tuning(int(shared[0]), int(shared[1]), int(shared[2]))
    U64 = b64.precond(Fs[:64], T[:1], rho)                             # warm
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        b64.precond(Fs[:64], T[:1], rho)
    e1.record()
    torch.cuda.synchronize()
    app_ms = e0.elapsed_time(e1) / 3
    K = int(shared[0])
    launches = -(-T[0] * ops[0].nP // K)
    nr = {0: 4, 1: 2, 2: 2}[int(shared[2])]
    slabs = -(-64 // nr)
    # per launch: each right-hand side reads u_j, u_{j-1} and F and writes two
    # fields (6 words per node); the medium (m, damping) is read once per slab
    alg_bytes = 4 * base.N * (6 * 64 + 2 * slabs)
    launch_us = app_ms * 1e3 / launches
    sub["shared_medium_tile"]["roofline"] = roofline_block(
        f"k_sweep2d_tb_mrhs<float> medium tile {int(shared[2])} ({nr} right-hand sides per "
        f"workgroup) depth={K}", launch_us, alg_bytes,
        flops_per_node_step(2, 9) * base.N * 64 * K, 4,
        traffic=_traffic(f"batch64-smooth2d-512|f32|v0|kmrhs|d{K}|t{int(shared[2])}"),
        effective_bytes=4 * base.N * 64 * (5 + 2.0 / 64) * K,
        note="launch time = one batched application (HIP events) / its launches; "
             "effective bytes: (5 + 2/64) words per right-hand side per node-step")
    sub["shared_medium_tile"]["application_ms"] = app_ms
    sub["speedup_shared_vs_per_field_tiles"] = (sub["shared_medium_tile"]["node_steps_per_s"] /
                                                sub["per_field_tiles"]["node_steps_per_s"])
    res["rhs64_on_one_medium"] = sub
    b64.close()
    log(f"form batched 64 rhs: shared tile {sub['shared_medium_tile']['node_steps_per_s']:.3g} "
        f"node-steps/s, per-field tiles {sub['per_field_tiles']['node_steps_per_s']:.3g}")

    # the plain single-solve paths on a sample of the same fields
    sample = [0, 1, 64, 65]
    for name, prec in (("f32", tdp.F32), ("f64", tdp.F64)):
        t_single, steps_single = 0.0, 0.0
        for q in sample:
            p = base if q < 64 else uneven[q - 64]
            op = tdp.operator_from_problem(p, prec=prec)
            op.solve(Fs[q], T=p.periods, rho=rho, tol=1e-6)
            ((_, info), dt1) = _timed(lambda: op.solve(Fs[q], T=p.periods, rho=rho, tol=1e-6))
            w = (64 if q < 64 else len(uneven)) / 2
            t_single += dt1 * w
            steps_single += info.steps * p.N * w
            del op
        res[f"plain_{name}_single_solves_per_s_extrapolated"] = len(Fs) / t_single
        res[f"plain_{name}_single_node_steps_per_s"] = steps_single / t_single
        res[f"speedup_vs_plain_{name}"] = res["solves_per_s"] / (len(Fs) / t_single)
    res["plain_sample"] = "2 of the 64 sources and 2 of the 32 uneven problems, each solved " \
                          "alone, scaled to all 96 fields"
    return res, handoff


def abd_roofline(p, tun, us_step, word, prec):
    """Roofline of the I_abd sweep's launch.  Blocked (kernel 2): one launch
    runs k complex steps (both real parts of the field), so it lasts
    us_step * k; it must read x_n, x_{n-1} (complex), the cell slowness, the
    cell damping and F (complex) and write x_{n+k}, x_{n+k-1} (complex): 12
    words per node.  Flops per real node-step follow flops_per_node_step over
    the 9 points of A and the 5 of B (34), twice per complex node-step.  One
    step per launch (kernel 1): 10 words and 68 flops per node."""
    flops = 2 * flops_per_node_step(2, 9 + 5)
    traffic = measured_traffic("smooth2d-1024", prec, 1, tun, "cell")
    if tun["kernel"] == 2:
        K = tun["tb_depth"]
        kname = (f"k_sweep2d_abd_tb2<{'double' if word == 8 else 'float'}> tile={tun['tile']} "
                 f"depth={K} (both real parts, {K} steps per launch)")
        return roofline_block(kname, us_step * K, 12 * word * p.N, flops * K * p.N, word,
                              traffic=traffic, effective_bytes=10 * word * p.N * K,
                              effective_label="10word")
    return roofline_block("k_sweep_abd (one complex step per launch)", us_step, 10 * word * p.N,
                          flops * p.N, word, traffic=traffic)


def form_cell_damping(rho):
    """Sec. 6 path on the headline workload: smooth2d-1024 with the cell
    (non-diagonal) damping Im H = omega sum_cells r_cell M_cell, preconditioned
    by S_T^abd (I_abd), to a true relative residual of 1e-6, with FP64 and with
    FP32 recurrence fields (GMRES, H and the residuals in FP64 either way), on
    the autotuner's sweep (blocked 2-D I_abd or one step per launch).  Rates use
    10 words per complex node-step (u_n, u_{n-1} and F complex, the two cell
    arrays, u_{n+1} complex)."""
    import torch
    from paper_2006_16861_amd import inputs, tdp
    p = inputs.smooth2d(1024)
    F = torch.as_tensor(p.F, device="cuda")
    res = {"workload": "smooth2d-1024, cell damping (Sec. 6, I_abd)"}
    for name, prec in (("f64", tdp.F64), ("f32", tdp.F32)):
        op = tdp.operator_from_problem(p, damping="cell", prec=prec)
        op.autotune(T=4, rho=rho, variant=1)
        op.solve(F, T=p.periods, rho=rho, tol=1e-6)                     # warm (graph)
        (U, info), dt = _timed(lambda: op.solve(F, T=p.periods, rho=rho, tol=1e-6))
        r = float(torch.linalg.norm(F - op.apply_H(U)) / torch.linalg.norm(F))
        _, step_ms = sweep_timing(op, F, p.periods, rho, 1, torch.cuda.current_stream(), variant=1)
        us = step_ms * 1e3
        word = 8 if prec == tdp.F64 else 4
        log(f"form cell damping {name}: {dt:.3f} s, iters {info.iters}, relres {r:.2e}, "
            f"{us:.2f} us/step")
        tun = op.get_tuning()
        res[name] = {"n_P": op.nP, "omega_c": op.omega_c, "solves_per_s": 1.0 / dt,
                     "seconds": dt, "iters": info.iters,
                     "precond_applications": info.steps // (p.periods * op.nP), "true_relres": r,
                     "sweep_us_per_step": us, "tuning": tun,
                     "sweep_algorithmic_GBps": 10 * word * p.N / (us * 1e-6) / 1e9,
                     "roofline": abd_roofline(p, tun, us, word, name)}
        del op
    return res


def form_adjoint(rho):
    """Differentiation form: 128^3 smooth medium in [1.5, 3.0], 4 sources, 256
    receivers on the top face, misfit 1/2 ||P_r U(m) - d||^2; one gradient
    evaluation = 4 forward + 4 adjoint solves to 1e-6, at n_P = 10 (the
    smallest integer above the CFL bound at 8 ppw)."""
    import torch
    from paper_2006_16861_amd import inputs, tdp
    from paper_2006_16861_amd.autograd import helmholtz_solve
    p = inputs.smooth3d(128, width=16)
    F = torch.as_tensor(inputs.sources_on_plane(p.n, 4, seed=8, plane=18), device="cuda")
    mask = torch.as_tensor(inputs.receiver_mask(p.n, plane=17, per_side=16).astype(np.float64),
                           device="cuda")
    m0 = 1.0 / p.c ** 2
    m_true = m0 * (1.0 + 0.05 * inputs.gaussian_blob(p.n, seed=9))
    R = torch.as_tensor(p.R, device="cuda")
    with torch.no_grad():
        d = helmholtz_solve(torch.as_tensor(m_true, device="cuda"), F, R, p.omega, p.h,
                            T=p.periods, tol=1e-6, steps_per_period=-1) * mask

    def grad_eval():
        m = torch.as_tensor(m0, device="cuda").clone().requires_grad_(True)
        U = helmholtz_solve(m, F, R, p.omega, p.h, T=p.periods, tol=1e-6, steps_per_period=-1)
        L = 0.5 * (((U - d) * mask).abs() ** 2).sum()
        L.backward()
        return m.grad

    grad_eval()
    g, dt = _timed(grad_eval)
    log(f"form adjoint: gradient in {dt:.3f} s")
    # preconditioner applications of the forward solves (the adjoint solves
    # use the same operator and right-hand sides of the same kind)
    op = tdp.Operator(torch.rsqrt(torch.as_tensor(m0, device="cuda")).contiguous(), R, p.omega,
                      p.h, steps_per_period=-1)
    napply = []
    Fs = [F[s_].contiguous() for s_ in range(F.shape[0])]
    for Fk in Fs:
        _, info = op.solve(Fk, T=p.periods, tol=1e-6)
        napply.append(info.steps // (p.periods * op.nP))
    # the plain FP64 GPU path on the same configuration: the forward solves
    # alone, without autograd, the adjoint solves and the gradient kernels
    _, dt_plain = _timed(lambda: [op.solve(Fk, T=p.periods, tol=1e-6) for Fk in Fs])
    res = {"workload": "smooth3d-128, 4 sources, 256 receivers", "gradients_per_s": 1.0 / dt,
           "solves_per_s": 8.0 / dt, "seconds": dt, "grad_norm": float(torch.linalg.norm(g)),
           "forward_precond_applications": napply,
           "plain_f64_solves_per_s": len(Fs) / dt_plain,
           "solves_per_s_vs_plain_f64": (8.0 / dt) / (len(Fs) / dt_plain)}
    return res, {"problem": p, "n_P": op.nP, "napply_per_gradient": 2 * sum(napply)}


XGMI_LINK_GBS = 153.0           # one MI355X xGMI link, one direction, published


def study_shard(ngpu=8, rho=0.25):
    """One GPU's share of a slab decomposition along axis 0 over `ngpu` GPUs:
    the sweep at the slab's real shape (its interior plus the halo planes the
    kernel needs), against 1/ngpu of the full-grid step, and the halo each step
    (or block of k steps) would exchange with each neighbour: bytes, the time
    of one device copy of it (the staging cost, if a staging buffer is used;
    slabs along axis 0 have contiguous faces, so none is needed) and its time on
    one xGMI link at the published rate.  Nothing here moves data between GPUs."""
    import torch
    from paper_2006_16861_amd import inputs, tdp
    out = {"study": "shard", "gpus_modelled": ngpu, "xgmi_link_GBps": XGMI_LINK_GBS}

    def slab_op(p, lo, hi, prec, spp):
        sl = slice(lo, hi)
        c = torch.as_tensor(np.ascontiguousarray(p.c[sl]), device="cuda")
        R = torch.as_tensor(np.ascontiguousarray(p.R[sl]), device="cuda")
        F = torch.as_tensor(np.ascontiguousarray(p.F[sl]), device="cuda")
        op = tdp.Operator(c, R, p.omega, p.h, prec=prec, steps_per_period=spp)
        op._keep = (c, R)
        return op, F

    def step_us(op, F, T):
        best, _ = op.autotune(T=4, rho=rho)
        ms, step_ms = sweep_timing(op, F, T, rho, 3, torch.cuda.current_stream())
        return step_ms * 1e3, best

    def copy_us(nbytes):
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        b.copy_(a)
        e0.record()
        for _ in range(20):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 20 * 1e3

    # 3-D: layered3d-256, slabs of 256/ngpu planes, one halo plane per side for
    # the one-step kernels, two for the two-step kernel
    p = inputs.layered3d(256)
    own = p.n[0] // ngpu
    lo = p.n[0] // 2 - own // 2
    res3 = {"workload": "layered3d-256", "slab_planes": own}
    for name, prec in (("f64", tdp.F64), ("f32", tdp.F32)):
        word = 8 if prec == tdp.F64 else 4
        full_op, Ff = slab_op(p, 0, p.n[0], prec, -1)
        full_us, full_best = step_us(full_op, Ff, p.periods)
        del full_op, Ff
        torch.cuda.empty_cache()
        r = {"full_grid_us_per_step": full_us, "full_grid_tuning": full_best}
        for halo in (1, 2):
            op, F = slab_op(p, lo - halo, lo + own + halo, prec, -1)
            us, best = step_us(op, F, p.periods)
            r[f"halo{halo}"] = {"grid": list(op.n), "us_per_step": us, "tuning": best,
                                "vs_ideal": (full_us / ngpu) / us}
            del op, F
            torch.cuda.empty_cache()
        face = p.n[1] * p.n[2] * word
        r["face_bytes"] = face
        r["face_copy_us"] = copy_us(face)
        r["face_xgmi_us"] = face / (XGMI_LINK_GBS * 1e3)
        res3[name] = r
        log(f"shard 3-D {name}: full {full_us:.1f} us/step, slab {r['halo1']['us_per_step']:.1f} "
            f"us/step, face {face >> 10} KiB ({r['face_xgmi_us']:.2f} us on one link)")
    out["3d"] = res3

    # 2-D: smooth2d-1024, slabs of 1024/ngpu rows; the blocked kernel of depth k
    # needs k halo rows per side and one exchange every k steps
    p = inputs.smooth2d(1024)
    own = p.n[0] // ngpu
    lo = p.n[0] // 2 - own // 2
    full_op, Ff = slab_op(p, 0, p.n[0], tdp.F64, 0)
    full_us, full_best = step_us(full_op, Ff, p.periods)
    del full_op, Ff
    res2 = {"workload": "smooth2d-1024", "slab_rows": own, "full_grid_us_per_step": full_us,
            "full_grid_tuning": full_best}
    for k in (4, 8):
        op, F = slab_op(p, lo - k, lo + own + k, tdp.F64, 0)
        op.set_tuning(kernel=2, tb_depth=k, tile=5)
        ms, step_ms = sweep_timing(op, F, p.periods, rho, 3, torch.cuda.current_stream())
        face = k * p.n[1] * 8
        res2[f"depth{k}"] = {"grid": list(op.n), "us_per_step": step_ms * 1e3,
                             "vs_ideal": (full_us / ngpu) / (step_ms * 1e3),
                             "face_bytes_per_exchange": face,
                             "face_xgmi_us": face / (XGMI_LINK_GBS * 1e3),
                             "compute_us_between_exchanges": k * step_ms * 1e3}
        del op, F
    out["2d"] = res2
    log(f"shard 2-D: full {full_us:.2f} us/step; slab {res2['depth8']['us_per_step']:.2f} us/step")
    print(json.dumps(out), flush=True)


def study_convergence(model, Ts=(10, 20, 40, 80, 160, 320), rhos=(0.0, 0.25, 0.5, 0.75),
                      gmres_Ts=(5, 10, 20, 40, 80), ref_tol=1e-12):
    """Sec. 5.1's convergence studies on the constant model and the resonant disc
    model (6 points per wavelength, 8 steps per period, 32-node damping layers):
    (a) the relative error of S_T F against H^-1 F as T grows, for each taper rho
        (rho = 0: the forcing ramps up over one period);
    (b) preconditioned GMRES (rho = 0.25) to a true relative residual of 1e-6 for
        several T: iterations, total periods (one application per iteration plus
        the one for the right-hand side) and the error against H^-1 F, next to the
        direct application S_T F of the sweep in (a).
    H^-1 F is the GMRES solution at true relative residual ref_tol."""
    import torch
    from paper_2006_16861_amd import inputs, tdp
    out = {"study": "convergence", "model": model, "ppw": 6.0, "layer": 32}
    for mk in (inputs.open2d, inputs.disc2d):
        p = mk(model)
        op = tdp.operator_from_problem(p)
        F = torch.as_tensor(p.F, device="cuda")
        t0 = time.perf_counter()
        Uref, iref = op.solve(F, T=p.periods, tol=ref_tol, max_iters=20000)
        log(f"study {p.name}: n={p.n} omega={p.omega:.1f} n_P={op.nP}; reference: "
            f"{iref.iters} its, relres {iref.relres:.1e}, {time.perf_counter() - t0:.1f} s")
        nref = float(torch.linalg.norm(Uref))
        err = lambda U: float(torch.linalg.norm(U - Uref)) / nref
        res = {"n": list(p.n), "omega": p.omega, "n_P": op.nP,
               "reference": {"iters": iref.iters, "relres": iref.relres}}
        direct = {}
        for rho in rhos:
            row = []
            for T in Ts:
                row.append(err(op.precond(F, T, rho)))
            direct[str(rho)] = dict(zip(map(str, Ts), row))
            log(f"  S_T F error, rho={rho:<4}: " + "  ".join(f"T={T}:{e:.1e}" for T, e in zip(Ts, row)))
        res["precond_error"] = direct
        gm = {}
        for T in gmres_Ts:
            U, info = op.solve(F, T=T, rho=0.25, tol=1e-6, max_iters=5000)
            periods = info.steps // op.nP
            gm[str(T)] = {"iters": info.iters, "restarts": info.restarts, "periods": int(periods),
                          "relres": info.relres, "error": err(U), "status": info.status}
            log(f"  GMRES T={T:<4}: {info.iters:4d} its, {periods:6d} periods, relres "
                f"{info.relres:.1e}, error {err(U):.1e}")
        res["gmres"] = gm
        out[p.name] = res
        del op
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="smooth2d-1024")
    ap.add_argument("--prec", choices=["f64", "f32"], default="f64")
    ap.add_argument("--rho", type=float, default=0.25)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--periods", type=int, default=0,
                    help="T, periods per preconditioner application (0: the workload's, "
                         "about the model size in wavelengths)")
    ap.add_argument("--steps-per-period", type=int, default=0,
                    help="n_P: 0 the smallest multiple of 4 above the CFL bound (Table 1), "
                         "-1 the smallest integer >= 3 above it (Im U by the 2x2 solve)")
    ap.add_argument("--scheme", choices=["compact", "fd2", "q1"], default="compact",
                    help="fd2: the second-order 5-/7-point scheme of Sec. 3.1 instead of the "
                         "compact fourth-order one; q1: bilinear / trilinear elements (all 27 "
                         "points in 3-D)")
    ap.add_argument("--damping", choices=["node", "cell"], default="node",
                    help="cell: the non-diagonal damping of Sec. 6 (I_abd; needs --variant 1)")
    ap.add_argument("--variant", type=int, default=0,
                    help="0: Table 1 real-field preconditioner, 1: Definition 4 complex field")
    ap.add_argument("--kernel", type=int, default=0)
    ap.add_argument("--tb-depth", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--sweep-reps", type=int, default=3)
    ap.add_argument("--tune-only", action="store_true",
                    help="print the autotuner's per-variant step times and exit")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the precision / batched / adjoint form measurements")
    ap.add_argument("--forms", default="",
                    help="comma list of forms to measure (precision, batched, adjoint, "
                         "cell_damping); default all")
    ap.add_argument("--profile-sweeps", type=int, default=0,
                    help="profiling mode: one 256 MiB device copy (counter calibration), then "
                         "this many preconditioner applications, then exit")
    ap.add_argument("--profile-batched", type=int, default=0,
                    help="profiling mode for the batched form: one 256 MiB device copy, then this "
                         "many applications of the 64 right-hand sides on one 512^2 medium (FP32 "
                         "fields) with --tb-depth, --tile and --medium-tile, then exit")
    ap.add_argument("--medium-tile", type=int, default=1,
                    help="shared-medium tile of --profile-batched (-1: every field on its own tile)")
    ap.add_argument("--study", choices=["convergence", "shard"], default=None,
                    help="convergence: Sec. 5.1's convergence study on the constant and "
                         "resonant models; shard: the sweep at one GPU's slab of an 8-GPU "
                         "decomposition, with its halo sizes (instead of the benchmark)")
    ap.add_argument("--study-model", type=int, default=320,
                    help="model size (nodes per axis, without the damping layers)")
    args = ap.parse_args()
    if args.study == "convergence":
        study_convergence(args.study_model)
        return
    if args.study == "shard":
        study_shard()
        return
    if args.profile_batched:
        profile_batched(args)
        return
    if args.damping == "cell" and args.variant != 1:
        raise SystemExit("--damping cell runs S_T^abd: pass --variant 1")
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "slab decomposition is a design note, not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2006_16861_amd import tdp

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log(f"workload {args.workload}: generating inputs")
    p = make_problem(args.workload)
    prec = tdp.F64 if args.prec == "f64" else tdp.F32
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        t = time.perf_counter()
        op = tdp.operator_from_problem(p, prec=prec, damping=args.damping,
                                       scheme=None if args.scheme == "compact" else args.scheme,
                                       steps_per_period=args.steps_per_period)
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t) * 1e3
        tune_table = []
        if args.kernel == 0 and not args.no_graph:
            t = time.perf_counter()
            # 2-D: candidates timed over a whole application (the resident
            # kernel's per-launch set-up and its check after each application
            # are spread over the real number of steps); 3-D over four periods
            T_tune = (args.periods if args.periods > 0 else p.periods) if len(p.n) == 2 else 4
            best, tune_table = op.autotune(T=T_tune, rho=args.rho, variant=args.variant)
            log(f"autotune ({(time.perf_counter() - t) * 1e3:.0f} ms): best {best}")
            for row in tune_table:
                log(f"   kernel={int(row[0])} depth={int(row[1])} tile={int(row[2])}: "
                    f"{row[3]:.2f} us/step")
            if args.tune_only:
                return
        else:
            op.set_tuning(kernel=args.kernel, tb_depth=args.tb_depth, tile=args.tile,
                          use_graph=0 if args.no_graph else 1)
        T = args.periods if args.periods > 0 else p.periods
        Ns = T * op.nP
        F = torch.as_tensor(p.F, device="cuda")
        if args.profile_sweeps:
            src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
            dst = torch.empty_like(src)
            dst.copy_(src)                       # plain copy: 256 MiB read + 256 MiB written
            torch.cuda.synchronize()
            apply_ms, step_ms = sweep_timing(op, F, T, args.rho, args.profile_sweeps, stream,
                                             args.variant)
            tun = op.get_tuning()
            per = {2: tun["tb_depth"], 4: 2, 5: RES_MAX_STEPS}.get(tun["kernel"], 1)
            launches = -(-Ns // per)
            if args.variant == 1 and tun["kernel"] != 1 and not (args.damping == "cell"
                                                                  and tun["kernel"] == 2):
                launches *= 2                    # two real passes (one launch for both: I_abd)
            print(json.dumps({"mode": "profile", "workload": args.workload, "N": p.N,
                              "N_s": Ns, "tuning": tun, "launches_per_apply": launches,
                              "apply_ms": apply_ms, "us_per_step": step_ms * 1e3,
                              "us_per_launch": apply_ms * 1e3 / launches}), flush=True)
            return
        log(f"n={p.n} N={p.N} n_P={op.nP} T={T} N_s={Ns} setup {setup_ms:.1f} ms")
        infos = []
        for w in range(args.warmup):
            U, info = op.solve(F, T=T, rho=args.rho, tol=args.tol, restart=args.restart,
                               variant=args.variant)
            log(f"warmup {w}: iters={info.iters} relres={info.relres:.3e} {info.ms_total:.1f} ms")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            U, info = op.solve(F, T=T, rho=args.rho, tol=args.tol, restart=args.restart,
                               variant=args.variant)
            infos.append(info)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        for k, info in enumerate(infos):
            log(f"step {k}: status={info.status} iters={info.iters} relres={info.relres:.3e} "
                f"{info.ms_total:.1f} ms")
            if info.status != 0 or info.relres > args.tol:
                raise SystemExit(f"solve {k} did not reach tol: {info}")
        # true residual of the last solve, recomputed with the library's H in FP64
        r = F - op.apply_H(U)
        relres = float(torch.linalg.norm(r) / torch.linalg.norm(F))
        log(f"timed {args.steps} solves in {wall:.3f} s; last true relres {relres:.3e}")
        apply_ms, step_ms = sweep_timing(op, F, T, args.rho, args.sweep_reps, stream,
                                         args.variant)
    word = 8 if prec == tdp.F64 else 4
    words = WORDS_PER_NODE_STEP if args.variant == 0 else 10
    bytes_per = words * word
    tun = op.get_tuning()
    blocked = tun["kernel"] == 2
    steps_per_launch = {2: tun["tb_depth"], 4: 2, 5: min(RES_MAX_STEPS, Ns)}.get(tun["kernel"], 1)
    launches = -(-Ns // steps_per_launch)
    paired = args.damping == "cell" and tun["kernel"] == 2     # I_abd: both parts per launch
    if args.variant == 1 and tun["kernel"] != 1 and not paired:
        launches *= 2                            # Def. 4: two real passes
    napply = infos[-1].steps // Ns
    # average launch duration over the timed solves: the GPU time of their
    # preconditioner applications (HIP events on the op's stream around each
    # application) over the launches they made; the standalone application
    # (with its staging copies) is reported beside it
    launch_us = float(np.median([i.ms_precond for i in infos])) * 1e3 / (napply * launches)
    standalone_launch_us = apply_ms * 1e3 / launches
    # the per-step 7-word model over the steps of one launch (no reuse across
    # steps; above the HBM peak under temporal blocking)
    effective = p.N * bytes_per * (Ns / launches) / (launch_us * 1e-6) / 1e9
    tname = "double" if prec == tdp.F64 else "float"
    if paired:
        kname = (f"k_sweep2d_abd_tb2<{tname}> depth={steps_per_launch} tile={tun['tile']} "
                 "(I_abd, both real parts per launch)")
    elif args.damping == "cell":
        kname = f"k_sweep_abd<{tname}> (I_abd, one step per launch)"
    elif tun["kernel"] == 2:
        kname = (f"k_sweep2d_{'tb2' if tun['tile'] >= 4 else 'tb'}<{tname}> "
                 f"depth={steps_per_launch} tile={tun['tile']}")
    elif tun["kernel"] == 5:
        kname = (f"k_sweep2d_res<{tname}> exchange depth={tun['tb_depth']} "
                 f"(resident tiles, launches of up to {RES_MAX_STEPS} steps)")
    elif tun["kernel"] == 3:
        kname = f"k_sweep3d_stream<{tname}> shape={tun['tile']} z-chunk={tun['tb_depth']}"
    elif tun["kernel"] == 4:
        kname = f"k_sweep3d_stream2<{tname}> shape={tun['tile']} z-chunk={tun['tb_depth']} (2 steps)"
    else:
        kname = f"k_sweep<{tname}> (one step per launch)"
    # the counters were taken with the compact scheme
    # per-launch counters do not depend on n_P; they do on the stencil tables
    traffic = measured_traffic(args.workload, args.prec, args.variant, tun, args.damping,
                               args.scheme)
    ceiling = stream_probe()
    log(f"stream probe: copy {ceiling['copy']:.0f} GB/s, triad {ceiling['triad']:.0f} GB/s")
    # bytes one launch must move: a blocked or two-step launch reads u_j,
    # u_{j-1}, m, the damping factor and F once and writes two fields (8 words
    # per node); the blocked I_abd launch reads both parts of x_n and x_{n-1},
    # the two cell arrays and F and writes both parts of two fields (12); a
    # one-step launch moves the 7 words of one step; Def. 4 on the complex
    # field in one pass moves 10
    spl = Ns / launches
    cell = args.damping == "cell"
    if paired:
        words_launch = 12
    elif tun["kernel"] in (2, 4, 5):
        words_launch = WORDS_PER_NODE_LAUNCH
    else:
        words_launch = 10 if (args.variant == 1 and tun["kernel"] == 1) else WORDS_PER_NODE_STEP
    points = {("compact", 2): 9, ("fd2", 2): 5, ("q1", 2): 9, ("compact", 3): 19, ("fd2", 3): 7,
              ("q1", 3): 27}[(args.scheme, len(p.n))]
    if cell:
        points += 5 if len(p.n) == 2 else 7           # the damping stencil of I_abd
    flops = flops_per_node_step(len(p.n), points) * (
        2 if args.variant == 1 and (tun["kernel"] == 1 or paired) else 1)
    roof = roofline_block(kname, launch_us, p.N * word * words_launch, flops * p.N * spl, word,
                          traffic=traffic, effective_bytes=p.N * bytes_per * spl)
    log(f"precond apply {apply_ms:.3f} ms, {step_ms * 1e3:.2f} us/step; launch {launch_us:.2f} us: "
        f"bound {roof['bound']} ({roof['roof']} {roof['frac']:.3f}), effective {effective:.0f} GB/s")
    out = {
        "metric": "Helmholtz solves/s at 1e-6 residual; recurrence-step GB/s vs HBM peak",
        "value": args.steps / wall,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == tdp.F64 else "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "scheme": args.scheme, "n": list(p.n), "h": p.h,
                   "omega": p.omega,
                   "ppw": p.ppw, "damping_width": p.width, "periods_T": T, "n_P": op.nP,
                   "N_s": Ns, "rho": args.rho, "variant": args.variant, "restart": args.restart, "tol": args.tol,
                   "gmres_iters": infos[-1].iters, "gmres_restarts": infos[-1].restarts,
                   "switched": [int(i.switched) for i in infos],
                   "precond_applications": int(napply),
                   "true_relres": relres, "setup_ms": setup_ms,
                   "solve_ms": [round(i.ms_total, 3) for i in infos],
                   "precond_ms": [round(i.ms_precond, 3) for i in infos],
                   "H_ms": [round(i.ms_H, 3) for i in infos],
                   "arnoldi_ms": [round(i.ms_arnoldi, 3) for i in infos],
                   "solve_ms_median": float(np.median([i.ms_total for i in infos])),
                   "kernel": op.get_tuning(), "parallelism": "single-gpu"},
        "recurrence_GBps_7word": effective,
        "roofline": dict(roof, **{
            "words_per_node_launch": words_launch, "word_bytes": word,
            "bytes_per_node_step_7word": bytes_per, "nodes_per_launch": p.N,
            "steps_per_launch": spl, "flops_per_node_step": flops,
            "avg_launch_us_source": "HIP events around the preconditioner applications of "
                                    "the timed solves",
            "standalone_launch_us": standalone_launch_us,
            "measured_ceiling_GBps": ceiling}),
    }
    handoff = {}
    if not args.no_forms and args.workload == "smooth2d-1024":
        forms = {}
        chosen = set(args.forms.split(",")) if args.forms else None
        for name, fn in (("precision", form_precision), ("batched", form_batched),
                         ("adjoint", form_adjoint), ("cell_damping", form_cell_damping)):
            if chosen is not None and name not in chosen:
                continue
            log(f"form {name} ...")
            r = fn(args.rho)
            if isinstance(r, tuple):
                forms[name], handoff[name] = r
            else:
                forms[name] = r
            torch.cuda.empty_cache()
        out["forms"] = forms
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(p, T, args.rho, int(napply), workload=args.workload,
                                           handoff=handoff)
        # the oracle's checks of the forms' GPU results go back beside them
        for name, leg in out["cpu_baseline"].get("legs", {}).items():
            if "oracle_check" in leg and name in out.get("forms", {}):
                out["forms"][name]["oracle_check"] = leg["oracle_check"]
        log(f"cpu baseline {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
