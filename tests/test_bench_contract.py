"""bench.py's one-line JSON contract: required fields, units and the
roofline / cpu_baseline objects (GPU), and the refusal of more than one GPU
(CPU: exits before touching a device)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REQUIRED = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
            "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config")


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.gpu
def test_bench_json_line():
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--steps", "1",
                        "--warmup", "0", "--no-forms", "--no-cpu"],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    out = json.loads(r.stdout.strip().splitlines()[-1])
    for k in REQUIRED:
        assert k in out, k
    assert out["unit"] == "solves/s" and out["value"] > 0 and out["n_gpus"] == 1
    assert out["dtype"] == "f64" and out["config"]["workload"] == "smooth2d-1024"
    assert out["config"]["true_relres"] <= 1e-6
    rf = out["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in rf, k
    # frac is a fraction of a real roof: the larger of the HBM fraction of the
    # bytes a launch must move and the ALU fraction of its flops; bound names
    # that roof, or "latency" below half of it
    assert rf["bound"] in ("hbm", "alu", "latency") and rf["roof"] in ("hbm", "alu")
    assert (rf["unit"], rf["peak"]) == (("GB/s", 8000.0) if rf["roof"] == "hbm" else ("TFLOP/s", 78.6))
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) <= 1e-12
    assert 0 < rf["frac"] <= 1 and (rf["bound"] == "latency") == (rf["frac"] < 0.5)
    assert rf["frac"] == max(rf["hbm_frac"], rf["alu"]["frac"])
    launch_s = rf["avg_launch_us"] * 1e-6
    assert abs(rf["hbm_frac"] - rf["algorithmic_bytes_per_launch"] / launch_s / 8e12) <= 1e-9
    # the per-step 7-word model is kept apart from the roofline fraction
    assert rf["effective_GBps_7word"] > 0
    assert out["config"]["switched"] == [0]


def test_traffic_table_is_consistent():
    """profiles/traffic.json: every entry's bytes per launch is its scaled
    FETCH_SIZE + WRITE_SIZE (KiB), and names a committed profile summary."""
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        table = json.load(f)
    assert table
    for key, e in table.items():
        want = e["fetch_kib"] * 1024 * e["fetch_scale"] + e["write_kib"] * 1024 * e["write_scale"]
        # the KiB figures are stored to 0.1 KiB
        assert abs(e["bytes_per_launch"] - want) <= 0.05 * 1024 * (e["fetch_scale"] + e["write_scale"]), key
        assert os.path.exists(os.path.join(ROOT, "profiles", e["profile"])), key
        workload, prec, variant, kern, depth, tile = key.split("|")[:6]
        assert prec in ("f64", "f32") and variant in ("v0", "v1"), key
        assert kern.startswith("k") and depth.startswith("d") and tile.startswith("t"), key
