"""The benchmark's command-line contract: one GPU only, and one JSON line with
the fields a reader of the results relies on (metric, throughput, timing,
roofline of the dominant kernel, stage-2 bandwidth)."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_profiled_traffic_reads_the_byte_columns():
    """The traffic figure is the sum of the last two columns of the kernel's
    row in the committed counter summary, or None when the kernel sources
    changed since the counters were taken."""
    sys.path.insert(0, ROOT)
    import bench
    path = os.path.join(ROOT, "profiles", "compile_path_sc_d25_r25_hbm_bytes.txt")
    rows, digest = {}, None
    for line in open(path):
        if line.startswith("# kernel sources digest:"):
            digest = line.split(":", 1)[1].strip()
        elif line.strip() and not line.startswith("#") and not line.startswith("kernel "):
            f = line.split()
            rows[f[0].split("<")[0]] = float(f[-2]) + float(f[-1])
    for k in ("k_sweep", "k_bucket", "k_hash", "k_edge_write"):
        got = bench.profiled_traffic(k, "sc_d25_r25")
        assert got == (rows[k] if digest == bench.kernel_digest() else None), k
    assert bench.profiled_traffic("k_sweep", "no_such_workload") is None


@pytest.mark.gpu
def test_one_json_line_with_the_contract_fields():
    cmd = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--steps", "3", "--warmup", "1", "--latency-iters", "2",
           "--no-cpu-baseline", "--no-grad", "--no-autotune", "--batch-distances=", "--serve-distances=", "--configs=",
           "--table2-iters", "3"]
    print("case bench contract", flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    j = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "stage2"):
        assert k in j, k
    assert j["n_gpus"] == 1 and j["steps"] == 3 and j["warmup"] == 1 and j["value"] > 0
    assert j["config"]["workload"] == "sc_d25_r25" and j["unit"] == "faults/s"
    roof = j["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in roof, k
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-12
    assert 0 < j["stage2"]["frac_algorithmic"] < 1
    t2 = j["paper_table2"]
    assert len(t2) == 21 and {r["level"] for r in t2} == {0, 1, 2}
    for r in t2:
        assert r["faults"] > 0 and r["device_ms_mean"] > 0 and r["whole_path_ms"]["n"] == 3, r["workload"]
    g = j["graph_replay"]
    for mode in ("eager", "graph"):
        assert g[mode]["ms_per_step"] > 0 and g[mode]["single_run_ms_median"] > 0, mode
