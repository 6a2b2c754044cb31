"""bench.py's output contract, run as the benchmark is run (a child process,
one JSON line on stdout): the required keys, a roofline record for the
dominant kernel with achieved / peak = frac, the measured HBM traffic when the
profiled kernel sources are unchanged, the copy ceiling, the ensemble and
served sub-records, and the CPU-oracle baselines (all host cores and one)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                       capture_output=True, text=True, timeout=420)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1, r.stdout
    return json.loads(lines[0])


def test_default_line():
    d = _run("--steps", "200", "--warmup", "10", "--cpu-steps", "1", "--cpu-all-steps", "1",
             "--ensemble-steps", "20", "--served-requests", "6", "--served-time-limit", "15")
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 200 and d["unit"] == "MLUPS" and d["value"] > 0
    assert d["config"]["workload"] == "bulk_4096x4096_fp32" and d["dtype"] == "f32"
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["peak"] == 8000.0 and r["unit"] == "GB/s"
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    import bench
    rec = json.load(open(os.path.join(ROOT, "profiles", "step_kernel_traffic.json")))
    if all(v["kernel_hash"] == bench.kernel_source_hash() for v in rec.values()):
        assert r["traffic"] and 1.0 <= r["traffic"] / r["bytes_per_launch"] < 1.1
    cp = r["copy"]
    assert cp["ceiling_gbs"] == max(cp["memcpy_gbs"], cp["stream_copy_kernel_gbs"]) > 0
    assert abs(r["frac_of_copy"] - r["achieved"] / cp["ceiling_gbs"]) < 1e-3
    e = d["ensemble"]
    assert e["replicas"] == 256 and e["steps"] == 20 and e["mlups"] > 0
    assert abs(e["roofline"]["frac"] - e["roofline"]["achieved"] / 8000.0) < 1e-3
    assert e["sequential"]["mlups"] > 0 and e["speedup_vs_sequential"] > 0
    sv = d["served"]
    assert sv["requests"] == 6 and sv["completed"] + sv["unfinished"] == 6
    assert sv["mlups_active"] > 0 and 0 < sv["roofline"]["frac"] < 1
    assert sv["sequential"] is not None
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["cores"] >= 1 and c["value"] > 0 and c["unit"] == "MLUPS"
    one = c["single_thread"]
    assert one["kind"] == "oracle" and one["cores"] == 1 and one["value"] > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr
