"""bench.py's host-side logic, on the CPU: more than one GPU is refused
before anything else runs, and a sub-record measured in a child process
that fails is reported as an error record with the child's exit status
instead of taking the whole line down; the served trace's lane mapping
(which batch, on which stream, a request joins)."""
import argparse
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_on_the_host():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "8"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_failed_child_record_is_an_error_record(monkeypatch):
    import bench
    args = argparse.Namespace(ensemble_steps=1, served_requests=1, served_time_limit=1.0, lanes=6,
                              no_sequential=True)
    real = subprocess.run

    def failing(cmd, **kw):
        # the same child, asked for a record kind it does not know (argparse
        # rejects it with status 2)
        cmd = [c if c != "served" else "unknown" for c in cmd]
        return real(cmd, **kw)

    monkeypatch.setattr(subprocess, "run", failing)
    rec = bench.child_record("served", args)
    assert rec == {"error": "child exited with status 2"}


def test_serve_lanes_separate_storage_types_and_widths():
    from paper_2303_02210_amd.serve import lane_index
    types = ("fp64", "fp32", "fp16")
    # one lane per storage type; the 16-bit types share theirs
    assert sorted(lane_index({"precision": p, "L": 256}, 3) for p in types) == [0, 1, 2]
    assert lane_index({"precision": "bf16", "L": 256}, 3) == lane_index({"precision": "fp16", "L": 256}, 3)
    # six lanes split each type by width; every class has its own lane
    six = {lane_index({"precision": p, "L": L}, 6) for p in types for L in (128, 1023, 1024, 4096)}
    assert six == set(range(6))
    # a single lane takes everything
    assert {lane_index({"precision": p, "L": 4096}, 1) for p in types} == {0}
