"""bench.py's host-side logic, on the CPU: more than one GPU is refused
before anything else runs, and a sub-record measured in a child process
that fails is reported as an error record with the child's exit status
instead of taking the whole line down."""
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
    args = argparse.Namespace(ensemble_steps=1, served_requests=1, served_time_limit=1.0,
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
