"""Throughput of the growing-tissue D2Q9 LBM hot path on one MI355X.

Default workload: a 4096 x 4096 lattice, float32 storage and arithmetic, bulk
growth 1e-4 per step, noise amplitude 1e-3, tissue initially in rows 0-255,
fixed rear wall; the front heights h(x, t) are copied back every 100 steps.
One "step" is one pass of the fused step kernel over the whole lattice (every
site: stream, moments, growth, relax or reverse, noise, negative fix, store,
front heights, mass tallies) -- the full sweep, no windowing.

Prints one JSON line on stdout (progress goes to stderr).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM roofline at 1 GPU; ensemble runs/hour + p50/p99 latency"
HBM_PEAK_GBS = 8000.0
STORE_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16": "f16-offset/f32", "bf16": "bf16-offset/f32"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("lbm_step.hpp", "lbm_device.hpp", "lbm_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2303_02210_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, precision: str):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    key = f"{workload}/{precision}"
    e = rec.get(key)
    if not e or e.get("kernel_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(cfg: dict, steps: int) -> dict:
    """The FP64 oracle, as it stands, on the same lattice for a few steps."""
    from oracle import oracle as orc
    o = orc.Oracle(dict(cfg, precision="fp64"))
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    o.close()
    mlups = cfg["L"] * cfg["H"] * steps / dt / 1e6
    return {"value": round(mlups, 3), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"first {steps} steps of the same {cfg['L']}x{cfg['H']} workload, "
                      f"float64 oracle, single thread, {dt:.1f} s"}


def copy_ceiling(nbytes: int, reps: int = 10) -> float:
    """GB/s of a plain device-to-device copy moving nbytes (read + write) per
    call: the practical HBM ceiling to compare the step kernel with."""
    import torch
    half = nbytes // 2
    src = torch.empty(half // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return 2 * half / dt / 1e9


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", default="fp32", choices=sorted(STORE_BYTES))
    ap.add_argument("--h-every", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported in this build "
              "(the ensemble shards with no communication; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth_inputs as si
    from paper_2303_02210_amd import Sim

    cfg = dict(si.BULK_4096_FP32, precision=args.precision)
    L, H = cfg["L"], cfg["H"]
    bpu = 2 * 9 * STORE_BYTES[args.precision]          # read 9 + write 9 populations

    # warm-up on a scratch run
    sim = Sim(cfg)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    sim.close()
    del sim

    sim = Sim(cfg)
    stream = sim.stream
    torch.cuda.synchronize()
    K, every = args.steps, max(1, args.h_every)
    nchunks = (K + every - 1) // every
    hist = torch.empty((nchunks, L), dtype=torch.int32, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * nchunks + 2)]
    log(f"timing {K} steps of {L}x{H} {args.precision} ...")
    wall0 = time.perf_counter()
    ev[0].record(stream)
    done, k = 0, 0
    while done < K:
        n = min(every, K - done)
        ev[1 + 2 * k].record(stream)
        sim.step(n)
        ev[2 + 2 * k].record(stream)
        sim.front_heights_async(hist[k])
        done += n
        k += 1
    ev[-1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = ev[0].elapsed_time(ev[-1])
    kern_ms = sum(ev[1 + 2 * i].elapsed_time(ev[2 + 2 * i]) for i in range(k))
    d = sim.diagnostics()
    h_last = hist[k - 1].cpu()
    log(f"done: {total_ms:.1f} ms (host wall {wall * 1e3:.1f} ms); hbar {d['hbar']:.2f} "
        f"W {d['W']:.3f} mass {d['mass']:.6g}; h(x) last {int(h_last.min())}..{int(h_last.max())}")

    mlups = L * H * K / (total_ms / 1e3) / 1e6
    per_launch_s = kern_ms / 1e3 / K
    alg_bytes = L * H * bpu
    achieved = alg_bytes / per_launch_s / 1e9
    traffic = measured_traffic(cfg["name"], args.precision)
    ceiling = copy_ceiling(alg_bytes)
    log(f"step kernel {achieved:.0f} GB/s; device copy of the same bytes {ceiling:.0f} GB/s")
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": round(total_ms / K, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[args.precision], "data": "synthetic",
        "config": {"workload": cfg["name"], "L": L, "H": H, "precision": args.precision,
                   "growth": "bulk", "growth_rate": cfg["growth_rate"], "sigma": cfg["sigma"],
                   "init_rows": cfg["init_rows"], "h_every": every, "sweep": "full",
                   "bytes_per_update": bpu},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": "step_kernel", "bytes_per_launch": alg_bytes,
                     "launch_ms": round(per_launch_s * 1e3, 5),
                     "copy_ceiling_gbs": round(ceiling, 1),
                     "frac_of_copy": round(achieved / ceiling, 4)},
        "cpu_baseline": None,
    }
    sim.close()
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle, {args.cpu_steps} steps ...")
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
