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
    for f in ("lbm_step.hpp", "lbm_d2q7.hpp", "lbm_device.hpp", "lbm_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2303_02210_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, precision: str, launch: dict):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source and launch shape."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    key = f"{workload}/{precision}"
    e = rec.get(key)
    if not e or e.get("kernel_hash") != kernel_source_hash():
        return None
    if e.get("launch", launch) != launch:
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
                      f"float64 oracle, single thread, {dt:.1f} s, on {_cpu_model()}"}


# One host process of the all-cores baseline: builds its oracle, reports
# "ready", waits for "go" on stdin, steps and prints its elapsed seconds.
_CPU_WORKER = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
from oracle import oracle as orc
cfg, steps = json.loads(sys.argv[2]), int(sys.argv[3])
o = orc.Oracle(cfg)
print("ready", flush=True)
sys.stdin.readline()
t0 = time.perf_counter()
o.step(steps)
print(time.perf_counter() - t0, flush=True)
"""


def host_cores() -> int:
    """Cores this process may use, at most 16 (one GPU's share of its host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline_all_cores(cfg: dict, steps: int, procs: int) -> dict:
    """The same single-threaded oracle on every host core at once: `procs`
    independent processes (each its own copy of the workload, as independent
    runs on a host share it), started together; throughput = all their site
    updates over the slowest one's time."""
    import subprocess
    c = dict(cfg, precision="fp64")
    c = {k: v for k, v in c.items() if isinstance(v, (int, float, str, bool))}
    ps = [subprocess.Popen([sys.executable, "-c", _CPU_WORKER, ROOT, json.dumps(c), str(steps)],
                           stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True)
          for _ in range(procs)]
    for p in ps:
        if p.stdout.readline().strip() != "ready":
            raise RuntimeError("oracle worker failed to start")
    for p in ps:
        p.stdin.write("go\n")
        p.stdin.flush()
    times = [float(p.stdout.readline()) for p in ps]
    for p in ps:
        p.wait()
    dt = max(times)
    mlups = procs * cfg["L"] * cfg["H"] * steps / dt / 1e6
    return {"value": round(mlups, 3), "unit": "MLUPS", "cores": procs, "kind": "oracle",
            "sample": f"{procs} concurrent single-threaded oracle processes, each the first "
                      f"{steps} steps of the same {cfg['L']}x{cfg['H']} workload in float64; "
                      f"slowest {dt:.1f} s, fastest {min(times):.1f} s, on {_cpu_model()}"}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "an unidentified CPU"


def copy_ceiling(nbytes: int, reps: int = 10) -> dict:
    """Device copies moving nbytes (half read, half written) per call: the
    runtime's device-to-device copy (torch's copy_) and the library's
    streaming copy kernel (16-byte nontemporal loads and stores).  The faster
    is the practical HBM ceiling the step kernel is compared with."""
    import ctypes
    import torch
    from paper_2303_02210_amd import _ffi
    half = (nbytes // 2) // 16 * 16
    src = torch.empty(half // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    lib = _ffi.lib()

    def kernel_copy():
        rc = lib.lbm_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                 half, ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise _ffi.LbmError(rc, "lbm_stream_copy")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) / 1e3 / reps)
        return 2 * half / best / 1e9

    memcpy = timed(lambda: dst.copy_(src))
    kern = timed(kernel_copy)
    assert torch.equal(dst, src)
    del src, dst
    return {"memcpy_gbs": round(memcpy, 1), "stream_copy_kernel_gbs": round(kern, 1),
            "ceiling_gbs": round(max(memcpy, kern), 1)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", default="fp32", choices=sorted(STORE_BYTES))
    ap.add_argument("--h-every", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=16)
    ap.add_argument("--cpu-all-steps", type=int, default=6,
                    help="steps per process of the all-cores CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="bulk: skip the 256-replica ensemble figures")
    ap.add_argument("--ensemble-steps", type=int, default=200,
                    help="bulk: steps of the ensemble figures (batched and sequential)")
    ap.add_argument("--no-served", action="store_true",
                    help="bulk: skip the served-trace figures")
    ap.add_argument("--served-requests", type=int, default=40,
                    help="bulk: arrivals of the short served trace")
    ap.add_argument("--served-time-limit", type=float, default=90.0,
                    help="bulk: wall-clock limit of each served-trace run (s)")
    ap.add_argument("--requests", type=int, default=600, help="served: trace length")
    ap.add_argument("--time-limit", type=float, default=300.0, help="served: wall-clock limit (s)")
    ap.add_argument("--lanes", type=int, default=6,
                    help="served: batches by storage type, each on its own stream")
    ap.add_argument("--no-sequential", action="store_true",
                    help="ensemble/served: skip the one-run-at-a-time comparison")
    ap.add_argument("--out", default=None, help="precision: write the curves to this JSON file")
    ap.add_argument("--workload", default="bulk",
                    choices=["bulk", "edge", "ensemble", "served", "precision", "appb", "scaling",
                             "extremes", "dispersion"],
                    help="bulk: 4096 x 4096 bulk growth (default); edge: 2048 x 8192 growth "
                         "within 8 rows of the front; ensemble: 256 replicas of uneven size, "
                         "batched, against the same runs stepped one after another")
    ap.add_argument("--growth", default=None, choices=["bulk", "division", "division_density"],
                    help="bulk / edge: the growth law (default: the workload's own, a "
                         "continuous source); division draws discrete cell divisions per site, "
                         "division_density accepts them with Eq. 5's density weight")
    ap.add_argument("--lattice", default=None, choices=["d2q9", "d2q7"],
                    help="the square D2Q9 lattice or the paper's triangular D2Q7 lattice "
                         "(default: D2Q9 for bulk / edge, D2Q7 for the paper's experiments)")
    ap.add_argument("--sigma", type=float, default=None,
                    help="appb / scaling / extremes / dispersion: noise amplitude in units of "
                         "rho_init (default: the paper's 0.01 on 0.1, i.e. 0.1)")
    ap.add_argument("--tuned", action="store_true", help="launch shapes from the autotuner cache")
    ap.add_argument("--all-batched", action="store_true",
                    help="ensemble: step every member through the batch (no solo members)")
    ap.add_argument("--persistent", action="store_true",
                    help="ensemble: each table group runs a run of steps in one cooperative "
                         "launch (lbm_batch_persistent)")
    ap.add_argument("--stochastic-round", action="store_true",
                    help="bulk / edge with fp16 / bf16 storage: round the stored offsets "
                         "stochastically instead of to nearest")
    ap.add_argument("--shape", default=None, help="force a launch shape: kernel_vb,kernel_ty")
    ap.add_argument("--order", type=int, default=None,
                    help="force the strip dispatch order (kernel_order: 1 wall up, 2 spread)")
    ap.add_argument("--emit-sub", default=None, choices=["ensemble", "served"],
                    help=argparse.SUPPRESS)
    args = ap.parse_args()

    if args.emit_sub:
        # a sub-record of the default line, in its own process
        if args.emit_sub == "ensemble":
            rec = run_ensemble(args.ensemble_steps, 10, tuned=True,
                               sequential=not args.no_sequential)
        else:
            rec = run_served(args.served_requests, args.served_time_limit, tuned=False,
                             sequential=not args.no_sequential, lanes=args.lanes)
        print(json.dumps(rec), flush=True)
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(ensembles shard over GPUs with no communication, one process per GPU)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth_inputs as si
    from paper_2303_02210_amd import Sim

    if args.workload == "ensemble":
        return bench_ensemble(args)
    if args.workload == "served":
        return bench_served(args)
    if args.workload == "precision":
        return bench_precision(args)
    if args.workload == "appb":
        return bench_appb(args)
    if args.workload in ("scaling", "extremes", "dispersion"):
        return {"scaling": bench_scaling, "extremes": bench_extremes,
                "dispersion": bench_dispersion}[args.workload](args)
    args.lattice = args.lattice or "d2q9"
    base = si.BULK_4096_FP32 if args.workload == "bulk" else si.EDGE_2048x8192
    cfg = dict(base, precision=args.precision)
    if args.growth and args.growth != cfg["growth"]:
        cfg.update(growth=args.growth, name=f"{cfg['name']}_{args.growth}")
    if args.lattice != "d2q9":
        cfg.update(lattice=args.lattice, name=f"{cfg['name']}_{args.lattice}")
    if args.stochastic_round:
        cfg.update(stochastic_round=True, name=f"{cfg['name']}_sr")
    if args.tuned:
        from paper_2303_02210_amd import autotune
        cfg = autotune.apply(cfg)
    if args.shape:
        v = [int(x) for x in args.shape.split(",")]
        cfg.update(kernel_vb=v[0], kernel_ty=v[1])
    if args.order is not None:
        cfg.update(kernel_order=args.order)
    L, H = cfg["L"], cfg["H"]
    nq = 7 if args.lattice == "d2q7" else 9
    bpu = 2 * nq * STORE_BYTES[args.precision]         # read Q + write Q populations

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
    launch = {"kernel_vb": cfg.get("kernel_vb", 0), "kernel_ty": cfg.get("kernel_ty", 0),
              "kernel_order": cfg.get("kernel_order", 0)}
    traffic = measured_traffic(cfg["name"], args.precision, launch)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    copies = copy_ceiling(alg_bytes)
    ceiling = copies["ceiling_gbs"]
    log(f"step kernel {achieved:.0f} GB/s; copies of the same bytes: {copies}")
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": round(total_ms / K, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[args.precision], "data": "synthetic",
        "config": {"workload": cfg["name"], "L": L, "H": H, "precision": args.precision,
                   "lattice": args.lattice, "growth": cfg["growth"], "region": cfg["region"],
                   "growth_rate": cfg["growth_rate"], "tau": cfg["tau"], "sigma": cfg["sigma"],
                   "init_rows": cfg["init_rows"], "h_every": every, "sweep": "full",
                   "bytes_per_update": bpu,
                   "rounding": "stochastic" if cfg.get("stochastic_round") else "nearest",
                   "launch": launch},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": "step_kernel", "bytes_per_launch": alg_bytes,
                     "launch_ms": round(per_launch_s * 1e3, 5),
                     "copy": copies,
                     "copy_ceiling_gbs": ceiling,
                     "frac_of_copy": round(achieved / ceiling, 4)},
        "cpu_baseline": None,
    }
    if args.workload == "bulk" and not args.no_ensemble:
        out["ensemble"] = child_record("ensemble", args)
    if args.workload == "bulk" and not args.no_served:
        # (the served runs use the library's default shapes: the tuned solo
        # shapes split the served batch into more groups and measured slower)
        out["served"] = child_record("served", args)
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle, {args.cpu_steps} steps, one thread ...")
        single = cpu_baseline(cfg, args.cpu_steps)
        procs = host_cores()
        log(f"cpu baseline: oracle, {args.cpu_all_steps} steps, {procs} processes ...")
        out["cpu_baseline"] = dict(cpu_baseline_all_cores(cfg, args.cpu_all_steps, procs),
                                   single_thread=single)
    print(json.dumps(out), flush=True)


def child_record(kind: str, args) -> dict:
    """The ensemble or served sub-record of the default line, measured in a
    child process (after this one has released the GPU memory it used), so
    that a failure there costs that record only; its exit status is then
    reported in place of the figures."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--emit-sub", kind,
           "--ensemble-steps", str(args.ensemble_steps),
           "--served-requests", str(args.served_requests),
           "--served-time-limit", str(args.served_time_limit), "--lanes", str(args.lanes)]
    if args.no_sequential:
        cmd.append("--no-sequential")
    limit = 600 + 3 * args.served_time_limit
    log(f"{kind}: measured in a child process ...")
    try:
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=None, text=True, timeout=limit)
    except subprocess.TimeoutExpired:
        return {"error": f"no result within {limit:.0f} s"}
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    if r.returncode != 0 or not lines:
        return {"error": f"child exited with status {r.returncode}"}
    return json.loads(lines[-1])


def run_ensemble(K: int, warmup: int, tuned: bool = True, sequential: bool = True,
                 solo_min_sites="default", persistent: bool = False) -> dict:
    """256 replicas (widths 128..2048 with 96/64/48/32/16 copies, height 4L,
    bulk growth 1e-4, noise 1e-3, float32) advanced together for K steps,
    against the same runs stepped one after another on their own."""
    import torch
    import synth_inputs as si
    from paper_2303_02210_amd import Ensemble, Sim

    cfgs = si.ensemble()
    if tuned:
        from paper_2303_02210_amd import autotune
        cfgs = [autotune.apply(c) for c in cfgs]
    sites = sum(c["L"] * c["H"] for c in cfgs)
    bpu = 2 * 9 * STORE_BYTES["fp32"]
    log(f"ensemble: {len(cfgs)} replicas, {sites} sites, {K} steps each")
    kw = {} if solo_min_sites == "default" else {"solo_min_sites": solo_min_sites}
    ens = Ensemble(cfgs, persistent=persistent, **kw)
    n_alone = len(ens.stepped_alone)
    log(f"{n_alone} members step alone, {len(cfgs) - n_alone} through the batch")
    ens.step(warmup)
    ens.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(ens.stream)
    done = 0
    while done < K:
        n = min(100, K - done)
        ens.step(n)
        done += n
    e1.record(ens.stream)
    ens.synchronize()
    t_batch = e0.elapsed_time(e1) / 1e3
    W = [m.diagnostics()["W"] for m in ens.members]
    ens.close()
    for m in list(ens.members):
        m.close()
    del ens
    torch.cuda.empty_cache()
    log(f"batched: {t_batch:.3f} s; mean W {sum(W) / len(W):.3f}")
    # the same runs, one after another, each on its own
    t_seq = 0.0
    for c in (cfgs if sequential else []):
        sim = Sim(c)
        sim.step(warmup)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(sim.stream)
        sim.step(K)
        b.record(sim.stream)
        torch.cuda.synchronize()
        t_seq += a.elapsed_time(b) / 1e3
        sim.close()
    if sequential:
        log(f"sequential: {t_seq:.3f} s")
    full_steps = si.ensemble()[0]["steps"]
    gbs = sites * bpu / (t_batch / K) / 1e9
    return {
        "workload": "ensemble_256_fp32", "replicas": len(cfgs),
        "widths": list(si.ENSEMBLE_WIDTHS), "counts": list(si.ENSEMBLE_COUNTS),
        "height": "4L", "sites": sites, "steps": K, "bytes_per_update": bpu,
        "members_stepped_alone": n_alone,
        "launches": ("one cooperative launch per table group per 100 steps" if persistent
                     else "one per group per step, 100-step runs replayed from a graph"),
        "mlups": round(sites * K / t_batch / 1e6, 1), "ms_per_step": round(t_batch / K * 1e3, 4),
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)},
        "runs_per_hour": round(len(cfgs) / (t_batch * full_steps / K) * 3600, 1),
        "sequential": None if not t_seq else {
            "mlups": round(sites * K / t_seq / 1e6, 1),
            "runs_per_hour": round(len(cfgs) / (t_seq * full_steps / K) * 3600, 1)},
        "speedup_vs_sequential": round(t_seq / t_batch, 3) if t_seq else None,
        "mean_W": round(sum(W) / len(W), 4),
    }


def bench_ensemble(args):
    """The ensemble on its own JSON line."""
    e = run_ensemble(args.steps, args.warmup, tuned=args.tuned, sequential=not args.no_sequential,
                     solo_min_sites=None if args.all_batched else "default",
                     persistent=args.persistent)
    out = {
        "metric": METRIC, "value": e["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": e["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {k: e[k] for k in ("workload", "replicas", "widths", "counts", "height",
                                     "sites", "bytes_per_update", "members_stepped_alone",
                                     "launches")},
        "roofline": dict(e["roofline"], traffic=None),
        "runs_per_hour": e["runs_per_hour"], "sequential": e["sequential"],
        "speedup_vs_sequential": e["speedup_vs_sequential"], "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_served(n: int, time_limit: float, tuned: bool = False, sequential: bool = True,
               lanes: int = 6) -> dict:
    """Poisson arrivals at 20 requests/s of runs with L in {128..4096}, H in
    [2L, 4L], 1000-50000 steps, bulk or front-band growth, FP64 / FP32 /
    FP16-offset; admitted by HBM footprint into the running batch; rear wall
    following the front; only live rows swept; front heights streamed back
    every tick; one batch per storage-type lane, each on its own stream.
    Throughput counts the rows actually swept (active MLUPS); its roofline
    fraction is their algorithmic bytes over the GPU-busy time."""
    import torch
    import synth_inputs as si
    from paper_2303_02210_amd.serve import Server, serve_sequential

    reqs = si.served_trace(n=n)
    if tuned:
        from paper_2303_02210_amd import autotune
        reqs = [autotune.apply(c) for c in reqs]
    srv = Server(hbm_budget=200e9, tick_steps=100, lanes=lanes)
    summ = srv.serve(reqs, time_limit=time_limit, log=log)
    srv.close()
    log(json.dumps(summ))
    seq = None
    if sequential:
        torch.cuda.empty_cache()
        seq = serve_sequential(reqs, time_limit=time_limit, tick_steps=100, log=log)
        log("sequential: " + json.dumps(seq))

    def figures(sm):
        gbs = sm["active_bytes"] / sm["gpu_busy_s"] / 1e9 if sm["gpu_busy_s"] > 0 else 0.0
        return {"runs_per_hour": round(sm["runs_per_hour"], 1), "completed": sm["completed"],
                "unfinished": sm["running"] + sm["queued"],
                "p50_latency_s": sm["p50_latency_s"], "p99_latency_s": sm["p99_latency_s"],
                "mlups_active": round(sm["mlups_active"], 1),
                "mlups_active_busy": round(sm["mlups_active_busy"], 1),
                "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                             "over": "GPU-busy time, swept rows only"},
                "gpu_busy_frac": round(sm["gpu_busy_frac"], 4), "wall_s": round(sm["wall_s"], 2)}

    out = {"workload": f"served_poisson20_{n}", "requests": n, "rate_hz": 20.0,
           "widths": [128, 256, 512, 1024, 2048, 4096], "steps_range": [1000, 50000],
           "wall": "follow", "sweep": "window", "hbm_budget_bytes": 200e9, "tick_steps": 100,
           "time_limit_s": time_limit, "lanes": lanes,
           "launch_shapes": "autotuner cache" if tuned else "library defaults"}
    out.update(figures(summ))
    out["sequential"] = None if seq is None else figures(seq)
    out["speedup_vs_sequential"] = (None if seq is None or not seq["runs_per_hour"] else
                                    round(summ["runs_per_hour"] / seq["runs_per_hour"], 3))
    return out


def bench_served(args):
    """The served trace on its own JSON line."""
    sv = run_served(args.requests, args.time_limit, tuned=args.tuned,
                    sequential=not args.no_sequential, lanes=args.lanes)
    out = {
        "metric": METRIC, "value": sv["runs_per_hour"], "unit": "runs/hour",
        "n_gpus": 1, "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "mixed f64/f32/f16-offset",
        "data": "synthetic",
        "config": {k: sv[k] for k in ("workload", "requests", "rate_hz", "widths", "steps_range",
                                      "wall", "sweep", "hbm_budget_bytes", "tick_steps",
                                      "time_limit_s", "lanes", "launch_shapes")},
        "cpu_baseline": None,
    }
    out.update({k: v for k, v in sv.items() if k not in out["config"]})
    print(json.dumps(out), flush=True)


def _curves(sims, steps, every, stream_sync, times=None):
    """Advance sims together and record hbar(t), W(t) and mass every `every`
    steps, or at the given increasing times (sims: an Ensemble)."""
    import numpy as np
    rec = {"t": [], "hbar": [], "W": [], "mass": [], "wmass": []}
    marks = list(times) if times is not None else list(range(every, steps + every, every))
    done = 0
    for mark in marks:
        mark = min(int(mark), steps)
        if mark <= done:
            continue
        sims.step(mark - done)
        done = mark
        stream_sync()
        if len(rec["t"]) % 20 == 19:
            log(f"  t = {done}")
        ds = [m.diagnostics() for m in sims.members]
        rec["t"].append(done)
        rec["hbar"].append([d["hbar"] for d in ds])
        rec["W"].append([d["W"] for d in ds])
        rec["mass"].append([d["mass"] - d["src_total"] - d["fix_total"] + d["retired"] for d in ds])
        rec["wmass"].append([d["mass"] for d in ds])
    return {k: np.asarray(v) for k, v in rec.items()}


def bench_appb(args):
    """Appendix B: w(t) and the front profile at L = 640 under the
    density-dependent division law (Eq. 5) and under uniform divisions held
    to the 30 rows above the rear wall, 4 seeds each, batched (float32, wall
    following the front).  Reports w(t) per regime (mean and 95% interval
    over seeds), the final profiles h(x) - hbar, and the batch throughput."""
    import numpy as np
    import torch
    import synth_inputs as si
    from paper_2303_02210_amd import Ensemble

    nseed = 4
    cfgs = si.appendix_b(nseed, lattice=args.lattice or "d2q7")
    if args.sigma is not None:
        cfgs = [dict(c, sigma=args.sigma) for c in cfgs]
    steps = args.steps
    every = max(100, steps // 200)
    log(f"appendix B: {len(cfgs)} runs of {cfgs[0]['L']}x{cfgs[0]['H']}, {steps} steps")
    ens = Ensemble(cfgs)
    t0 = time.perf_counter()
    c = _curves(ens, steps, every, ens.synchronize)
    wall = time.perf_counter() - t0
    prof = [m.front_heights().astype(np.float64) for m in ens.members]
    dg = [m.diagnostics() for m in ens.members]
    ens.close()
    for m in ens.members:
        m.close()
    W = c["W"]
    regimes = {"density_dependent": slice(0, nseed), "rear_band_30": slice(nseed, 2 * nseed)}
    res = {}
    for name, sl in regimes.items():
        w = W[:, sl]
        ci = 1.96 * w.std(1, ddof=1) / np.sqrt(nseed)
        res[name] = {
            "W_mean": np.round(w.mean(1), 4).tolist(), "W_ci95": np.round(ci, 4).tolist(),
            "W_final_mean": float(w[-1].mean()), "W_final_ci95": float(ci[-1]),
            "hbar_final_mean": float(c["hbar"][-1, sl].mean()),
            "divisions_mean": float(np.mean([d["divisions"] for d in dg[sl]])),
            # mass budget: what the divisions and the negative-population fix
            # (App. A step 7) added, and the window's mass at the end against
            # its start (a run whose window mass grows without bound has left
            # the lattice Boltzmann regime)
            "src_total_mean": float(np.mean([d["src_total"] for d in dg[sl]])),
            "fix_total_mean": float(np.mean([d["fix_total"] for d in dg[sl]])),
            "window_mass_growth_max": float(np.max(c["wmass"][-1, sl] / c["wmass"][0, sl])),
            "profile_seed0": np.round(prof[sl.start] - prof[sl.start].mean(), 2).tolist(),
        }
        log(f"{name}: W(final) {res[name]['W_final_mean']:.3f} +- {res[name]['W_final_ci95']:.3f}, "
            f"hbar {res[name]['hbar_final_mean']:.1f}")
    sites = sum(cf["L"] * cf["H"] for cf in cfgs)
    out = {
        "metric": "appendix_b_w_final_ratio",
        "value": round(res["density_dependent"]["W_final_mean"] /
                       max(res["rear_band_30"]["W_final_mean"], 1e-12), 3),
        "unit": "ratio", "n_gpus": 1, "steps": steps, "warmup": 0,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "appendix_b_640", "lattice": cfgs[0]["lattice"],
                   "L": cfgs[0]["L"], "H": cfgs[0]["H"],
                   "seeds": nseed, "every": every,
                   "params": {k: cfgs[0][k] for k in ("tau", "mu", "rho_c", "rho_init", "init_amp",
                                                      "sigma", "growth_rate", "rho_cell", "rho0",
                                                      "wall_min_gap", "wall_w_factor")}},
        "t": c["t"].tolist(), "regimes": res,
        "batch_lattice_mlups": round(sites * steps / wall / 1e6, 1),
        "wall_s": round(wall, 2),
    }
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(out, fh)
        log(f"wrote {args.out}")
    out.pop("t")
    for r in out["regimes"].values():
        r.pop("W_mean"), r.pop("W_ci95"), r.pop("profile_seed0")
    print(json.dumps(out), flush=True)


def _paper_params(c):
    return {k: c[k] for k in ("lattice", "tau", "mu", "rho_c", "rho_init", "init_amp", "sigma",
                              "growth", "growth_rate", "rho_cell", "rho0", "wall_min_gap",
                              "wall_w_factor", "H", "precision")}


def bench_scaling(args):
    """Fig. 2: w(L, t) of uniform divisions at L = 40, 80, 160, 320 (8 seeds
    each, batched), the exponents beta, alpha and z fitted from the seed-mean
    curves, and the spread of the collapse with the fitted and with the KPZ
    exponents (1/2, 3/2)."""
    import numpy as np
    import synth_inputs as si
    from paper_2303_02210_amd import Ensemble
    from paper_2303_02210_amd import scaling as sc

    nseed = 8
    cfgs = si.scaling_runs(nseed=nseed, lattice=args.lattice or "d2q7")
    if args.sigma is not None:
        cfgs = [dict(c, sigma=args.sigma) for c in cfgs]
    steps = args.steps
    every = 0
    # log-spaced samples, so that the early power law is resolved
    times = np.unique(np.round(np.logspace(0, np.log10(steps), 300)).astype(int))
    log(f"scaling: {len(cfgs)} runs, widths {si.SCALING_WIDTHS}, {steps} steps")
    ens = Ensemble(cfgs)
    t0 = time.perf_counter()
    c = _curves(ens, steps, 0, ens.synchronize, times=times)
    wall = time.perf_counter() - t0
    dg = [m.diagnostics() for m in ens.members]
    ens.close()
    for m in ens.members:
        m.close()
    curves, per_L = {}, {}
    for i, L in enumerate(si.SCALING_WIDTHS):
        sl = slice(i * nseed, (i + 1) * nseed)
        w = c["W"][:, sl]
        curves[L] = (c["t"], w.mean(1))
        per_L[L] = {"W_final_mean": float(w[-1].mean()),
                    "fix_over_src": float(np.mean([d["fix_total"] / max(d["src_total"], 1e-30)
                                                   for d in dg[sl]])),
                    "window_mass_growth_max": float(np.max(c["wmass"][-1, sl] / c["wmass"][0, sl]))}
    fit = sc.fit_exponents(curves)
    _, spread_fit = sc.collapse(curves, fit["alpha"], fit["z"])
    _, spread_kpz = sc.collapse(curves, 0.5, 1.5)
    for L in si.SCALING_WIDTHS:
        per_L[L].update({k: fit["sizes"][L][k] for k in ("w_inf", "w_inf_se", "beta", "t_inf")})
    out = {"metric": "scaling_exponents", "value": round(fit["alpha"], 4), "unit": "alpha",
           "n_gpus": 1, "steps": steps, "data": "synthetic",
           "config": {"workload": "scaling_fig2", "widths": list(si.SCALING_WIDTHS),
                      "seeds": nseed, "every": every, "params": _paper_params(cfgs[0])},
           "alpha": fit["alpha"], "beta": fit["beta"], "z": fit["z"],
           "alpha_over_beta": fit["alpha_over_beta"],
           "collapse_spread_fitted": spread_fit, "collapse_spread_kpz": spread_kpz,
           "sizes": {str(L): v for L, v in per_L.items()}, "wall_s": round(wall, 2)}
    log(f"alpha {fit['alpha']:.3f} beta {fit['beta']:.3f} z {fit['z']:.3f}; collapse spread "
        f"fitted {spread_fit:.3f}, KPZ {spread_kpz:.3f}")
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(dict(out, t=c["t"].tolist(),
                           W={str(L): np.asarray(curves[L][1]).tolist() for L in curves}), fh)
    print(json.dumps(out), flush=True)


def bench_extremes(args):
    """Fig. 3c: under Eq. 5, the divisions in the 21 x 20 rectangles below
    h_max and below h_min, their difference sampled every interval (the map
    cleared each time) after a warm-up, at L = 40 (16 seeds) and L = 640
    (4 seeds)."""
    import numpy as np
    import synth_inputs as si
    from paper_2303_02210_amd import Ensemble
    from paper_2303_02210_amd import scaling as sc

    cfgs = si.extremes_runs(lattice=args.lattice or "d2q7")
    if args.sigma is not None:
        cfgs = [dict(c, sigma=args.sigma) for c in cfgs]
    steps = args.steps
    warm = steps // 5
    every = max(100, steps // 200)
    log(f"extremes: {len(cfgs)} runs, {steps} steps (warm-up {warm}, every {every})")
    ens = Ensemble(cfgs)
    ens.step(warm)
    ens.synchronize()
    for m in ens.members:
        m.division_map(clear=True)
    diffs = {40: [], 640: []}
    done = warm
    t0 = time.perf_counter()
    while done < steps:
        ens.step(every)
        done += every
        ens.synchronize()
        for c, m in zip(cfgs, ens.members):
            dmap = m.division_map(clear=True)
            h = m.front_heights()
            diffs[c["L"]].append(sc.division_difference(dmap, h, m.diagnostics()["y_wall"]))
    wall = time.perf_counter() - t0
    W = {L: float(np.mean([m.diagnostics()["W"] for c, m in zip(cfgs, ens.members)
                           if c["L"] == L])) for L in diffs}
    ens.close()
    for m in ens.members:
        m.close()
    res = {}
    for L, d in diffs.items():
        d = np.asarray(d, float)
        hist, edges = np.histogram(d, bins=21)
        res[str(L)] = {"samples": int(d.size), "mean": float(d.mean()), "std": float(d.std()),
                       "se": float(d.std() / np.sqrt(d.size)),
                       "frac_positive": float((d > 0).mean()), "W_final_mean": W[L],
                       "hist": hist.tolist(), "edges": np.round(edges, 2).tolist()}
        log(f"L={L}: mean difference {d.mean():.2f} +- {d.std() / np.sqrt(d.size):.2f} "
            f"(positive {100 * (d > 0).mean():.0f}%), W {W[L]:.2f}")
    out = {"metric": "extremes_division_difference", "value": res["640"]["mean"],
           "unit": "divisions", "n_gpus": 1, "steps": steps, "data": "synthetic",
           "config": {"workload": "extremes_fig3c", "widths": [40, 640], "warmup": warm,
                      "every": every, "params": _paper_params(cfgs[0])},
           "sizes": res, "wall_s": round(wall, 2)}
    print(json.dumps(out), flush=True)


def bench_dispersion(args):
    """Eq. 7: flat fronts perturbed by one cosine mode (amplitude 8 rows, modes
    n = 1..8 of L = 640, 6 seeds each) under Eq. 5; the growth rate omega(q)
    of each mode's amplitude over the run and the fit omega = k - gamma q^2."""
    import numpy as np
    import synth_inputs as si
    from paper_2303_02210_amd import Ensemble
    from paper_2303_02210_amd import scaling as sc

    cfgs = si.dispersion_runs(lattice=args.lattice or "d2q7")
    if args.sigma is not None:
        cfgs = [dict(c, sigma=args.sigma) for c in cfgs]
    steps = args.steps
    every = max(20, steps // 100)
    h0 = 150.0
    log(f"dispersion: {len(cfgs)} runs, modes {si.DISPERSION_MODES}, {steps} steps")
    ens = Ensemble(cfgs)
    for c, m in zip(cfgs, ens.members):
        L, H = c["L"], c["H"]
        x = np.arange(L)
        h = np.floor(h0 + c["amplitude"] * np.cos(2 * np.pi * c["mode"] * x / L) + 0.5).astype(np.int32)
        Q = m.Q
        w = np.array([0.5] + [1 / 12] * 6) if Q == 7 else \
            np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
        f = np.zeros((Q, H, L))
        rows = np.arange(H)[:, None]
        f[:, :, :] = w[:, None, None] * (rows < h[None, :]) * c["rho_init"]
        m.set_populations(f)
        m.set_front_heights(h)
    amps = {c["name"]: [] for c in cfgs}
    ts = []
    done = 0
    t0 = time.perf_counter()
    while done < steps:
        ens.step(every)
        done += every
        ens.synchronize()
        ts.append(done)
        for c, m in zip(cfgs, ens.members):
            amps[c["name"]].append(sc.mode_amplitude(m.front_heights(), c["mode"]))
    wall = time.perf_counter() - t0
    ens.close()
    for m in ens.members:
        m.close()
    L = cfgs[0]["L"]
    q, om, om_se = [], [], []
    per = {}
    for n in si.DISPERSION_MODES:
        rates = [sc.growth_rate(ts, amps[c["name"]]) for c in cfgs if c["mode"] == n]
        q.append(2 * np.pi * n / L)
        om.append(float(np.mean(rates)))
        om_se.append(float(np.std(rates, ddof=1) / np.sqrt(len(rates))))
        per[str(n)] = {"q": q[-1], "omega": om[-1], "omega_se": om_se[-1]}
    fit = sc.fit_dispersion(q, om)
    log(f"omega(q): {np.round(om, 6).tolist()}; k {fit['k']:.3g} gamma {fit['gamma']:.3g}")
    out = {"metric": "dispersion_fit", "value": fit["k"], "unit": "per step", "n_gpus": 1,
           "steps": steps, "data": "synthetic",
           "config": {"workload": "dispersion_eq7", "L": L, "modes": list(si.DISPERSION_MODES),
                      "amplitude": cfgs[0]["amplitude"], "h0": h0, "every": every,
                      "params": _paper_params(cfgs[0])},
           "modes": per, "k": fit["k"], "gamma": fit["gamma"], "q_c": fit["q_c"],
           "L_c": fit["L_c"], "wall_s": round(wall, 2)}
    print(json.dumps(out), flush=True)


def bench_precision(args):
    """W(L,t), mean front height and mass balance of the float32 and 16-bit
    offset storages (rounded to nearest, and stochastically: "_sr") against
    float64 (bit-identical to the oracle).  (a) The 2048 x 8192 edge-growth
    strip at full size, one run per storage, from 128 tissue rows so that
    the front moves within the run; (b) the same model at 256 x 1024 as 8
    seeds per storage, batched, for means and 95% intervals."""
    import numpy as np
    import synth_inputs as si
    from paper_2303_02210_amd import Ensemble

    precs = ["fp64", "fp32", "fp16", "bf16", "fp16_sr", "bf16_sr"]

    def storage(p):
        return dict(precision=p[:4], stochastic_round=p.endswith("_sr"))

    steps = args.steps
    every = max(100, steps // 100)
    res = {"full": {}, "seeds": {}}
    # (a) full size, all four storages in one batch
    cfgs = [dict(si.EDGE_ACCURACY, **storage(p)) for p in precs]
    ens = Ensemble(cfgs)
    log(f"precision (a): 2048x8192 from 128 rows x {steps} steps, {precs}")
    c = _curves(ens, steps, every, ens.synchronize)
    ens.close()
    for m in ens.members:
        m.close()
    ref_h, ref_W = c["hbar"][:, 0], c["W"][:, 0]
    m0 = c["mass"][0]
    t_full = np.asarray(c["t"])
    init_full = float(si.EDGE_ACCURACY["init_rows"])
    for i, p in enumerate(precs):
        moved = c["hbar"][:, i] > init_full + 0.5
        res["full"][p] = {
            "front_starts_t": float(t_full[np.argmax(moved)]) if moved.any() else None,
            "hbar_final": float(c["hbar"][-1, i]), "W_final": float(c["W"][-1, i]),
            "max_W": float(np.max(c["W"][:, i])),
            "max_abs_dhbar": float(np.max(np.abs(c["hbar"][:, i] - ref_h))),
            "max_rel_dW": float(np.max(np.abs(c["W"][:, i] - ref_W) / np.maximum(ref_W, 1e-9))),
            "mass_balance_drift_rel": float(np.max(np.abs(c["mass"][:, i] - m0[i])) / m0[i]),
        }
    res["full_curves"] = {"t": c["t"].tolist(), "hbar": c["hbar"].tolist(), "W": c["W"].tolist()}
    # (b) 8 seeds per storage at 256 x 1024
    nseed = 8
    small = []
    for p in precs:
        for sd in range(nseed):
            small.append(dict(si.EDGE_2048x8192, name=f"edge256_{p}_s{sd}", L=256, H=1024,
                              init_rows=128, seed=100 + sd, replica=sd, **storage(p)))
    ens = Ensemble(small)
    log(f"precision (b): 256x1024 x {steps} steps, {nseed} seeds x {precs}")
    c = _curves(ens, steps, every, ens.synchronize)
    ens.close()
    for m in ens.members:
        m.close()
    W = c["W"].reshape(len(c["t"]), len(precs), nseed)
    Hb = c["hbar"].reshape(len(c["t"]), len(precs), nseed)
    # time at which each run's front first leaves its initial row
    t_arr = np.asarray(c["t"])
    init_h = float(small[0]["init_rows"])
    adv = np.where((Hb > init_h + 0.5).any(0), t_arr[np.argmax(Hb > init_h + 0.5, axis=0)], -1)
    for i, p in enumerate(precs):
        dW = W[:, i].mean(1) - W[:, 0].mean(1)
        seW = np.sqrt(W[:, i].var(1, ddof=1) / nseed + W[:, 0].var(1, ddof=1) / nseed)
        dH = Hb[:, i].mean(1) - Hb[:, 0].mean(1)
        seH = np.sqrt(Hb[:, i].var(1, ddof=1) / nseed + Hb[:, 0].var(1, ddof=1) / nseed)
        ta = adv[i][adv[i] >= 0]
        res["seeds"][p] = {
            "front_starts_t_mean": float(ta.mean()) if ta.size else None,
            "front_starts_t_ci95": float(1.96 * ta.std(ddof=1) / np.sqrt(ta.size)) if ta.size > 1 else None,
            "runs_advanced": int(ta.size),
            "W_mean_final": float(W[-1, i].mean()), "W_ci95_final": float(1.96 * W[-1, i].std(ddof=1) / np.sqrt(nseed)),
            "hbar_ci95_final": float(1.96 * Hb[-1, i].std(ddof=1) / np.sqrt(nseed)),
            "hbar_mean_final": float(Hb[-1, i].mean()),
            "max_dW_over_se": float(np.max(np.abs(dW) / np.maximum(seW, 1e-12))) if i else 0.0,
            "max_dhbar_over_se": float(np.max(np.abs(dH) / np.maximum(seH, 1e-12))) if i else 0.0,
            "max_abs_dW_mean": float(np.max(np.abs(dW))), "max_abs_dhbar_mean": float(np.max(np.abs(dH))),
        }
    res["seed_curves"] = {"t": c["t"].tolist(), "W_mean": W.mean(2).tolist(), "hbar_mean": Hb.mean(2).tolist()}
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(res, fh)
    summ = {k: v for k, v in res.items() if k in ("full", "seeds")}
    out = {"metric": METRIC, "value": None, "unit": None, "n_gpus": 1, "steps": steps,
           "warmup": 0, "higher_is_better": True, "vs_baseline": None, "data": "synthetic",
           "dtype": "f64/f32/f16-offset/bf16-offset (nearest and stochastic rounding)",
           "config": {"workload": "precision_edge", "full": "2048x8192 from 128 tissue rows",
                      "seeds": "8 x 256x1024", "every": every},
           "accuracy": summ}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
