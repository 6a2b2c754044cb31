"""Continuous batching of simulation requests on one GPU.

Requests (workload dicts with a step count and an arrival time) are admitted
in arrival order whenever their device workspace fits the HBM budget, join the
running ensemble at the next tick, and leave it as soon as their own step
count is reached; runs that arrive while others are on the GPU therefore share
every launch with them.  Each tick advances the resident runs of a lane by
the same number of steps (at most ``tick_steps``, never past the end of any
of that lane's runs) through the batch API and copies every run's front
heights h(x) back to pinned host memory.  Results are those of the run stepped alone: the batch changes only
how tiles are grouped into launches.

The resident runs are split into ``lanes`` batches by storage type and lattice
width, each on a stream of its own: a served run's step is a chain of short
launches whose latency sets the pace, and the lanes' chains run side by side
on the GPU.
"""
from __future__ import annotations

import collections
import ctypes
import time

import numpy as np

from . import _ffi
from .ensemble import Ensemble, tiles
from .sim import _torch


def workspace_bytes(cfg: dict) -> int:
    p = _ffi.make_params(cfg)
    return int(_ffi.lib().lbm_workspace_bytes(ctypes.byref(p)))


def bytes_per_update(cfg: dict) -> int:
    """Algorithmic HBM bytes of one site update: every population read and
    written once."""
    q = _ffi.Q[cfg.get("lattice", "d2q9")]
    return 2 * q * _ffi.STORAGE_BYTES[cfg.get("precision", "fp64")]


def active_work(cfg: dict, diag: dict) -> tuple:
    """(site updates, algorithmic bytes) a run has swept so far: its width
    times the window rows its steps updated."""
    n = float(cfg["L"]) * float(diag["rows_swept"])
    return n, n * bytes_per_update(cfg)


_TYPE_CLASS = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 2}


def lane_index(req: dict, lanes: int) -> int:
    """The lane of a request: one class per storage type (16-bit types
    together), split further by lattice width (below 1024 columns or not)
    when there are at least six lanes; classes beyond the lanes wrap."""
    c = _TYPE_CLASS.get(req.get("precision", "fp64"), 0)
    if lanes >= 6 and int(req["L"]) >= 1024:
        c += 3
    return c % lanes


class Run:
    """One admitted request."""

    def __init__(self, req: dict, sim, arrival: float, admitted: float, pinned, lane=None):
        self.req = req
        self.sim = sim
        self.lane = lane
        self.arrival = arrival
        self.admitted = admitted
        self.remaining = int(req["steps"])
        self.h = pinned              # latest streamed front heights (pinned host)
        self.h_updates = 0
        self.finished = None
        self.diag = None


class Server:
    def __init__(self, hbm_budget: float = 200e9, tick_steps: int = 100, device: str = "cuda:0",
                 max_members: int = 1024, max_tiles: int = 1 << 23, keep_results: bool = False,
                 clock=time.perf_counter, lanes: int = 6):
        torch = _torch()
        self.torch = torch
        # one batch per lane, each on its own (default-priority) stream
        self.lanes = [Ensemble(device=device, max_members=max_members, max_tiles=max_tiles)
                      for _ in range(max(1, int(lanes)))]
        self.budget = float(hbm_budget)
        self.used = 0.0
        self.tick_steps = int(tick_steps)
        self.max_members = int(max_members)
        self.queue: collections.deque = collections.deque()
        self.running: list[Run] = []
        self.done: list[Run] = []
        self.keep_results = keep_results
        self.clock = clock
        self.t0 = None
        self.active_updates = 0.0     # site updates of swept rows, finished runs
        self.active_bytes = 0.0
        self.gpu_busy = 0.0
        self.ticks = 0

    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, req: dict) -> None:
        self.queue.append(req)

    # -- admission ---------------------------------------------------------
    def _admit(self, now: float) -> int:
        n = 0
        while self.queue and self.queue[0].get("arrival_s", 0.0) <= now:
            req = self.queue[0]
            need = workspace_bytes(req)
            if need == 0:
                raise ValueError(f"invalid request {req.get('name')}")
            if self.used + need > self.budget or len(self.running) >= self.max_members:
                break
            self.queue.popleft()
            lane = self.lanes[lane_index(req, len(self.lanes))]
            sim = lane.add(req)
            pinned = self.torch.empty(int(req["L"]), dtype=self.torch.int32).pin_memory()
            self.running.append(Run(req, sim, req.get("arrival_s", 0.0), now, pinned, lane))
            self.used += need
            n += 1
        return n

    # -- one tick ---------------------------------------------------------------
    def tick(self) -> None:
        # each lane advances by its own count: a run about to finish in one
        # lane does not shorten the others' ticks (nor re-capture their graphs)
        ks = {id(e): min([self.tick_steps] + [r.remaining for r in self.running if r.lane is e])
              for e in self.lanes if e.members}
        torch = self.torch
        # GPU-busy time of the tick: from an event every lane waits for to
        # one recorded after every lane's work
        first = self.lanes[0].stream
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(first)
        active = [e for e in self.lanes if e.members]
        for e in active:
            if e is not self.lanes[0]:
                e.stream.wait_event(ev0)
            e.step(ks[id(e)])
        for r in self.running:
            r.sim.front_heights_async(r.h)
        for e in active:
            if e is not self.lanes[0]:
                done = torch.cuda.Event()
                done.record(e.stream)
                first.wait_event(done)
        ev1.record(first)
        for e in self.lanes:
            e.synchronize()
        self.gpu_busy += ev0.elapsed_time(ev1) / 1e3
        self.ticks += 1
        now = self.now()
        still = []
        for r in self.running:
            r.remaining -= ks[id(r.lane)]
            r.h_updates += 1
            if r.remaining == 0:
                r.finished = now
                r.diag = r.sim.diagnostics()
                n, b = active_work(r.req, r.diag)
                self.active_updates += n
                self.active_bytes += b
                if self.keep_results:
                    r.result = (r.sim.populations(), r.sim.front_heights(), r.diag)
                r.lane.remove(r.sim)
                r.sim.close()
                r.sim = None
                self.used -= workspace_bytes(r.req)
                self.done.append(r)
            else:
                still.append(r)
        self.running = still

    # -- the loop -----------------------------------------------------------------
    def serve(self, requests, time_limit: float | None = None, log=None) -> dict:
        """Replay a request trace in real time; returns the summary."""
        for q in sorted(requests, key=lambda q: q.get("arrival_s", 0.0)):
            self.submit(q)
        self.t0 = self.clock()
        while self.queue or self.running:
            now = self.now()
            if time_limit is not None and now > time_limit:
                break
            self._admit(now)
            if not self.running:
                if self.queue:
                    time.sleep(max(0.0, min(self.queue[0].get("arrival_s", 0.0) - now, 0.05)))
                continue
            self.tick()
            if log and self.ticks % 50 == 0:
                log(f"t={self.now():.1f}s ticks={self.ticks} running={len(self.running)} "
                    f"queued={len(self.queue)} done={len(self.done)}")
        return self.summary()

    def summary(self) -> dict:
        wall = self.now()
        lat = np.array([r.finished - r.arrival for r in self.done]) if self.done else np.zeros(0)
        # work of the runs still resident counts too
        upd, byt = self.active_updates, self.active_bytes
        for r in self.running:
            if r.sim is not None:
                n, b = active_work(r.req, r.sim.diagnostics())
                upd += n
                byt += b
        return {
            "completed": len(self.done), "running": len(self.running), "queued": len(self.queue),
            "wall_s": wall,
            "runs_per_hour": len(self.done) / wall * 3600 if wall > 0 else 0.0,
            "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_latency_s": float(lat.mean()) if lat.size else None,
            "site_updates_active": upd,
            "active_bytes": byt,
            "mlups_active": upd / wall / 1e6 if wall > 0 else 0.0,
            "mlups_active_busy": upd / self.gpu_busy / 1e6 if self.gpu_busy > 0 else 0.0,
            "gpu_busy_s": self.gpu_busy,
            "gpu_busy_frac": self.gpu_busy / wall if wall > 0 else 0.0,
            "ticks": self.ticks,
        }

    def close(self) -> None:
        for r in self.running:
            if r.sim is not None:
                r.lane.remove(r.sim)
                r.sim.close()
        self.running = []
        for e in self.lanes:
            e.close()


def serve_sequential(requests, time_limit: float | None = None, tick_steps: int = 100,
                     device: str = "cuda:0", clock=time.perf_counter, log=None) -> dict:
    """The same trace served one run at a time, in arrival order, each run
    stepped alone (no batching): the plain queue that continuous batching is
    measured against.  Front heights are streamed back every tick_steps
    steps, as in Server.  Returns a summary with the same fields."""
    from .sim import Sim
    torch = _torch()
    reqs = sorted(requests, key=lambda q: q.get("arrival_s", 0.0))
    t0 = clock()
    lat, upd, byt, busy = [], 0.0, 0.0, 0.0
    done = 0
    for i, req in enumerate(reqs):
        now = clock() - t0
        if time_limit is not None and now > time_limit:
            break
        wait = req.get("arrival_s", 0.0) - now
        if wait > 0:
            time.sleep(wait)
        sim = Sim(req, device=device)
        pinned = torch.empty(int(req["L"]), dtype=torch.int32).pin_memory()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(sim.stream)
        left = int(req["steps"])
        cut = False
        while left > 0:
            k = min(tick_steps, left)
            sim.step(k)
            sim.front_heights_async(pinned)
            left -= k
            if time_limit is not None and clock() - t0 > time_limit:
                cut = True
                break
        ev1.record(sim.stream)
        sim.stream.synchronize()
        d = sim.diagnostics()                  # raises if the run latched an error
        busy += ev0.elapsed_time(ev1) / 1e3
        n, b = active_work(req, d)
        upd += n
        byt += b
        sim.close()
        if cut:
            break
        lat.append(clock() - t0 - req.get("arrival_s", 0.0))
        done += 1
        if log and done % 50 == 0:
            log(f"sequential: t={clock() - t0:.1f}s done={done}")
    wall = clock() - t0
    lat = np.array(lat) if lat else np.zeros(0)
    return {
        "completed": done, "running": 0, "queued": len(reqs) - done, "wall_s": wall,
        "runs_per_hour": done / wall * 3600 if wall > 0 else 0.0,
        "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
        "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
        "mean_latency_s": float(lat.mean()) if lat.size else None,
        "site_updates_active": upd,
        "active_bytes": byt,
        "mlups_active": upd / wall / 1e6 if wall > 0 else 0.0,
        "mlups_active_busy": upd / busy / 1e6 if busy > 0 else 0.0,
        "gpu_busy_s": busy,
        "gpu_busy_frac": busy / wall if wall > 0 else 0.0,
        "ticks": None,
    }

