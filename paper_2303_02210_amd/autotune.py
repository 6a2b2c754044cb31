"""Launch-shape autotuner.

The step kernel's launch shape -- its form and bytes of columns per lane
(``kernel_vb``: 1 = one column per lane, 2 = rows staged through LDS, or
4 / 8 / 16 bytes) and rows per thread (``kernel_ty``) -- changes speed, never
results (every site's update is the
same arithmetic in any shape).  ``tune`` times the candidates on the GPU for
one workload and ``apply`` fills a workload dict from the cache of tuned
shapes, keyed by storage type and the width and height rounded up to powers
of two.
"""
from __future__ import annotations

import json
import os

from .sim import Sim, _torch

_PKG = os.path.dirname(os.path.abspath(__file__))
SHIPPED = os.path.join(_PKG, "tuned.json")
USER = os.environ.get("LBMGROW_TUNE_CACHE", os.path.expanduser("~/.cache/lbmgrow/tuned.json"))

_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}


def _pow2(n: int) -> int:
    p = 1
    while p < n:
        p *= 2
    return p


def key(cfg: dict) -> str:
    """Storage, width and height rounded up to powers of two, and whether a
    division law runs or the 16-bit storage rounds stochastically (those
    kernels hold more registers), and whether growth is confined to a band
    at the front (the tissue rows then sit in one part of the lattice, and
    the best shape of the same lattice differs)."""
    div = "/div" if str(cfg.get("growth", "bulk")).startswith("division") else ""
    lat = "/d2q7" if cfg.get("lattice", "d2q9") == "d2q7" else ""
    band = "/band" if cfg.get("region", "all") == "front_band" else ""
    sr = "/sr" if cfg.get("stochastic_round", False) else ""
    return (f"{cfg.get('precision', 'fp64')}/L{_pow2(int(cfg['L']))}/H{_pow2(int(cfg['H']))}"
            f"{div}{lat}{band}{sr}")


def candidates(cfg: dict):
    esize = _BYTES[cfg.get("precision", "fp64")]
    if cfg.get("lattice", "d2q9") == "d2q7":      # no LDS-staged form
        for vb in [1] + [vb for vb in (4, 8, 16) if vb >= esize and int(cfg["L"]) % (vb // esize) == 0]:
            for ty in (1, 2, 4, 8):
                yield {"kernel_vb": vb, "kernel_ty": ty}
        return
    vbs = [1] + [vb for vb in (4, 8, 16) if vb >= esize and int(cfg["L"]) % (vb // esize) == 0]
    for vb in vbs:
        for ty in (1, 2, 4, 8):
            yield {"kernel_vb": vb, "kernel_ty": ty}
    if (esize != 2 or int(cfg["L"]) % 2 == 0) and not cfg.get("stochastic_round", False):
        for ty in (16, 32, 64):
            yield {"kernel_vb": 2, "kernel_ty": ty}


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def cache() -> dict:
    c = _load(SHIPPED)
    c.update(_load(USER))
    return c


def apply(cfg: dict) -> dict:
    """cfg with the tuned launch shape for its key, if one is known and the
    dict does not set one itself (a stochastically rounded run without a key
    of its own takes the shape of the same run rounded to nearest, unless
    that is the LDS-staged form, which has no stochastic rounding)."""
    if "kernel_vb" in cfg or "kernel_ty" in cfg:
        return cfg
    shape = cache().get(key(cfg))
    if shape is None and cfg.get("stochastic_round", False):
        shape = cache().get(key(dict(cfg, stochastic_round=False)))
        if shape and shape.get("kernel_vb") == 2:
            shape = None
    return dict(cfg, **shape) if shape else cfg


def time_shape(cfg: dict, shape: dict, steps: int = 100, warmup: int = 10,
               repeats: int = 2) -> float:
    """Milliseconds per step of cfg launched with shape: the fastest of
    `repeats` timings of `steps` steps each, after a warm-up."""
    torch = _torch()
    sim = Sim(dict(cfg, **shape))
    sim.step(warmup)
    best = float("inf")
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        sim.step(steps)
        e1.record(sim.stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / steps)
    sim.close()
    return best


def tune(cfg: dict, steps: int = 100, save: str | None = USER, verbose: bool = False) -> dict:
    """Time every candidate shape for cfg and remember the fastest."""
    best, best_ms = None, float("inf")
    for shape in candidates(cfg):
        ms = time_shape(cfg, shape, steps)
        if verbose:
            print(f"  {key(cfg)} {shape} {ms:.4f} ms/step", flush=True)
        if ms < best_ms:
            best, best_ms = shape, ms
    if save:
        os.makedirs(os.path.dirname(save) or ".", exist_ok=True)
        c = _load(save)
        c[key(cfg)] = best
        with open(save, "w") as fh:
            json.dump(c, fh, indent=1, sort_keys=True)
    return dict(best, ms_per_step=best_ms)


def main(argv=None):
    """Tune the shapes of the standard workloads and write them to a cache
    file: python -m paper_2303_02210_amd.autotune [--out PATH]."""
    import argparse
    import sys

    root = os.path.dirname(_PKG)
    if root not in sys.path:
        sys.path.insert(0, root)
    import synth_inputs as si

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--out", default=USER)
    ap.add_argument("--steps", type=int, default=100)
    args = ap.parse_args(argv)
    work = [dict(si.BULK_4096_FP32, precision=p) for p in ("fp64", "fp32", "fp16", "bf16")]
    work += [dict(si.EDGE_2048x8192, precision=p) for p in ("fp32", "fp16", "bf16")]
    work += [dict(si.BULK_4096_FP32, precision=p, growth="division")
             for p in ("fp64", "fp32", "fp16", "bf16")]
    work += [dict(si.BULK_4096_FP32, precision=p, lattice="d2q7")
             for p in ("fp64", "fp32", "fp16", "bf16")]
    work += [dict(base, precision=p, stochastic_round=True)
             for base in (si.BULK_4096_FP32, si.EDGE_2048x8192) for p in ("fp16", "bf16")]
    seen = set()
    for c in si.ensemble():
        if c["L"] not in seen:
            seen.add(c["L"])
            work.append(c)
    for c in work:
        best = tune(c, steps=args.steps, save=args.out, verbose=False)
        print(f"{key(c)}: {best}", flush=True)


if __name__ == "__main__":
    main()
