"""Seeded synthetic workloads for the growing-tissue D2Q9 LBM.

This module holds inputs only -- parameter sets, seeds and arrival traces --
and none of the method's arithmetic.  Both the GPU library's callers and the
oracle's callers take their inputs from here, so the two sides are always fed
the same workload.

Model parameters follow the paper's parameter list (Appendix A): tau = 1,
mu = 1e-3, and the ratio rho_c / rho_init = 0.05 / 0.1 = 1/2, with the
tissue at rho_init = 1.  The random numbers the method itself draws (initial
densities, noise) are not generated here: each side draws them from its own
Philox4x32-10 implementation keyed by (seed, replica), counter (x, y, t,
stream).
"""
from __future__ import annotations

import numpy as np

# Defaults shared by every workload (paper: Appendix A parameter list,
# rescaled to rho_init = 1).
BASE = dict(
    tau=1.0,
    mu=1e-3,
    rho_c=0.5,
    rho_init=1.0,
    init_amp=1e-3,
    growth="bulk",
    growth_rate=1e-3,
    region="all",
    region_width=0,
    sigma=0.0,
    ybc="fixed",
    wall_min_gap=50,
    wall_w_factor=10.0,
    seed=0,
    replica=0,
    precision="fp64",
    # division laws (Sec. II, Eq. 5): mass of one cell and the density above
    # which division stops, from the paper's 0.01 and 0.15 at rho_init = 0.1
    rho_cell=0.1,
    rho0=1.5,
)


def cfg(**kw) -> dict:
    c = dict(BASE)
    c.update(kw)
    return c


# 64 x 64, FP64, tissue rows 0-15 at rho = 1 (+-1e-3), bulk growth 1e-3 per
# step, no noise, fixed rear wall, 1000 steps, seed 0: the parity workload.
SMALL_FP64 = cfg(name="small_64x64_fp64", L=64, H=64, init_rows=16,
                 growth_rate=1e-3, sigma=0.0, precision="fp64", steps=1000)

# 4096 x 4096, FP32, bulk growth 1e-4, noise 1e-3, tissue rows 0-255,
# 20000 steps, front heights every 100 steps: the throughput workload.
BULK_4096_FP32 = cfg(name="bulk_4096x4096_fp32", L=4096, H=4096, init_rows=256,
                     growth_rate=1e-4, sigma=1e-3, precision="fp32", steps=20000,
                     h_every=100)

# 2048 wide x 8192 high, tau = 0.8, growth only within ell = 8 of the front,
# rate 1e-3, noise 1e-3, tissue rows 0-1023, 50000 steps; run in FP32 and in
# FP16 / BF16 offset storage.
EDGE_2048x8192 = cfg(name="edge_2048x8192", L=2048, H=8192, tau=0.8, init_rows=1024,
                     growth_rate=1e-3, region="front_band", region_width=8,
                     sigma=1e-3, precision="fp32", steps=50000)

# The same strip for the accuracy comparison of the storages.  The workload
# does not state the initial tissue rows; with 1024 the front cannot advance
# within 50000 steps (a void row above a flat front receives 1/6 of the
# interface density, so the density near the front must reach 3 rho_init,
# and growth in an 8-row band of 1024 rows raises the mean only by a factor
# exp(50000 * 8/1024 * 1e-3) ~ 1.5).  With 128 rows the front starts near
# t ~ 17600 (exp(t * 8/128 * 1e-3) ~ 3).  Only the rows that can hold mass
# are swept (the results do not depend on it).
EDGE_ACCURACY = dict(EDGE_2048x8192, name="edge_2048x8192_128rows", init_rows=128, window=True)

# Ensemble for roughness scaling: widths and replica counts, height 4L,
# bulk growth 1e-4, noise 1e-3, 10000 steps, FP32, seeds = replica ids.
ENSEMBLE_WIDTHS = (128, 256, 512, 1024, 2048)
ENSEMBLE_COUNTS = (96, 64, 48, 32, 16)


def ensemble(widths=ENSEMBLE_WIDTHS, counts=ENSEMBLE_COUNTS, steps=10000) -> list[dict]:
    out = []
    rep = 0
    for L, n in zip(widths, counts):
        for _ in range(n):
            out.append(cfg(name=f"ens_L{L}_r{rep}", L=L, H=4 * L, init_rows=L,
                           growth_rate=1e-4, sigma=1e-3, precision="fp32",
                           steps=steps, seed=rep, replica=rep))
            rep += 1
    return out


def served_trace(n: int = 600, rate_hz: float = 20.0, seed: int = 0,
                 widths=(128, 256, 512, 1024, 2048, 4096),
                 steps_range=(1000, 50000)) -> list[dict]:
    """Poisson arrivals of simulation requests of mixed size and precision.

    L uniform over powers of two in [128, 4096]; H uniform in [2L, 4L]
    rounded to 64; steps uniform in steps_range; growth bulk (1e-4) or front
    band (ell = 8, 1e-3) with equal odds; precision FP64 / FP32 / FP16-offset
    with equal odds; tissue initially in the first 128 rows; rear wall that
    follows the front (gap max(50, 10 w)); only rows that can hold mass are
    swept.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n):
        t += rng.exponential(1.0 / rate_hz)
        L = int(rng.choice(widths))
        H = int(round(rng.uniform(2 * L, 4 * L) / 64.0)) * 64
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        edge = bool(rng.integers(0, 2))
        prec = ["fp64", "fp32", "fp16"][int(rng.integers(0, 3))]
        c = cfg(name=f"req{k}", L=L, H=H, init_rows=128, sigma=1e-3,
                ybc="follow", window=True, precision=prec, steps=steps, seed=k, replica=0,
                arrival_s=t)
        if edge:
            c.update(growth_rate=1e-3, region="front_band", region_width=8)
        else:
            c.update(growth_rate=1e-4)
        out.append(c)
    return out


# The paper's runs (Sec. III, IV, Appendix A): its own D2Q7 lattice and the
# Appendix A parameters rescaled to rho_init = 1 (sigma 0.01 -> 0.1,
# rho_cell 0.01 -> 0.1, rho0 0.15 -> 1.5; initial density uniform on
# [0.9, 1.1] rho_init), the rear wall kept max(50, 10 w) behind the mean
# front, the sweep window on, float32.  The paper does not give heights or
# initial tissue rows; these leave room for the wall gap and a front several
# w rough.
PAPER_BASE = dict(BASE, lattice="d2q7", H=2048, init_rows=100, init_amp=0.1, sigma=0.1,
                  growth="division", growth_rate=1e-3, ybc="follow", wall_min_gap=50,
                  wall_w_factor=10.0, window=True, precision="fp32")
APPB_BASE = dict(PAPER_BASE, L=640)


def appendix_b(nseed: int = 4, lattice: str = "d2q7") -> list[dict]:
    """Appendix B at L = 640: nseed runs of the density-dependent division law
    (Eq. 5) everywhere, then nseed runs of uniform divisions held to the 30
    rows above the rear wall."""
    runs = []
    for sd in range(nseed):
        runs.append(dict(APPB_BASE, name=f"appb_density_s{sd}", growth="division_density",
                         lattice=lattice, seed=500 + sd, replica=sd))
    for sd in range(nseed):
        runs.append(dict(APPB_BASE, name=f"appb_rearband_s{sd}", growth="division",
                         region="rear_band", region_width=30, lattice=lattice, seed=600 + sd,
                         replica=sd))
    return runs


# Fig. 2: uniform divisions at several widths, for w(L, t) and its exponents.
SCALING_WIDTHS = (40, 80, 160, 320)


def scaling_runs(widths=SCALING_WIDTHS, nseed: int = 8, lattice: str = "d2q7",
                 growth: str = "division") -> list[dict]:
    return [dict(PAPER_BASE, name=f"scaling_L{L}_s{sd}", L=L, growth=growth, lattice=lattice,
                 seed=700 + 17 * i + sd, replica=sd)
            for i, L in enumerate(widths) for sd in range(nseed)]


# Fig. 3c: divisions near h_max and h_min under Eq. 5 at L = 40 and L = 640.
def extremes_runs(lattice: str = "d2q7") -> list[dict]:
    runs = [dict(PAPER_BASE, name=f"extremes_L40_s{sd}", L=40, growth="division_density",
                 division_map=True, lattice=lattice, seed=800 + sd, replica=sd) for sd in range(16)]
    runs += [dict(PAPER_BASE, name=f"extremes_L640_s{sd}", L=640, growth="division_density",
                  division_map=True, lattice=lattice, seed=900 + sd, replica=sd) for sd in range(4)]
    return runs


# Eq. 7: flat fronts with one cosine mode of amplitude 8 rows under Eq. 5.
DISPERSION_MODES = (1, 2, 3, 4, 6, 8)


def dispersion_runs(L: int = 640, modes=DISPERSION_MODES, nseed: int = 6,
                    lattice: str = "d2q7") -> list[dict]:
    return [dict(PAPER_BASE, name=f"dispersion_n{n}_s{sd}", L=L, growth="division_density",
                 lattice=lattice, mode=n, amplitude=8.0, init_rows=0, seed=1000 + 31 * n + sd,
                 replica=sd)
            for n in modes for sd in range(nseed)]
