"""Float64 parity with the oracle over seeded random configurations: every
lattice, growth law, region, boundary, sweep window and launch shape the
library accepts, drawn together, on small ragged lattices, compared bit for
bit (to 1e-12) at several checkpoints."""
import numpy as np
import pytest

import synth_inputs as si
from oracle import oracle as orc
from tests.test_gpu_parity import _compare_fp64, _sim

pytestmark = pytest.mark.gpu


def _draw(seed):
    rng = np.random.default_rng(seed)
    lattice = str(rng.choice(["d2q9", "d2q7"]))
    ybc = str(rng.choice(["fixed", "follow", "periodic"]))
    L = int(rng.integers(5, 300))
    H = int(rng.integers(8, 120))
    if lattice == "d2q7" and ybc == "periodic":
        H += H % 2
    growth = str(rng.choice(["none", "bulk", "division", "division_density"]))
    region = str(rng.choice(["all", "front_band", "rear_band"]))
    vbs = [0, 1, 8, 16] + ([2] if lattice == "d2q9" else [])
    cfg = si.cfg(
        lattice=lattice, L=L, H=H, ybc=ybc, growth=growth, region=region,
        region_width=int(rng.integers(0, 12)),
        init_rows=int(rng.integers(1, max(2, H // 2))),
        init_amp=float(rng.choice([0.0, 1e-3, 0.1])),
        tau=float(rng.choice([0.6, 0.8, 1.0, 1.5])),
        mu=float(rng.choice([0.0, 1e-3, 1e-2])),
        sigma=float(rng.choice([0.0, 1e-3, 1e-2, 5e-2])),
        growth_rate=float(rng.choice([1e-3, 5e-3, 2e-2])),
        rho_c=float(rng.choice([0.3, 0.5])),
        wall_min_gap=int(rng.integers(4, 20)), wall_w_factor=float(rng.choice([0.0, 4.0, 10.0])),
        window=bool(ybc != "periodic" and rng.integers(0, 2)),
        division_map=bool(rng.integers(0, 2)),
        kernel_vb=int(rng.choice(vbs)), kernel_ty=int(rng.choice([0, 1, 2, 3, 5])),
        seed=int(rng.integers(0, 2 ** 31)), replica=int(rng.integers(0, 8)), precision="fp64")
    return cfg


@pytest.mark.parametrize("seed", range(150))
def test_fp64_random_configuration(seed):
    cfg = _draw(seed)
    sim = _sim(cfg)
    o = orc.Oracle(cfg)
    _compare_fp64(sim, o, (seed, 0))
    t = 0
    for c in (1, 2, 9, 40):
        sim.step(c - t)
        o.step(c - t)
        t = c
        if o.diagnostics()["status"]:
            break        # past the domain-full latch the state is not defined
        _compare_fp64(sim, o, (seed, t, cfg))
        dg, do = sim.diagnostics(), o.diagnostics()
        assert dg["divisions"] == do["divisions"] and dg["lam"] == do["lam"], (seed, t)
        if cfg["division_map"]:
            assert np.array_equal(sim.division_map(), o.division_map()), (seed, t)
    sim.close()
    o.close()
