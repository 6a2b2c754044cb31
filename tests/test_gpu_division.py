"""GPU parity of the discrete cell-division growth laws (Sec. II; Eq. 5)
through the C ABI.  Float64 runs must match the oracle bit for bit: the
Poisson counts are decided by the same float64 operations on both sides and
the rates come from integer tallies.  Reduced-precision runs are checked one
step at a time from the GPU's own state (uniform law: the per-site mean does
not depend on the site's density, so both sides draw the same counts)."""
import numpy as np
import pytest

import synth_inputs as si
from oracle import oracle as orc
from tests import d2q9
from tests.test_gpu_parity import _compare_fp64, _one_step_check, _sim

pytestmark = pytest.mark.gpu


def _compare_div(sim, o, where):
    err = _compare_fp64(sim, o, where)
    dg, do = sim.diagnostics(), o.diagnostics()
    assert dg["divisions"] == do["divisions"], (where, dg["divisions"], do["divisions"])
    assert dg["lam"] == do["lam"], (where, dg["lam"], do["lam"])
    return err


def _run(cfg, checkpoints):
    sim = _sim(cfg)
    o = orc.Oracle(cfg)
    _compare_div(sim, o, 0)
    t = 0
    for c in checkpoints:
        sim.step(c - t)
        o.step(c - t)
        t = c
        _compare_div(sim, o, t)
    d = sim.diagnostics()
    sim.close()
    o.close()
    return d


@pytest.fixture(params=["vector", "scalar", "staged"])
def kernel_form(request):
    return {"vector": {}, "scalar": {"kernel_vb": 1}, "staged": {"kernel_vb": 2}}[request.param]


@pytest.mark.parametrize("law", ["division", "division_density"])
@pytest.mark.parametrize("L,H", [(96, 64), (130, 48), (7, 40)])
def test_fp64_division_parity(law, L, H, kernel_form):
    cfg = si.cfg(L=L, H=H, init_rows=H // 3, tau=0.8, sigma=1e-2, growth=law, growth_rate=2e-2,
                 rho_cell=0.1, rho0=1.5, seed=21, replica=3, **kernel_form)
    d = _run(cfg, [1, 2, 15, 60])
    assert d["divisions"] > 100


def test_fp64_division_front_band_and_rear_band():
    # the front climbs from row 24 to about row 72 by step 150 (the top row
    # would latch the domain-full error, after which the state is not defined)
    d = _run(si.cfg(L=80, H=96, init_rows=24, sigma=1e-2, growth="division", growth_rate=1e-2,
                    region="front_band", region_width=4, seed=5), [1, 10, 80, 150])
    assert d["h_hi"] > 60 and d["status"] == 0
    # the rear band packs past rho0, its Eq. 5 weight goes to zero and the
    # mean per unit weight runs into the cap of 8, then no site is eligible
    d = _run(si.cfg(L=80, H=64, init_rows=24, sigma=1e-2, growth="division_density",
                    growth_rate=3e-2, region="rear_band", region_width=10, seed=6), [1, 10, 80])
    assert d["lam"] == 0.0


def test_fp64_division_follow_wall_and_window():
    # rows the wall leaves behind leave m_tot too (integer tallies on both sides)
    cfg = si.cfg(L=72, H=96, init_rows=70, sigma=1e-2, growth="division", growth_rate=2e-2,
                 ybc="follow", wall_min_gap=12, wall_w_factor=4.0, window=True, seed=8)
    d = _run(cfg, [1, 3, 40, 150])
    assert d["y_wall"] > 0 and d["retired"] > 0


def test_fp64_division_periodic_from_set_state():
    L, H = 40, 24
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.3, 1.6, (H, L))
    f = d2q9.equilibrium(rho, rng.uniform(-0.05, 0.05, (H, L)), rng.uniform(-0.05, 0.05, (H, L)))
    for law in ("division", "division_density"):
        cfg = si.cfg(L=L, H=H, init_rows=H, ybc="periodic", tau=0.7, sigma=1e-2, growth=law,
                     growth_rate=5e-2, seed=12)
        sim = _sim(cfg)
        o = orc.Oracle(cfg)
        sim.set_populations(f)
        o.set_populations(f)
        _compare_div(sim, o, (law, 0))
        sim.step(30)
        o.step(30)
        _compare_div(sim, o, (law, 30))
        sim.close()
        o.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_reduced_precision_division_one_step(prec):
    cfg = si.cfg(L=200, H=120, init_rows=50, tau=0.8, sigma=1e-3, growth="division",
                 growth_rate=5e-2, precision=prec, seed=2)
    sim = _sim(cfg)
    sim.front_heights()
    errs = [_one_step_check(sim, cfg, prec)]
    sim.step(30)
    sim.front_heights()
    errs.append(_one_step_check(sim, cfg, prec))
    print(prec, "division one-step max |diff|", errs)
    sim.close()


def test_division_count_matches_n_s_at_size():
    """1024 x 1024 all-tissue periodic float32 lattice: over 100 steps the
    divisions add up to the paper's n_s = g m_tot / rho_cell per step, within
    Poisson fluctuations, and their mass is the injected mass."""
    L = H = 1024
    cfg = si.cfg(L=L, H=H, init_rows=H, ybc="periodic", growth="division", growth_rate=1e-3,
                 rho_cell=0.1, sigma=1e-3, precision="fp32", seed=4)
    sim = _sim(cfg)
    expect = 0.0
    d = sim.diagnostics()
    for _ in range(100):
        expect += 1e-3 * d["mass"] / 0.1
        sim.step(1)
        d = sim.diagnostics()
    got = d["divisions"]
    assert abs(got - expect) <= 5 * np.sqrt(expect), (got, expect)
    assert d["src_total"] == pytest.approx(got * 0.1, rel=1e-6)
    sim.close()


@pytest.mark.parametrize("lattice", ["d2q9", "d2q7"])
def test_division_map_equals_the_oracle_map(lattice):
    """Per-site division counts, bit for bit, through a front band and a wall
    that follows the front (the map moves with the window), then cleared."""
    cfg = si.cfg(L=72, H=96, init_rows=70, sigma=1e-2, growth="division_density",
                 growth_rate=2e-2, ybc="follow", wall_min_gap=12, wall_w_factor=4.0, window=True,
                 division_map=True, lattice=lattice, seed=8)
    sim = _sim(cfg)
    o = orc.Oracle(cfg)
    t = 0
    for c in (1, 5, 60, 150):
        sim.step(c - t)
        o.step(c - t)
        t = c
        mg, mo = sim.division_map(), o.division_map()
        assert np.array_equal(mg, mo), (lattice, t, np.argwhere(mg != mo)[:5])
    assert sim.diagnostics()["y_wall"] > 0 and mg.sum() > 0
    sim.division_map(clear=True)
    o.division_map(clear=True)
    sim.step(3)
    o.step(3)
    assert np.array_equal(sim.division_map(), o.division_map())
    sim.close()
    o.close()


def test_division_map_in_a_batch_equals_solo():
    from paper_2303_02210_amd import Ensemble, Sim
    cfgs = [si.cfg(L=128, H=96, init_rows=40, growth="division", growth_rate=1e-2, sigma=1e-3,
                   region="front_band", region_width=6, division_map=True, precision=p, seed=s)
            for p, s in (("fp32", 1), ("fp64", 2))]
    ens = Ensemble(cfgs)
    ens.step(25)
    ens.synchronize()
    for c, m in zip(cfgs, ens.members):
        solo = Sim(c)
        solo.step(25)
        assert np.array_equal(m.division_map(), solo.division_map())
        assert m.division_map().sum() == m.diagnostics()["divisions"] > 0
        solo.close()
