"""Stochastic rounding of 16-bit storage (LBM_FLAG_STOCHASTIC_ROUND): each
stored offset is within one ulp of the oracle's value (against half an ulp
when rounding to nearest), it is either of the two neighbours of the value
rounded to nearest, the rounding is unbiased (a growth increment below half
an ulp, which rounding to nearest loses every step, is kept on average), and
batched runs match solo runs bit for bit."""
import numpy as np
import pytest

import synth_inputs as si
from tests.fullstep import whole_step
from tests.test_gpu_fullsize import _half_ulp, _storage_offsets

pytestmark = pytest.mark.gpu


def _sim(cfg):
    from paper_2303_02210_amd import Sim
    return Sim(cfg)


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("lattice", ["d2q9", "d2q7"])
@pytest.mark.parametrize("form", [dict(), dict(kernel_vb=1), dict(kernel_vb=16, kernel_ty=2)])
@pytest.mark.parametrize("growth", ["bulk", "division"])
def test_one_step_within_one_ulp(prec, lattice, form, growth):
    cfg = si.cfg(lattice=lattice, L=200, H=96, init_rows=50, init_amp=0.1, tau=0.8, sigma=1e-2,
                 growth=growth, growth_rate=2e-2, rho_init=2.0, rho_ref=1.0, precision=prec,
                 stochastic_round=True, seed=5, **form)
    sim = _sim(cfg)
    sim.step(10)
    sim.front_heights()
    stats = whole_step(sim, cfg, lambda: sim.step(1), round_ulps=1.0)
    print(prec, lattice, form, growth, stats)
    sim.close()


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("lattice", ["d2q9", "d2q7"])
def test_stochastic_result_is_a_neighbour_of_the_nearest(prec, lattice):
    """From one state, one step with and one without stochastic rounding (no
    noise, so the two runs compute the same float32 values): every stored
    value agrees or differs by one ulp of the storage, and a good share of
    the tissue values differ (the rounding is active)."""
    base = si.cfg(lattice=lattice, L=128, H=64, init_rows=40, init_amp=0.1, tau=0.8,
                  sigma=0.0, growth_rate=1e-2, rho_init=2.0, rho_ref=1.0, precision=prec, seed=9)
    a = _sim(base)
    a.step(5)
    f0 = a.populations()
    h0 = a.front_heights()
    b = _sim(dict(base, stochastic_round=True))
    b.set_populations(f0)
    b.set_front_heights(h0)
    a.step(1)
    b.step(1)
    fa, fb = a.populations(), b.populations()
    W = _storage_offsets(base)[:, None, None]
    d = np.abs(fa - fb)
    ulp = 2 * _half_ulp(prec, np.maximum(np.abs(fa - W), np.abs(fb - W)))
    assert np.all((d == 0) | (np.abs(d - ulp) <= 1e-12 * np.maximum(1.0, np.abs(fa)))
                  | (np.abs(d - ulp / 2) <= 1e-12 * np.maximum(1.0, np.abs(fa))))
    live = (fa.sum(0) > 0)
    frac = float((d[:, live] > 0).mean())
    print(prec, lattice, "share of stored values that differ", frac)
    assert 0.05 < frac < 0.95
    a.close()
    b.close()


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_rounding_is_unbiased(prec):
    """A uniform all-tissue periodic lattice at rho = 3 (offsets stored about
    rho_ref = 1), at rest, growing by g = 1e-3 per step: every increment
    w_i g rho is below half an ulp of its BF16 offset, so rounding to nearest
    stores none of them and the stored mass stays put; stochastic rounding
    keeps the stored mass equal to the injected mass to within its
    statistical spread (about 8 over 200 steps here)."""
    cfg = si.cfg(L=128, H=64, ybc="periodic", init_rows=64, init_amp=0.0, rho_init=3.0,
                 rho_ref=1.0, tau=1.0, mu=0.0, sigma=0.0, growth_rate=1e-3, precision=prec,
                 seed=4)
    out = {}
    for sr in (False, True):
        sim = _sim(dict(cfg, stochastic_round=sr))
        m0 = sim.diagnostics()["mass"]
        sim.step(200)
        d = sim.diagnostics()
        out[sr] = (d["mass"] - m0, d["src_total"])
        sim.close()
    gained, injected = out[True]
    print(prec, "rounding to nearest: stored", out[False][0], "of", out[False][1],
          "; stochastic: stored", gained, "of", injected)
    assert injected > 5000
    assert abs(gained - injected) < 60.0
    if prec == "bf16":
        # to nearest, the increments are lost (after the first step settles
        # the initial rounding)
        assert abs(out[False][0]) < 0.2 * out[False][1]


def test_batch_members_match_solo_runs():
    from paper_2303_02210_amd import Ensemble
    cfgs = [si.cfg(L=96, H=64, init_rows=30, init_amp=0.1, sigma=1e-2, growth_rate=1e-2,
                   rho_init=2.0, rho_ref=1.0, precision=p, lattice=lat, stochastic_round=True,
                   seed=20 + i, replica=i)
            for i, (p, lat) in enumerate([("fp16", "d2q9"), ("bf16", "d2q9"), ("fp16", "d2q7"),
                                          ("bf16", "d2q7")])]
    cfgs.append(dict(cfgs[0], stochastic_round=False, seed=30))
    # a windowed member with a following wall (a group whose tile table the
    # device rebuilds each step)
    cfgs.append(si.cfg(L=64, H=96, init_rows=60, init_amp=0.1, sigma=1e-2, growth_rate=2e-2,
                       rho_init=2.0, rho_ref=1.0, precision="bf16", stochastic_round=True,
                       ybc="follow", wall_min_gap=12, wall_w_factor=2.0, window=True, seed=41))
    ens = Ensemble(cfgs)
    ens.step(7)
    ens.step(9)
    ens.synchronize()
    for c, m in zip(cfgs, ens.members):
        s = _sim(c)
        s.step(16)
        assert np.array_equal(m.populations(), s.populations()), c
        assert np.array_equal(m.front_heights(), s.front_heights()), c
        s.close()
    ens.close()
