"""GPU parity of the paper's triangular D2Q7 lattice (Sec. II) through the C
ABI: float64 bit for bit against the oracle (bulk growth, bands, noise,
ragged widths, the following wall with the sweep window, a periodic state
set from outside, both division laws), one-step checks of the reduced
precisions from the GPU's own state, and the host-side restrictions."""
import numpy as np
import pytest

import synth_inputs as si
from oracle import oracle as orc
from tests import d2q7
from tests.test_gpu_parity import _compare_fp64, _sim, _storage_half_ulp

pytestmark = pytest.mark.gpu


def cfg7(**kw):
    return si.cfg(lattice="d2q7", **kw)


def _run(cfg, checkpoints):
    sim = _sim(cfg)
    o = orc.Oracle(cfg)
    _compare_fp64(sim, o, 0)
    t = 0
    for c in checkpoints:
        sim.step(c - t)
        o.step(c - t)
        t = c
        _compare_fp64(sim, o, t)
        dg, do = sim.diagnostics(), o.diagnostics()
        assert dg["divisions"] == do["divisions"] and dg["lam"] == do["lam"], (t, dg, do)
    d = sim.diagnostics()
    sim.close()
    o.close()
    return d


def test_fp64_d2q7_64x64_bulk_1000_steps():
    _run(cfg7(L=64, H=64, init_rows=16, growth_rate=1e-3, sigma=1e-2, seed=3),
         [1, 2, 10, 100, 1000])


@pytest.mark.parametrize("L,H", [(130, 48), (7, 40), (256, 32)])
@pytest.mark.parametrize("ty", [0, 1, 3])
@pytest.mark.parametrize("vb", [0, 1, 16])
def test_fp64_d2q7_ragged_noise_front_band(L, H, ty, vb):
    # vb 0: the default (the vector form, 1 column per lane); 1: one column per
    # lane with direct neighbour loads; 16: the vector form with 2 columns per
    # lane (widths it does not divide run the one-column form)
    _run(cfg7(L=L, H=H, init_rows=H // 3, tau=0.8, sigma=1e-2, growth_rate=2e-3,
              region="front_band", region_width=4, seed=11, replica=2, kernel_ty=ty,
              kernel_vb=vb), [1, 7, 60])


def test_fp64_d2q7_rear_band_and_no_growth():
    _run(cfg7(L=96, H=64, init_rows=30, sigma=1e-2, growth_rate=5e-3, region="rear_band",
              region_width=6, seed=4), [1, 50])
    _run(cfg7(L=96, H=64, init_rows=30, sigma=1e-2, growth="none", seed=5), [1, 50])


@pytest.mark.parametrize("vb", [0, 1, 16])
def test_fp64_d2q7_follow_wall_and_window(vb):
    d = _run(cfg7(L=72, H=96, init_rows=70, sigma=1e-2, growth_rate=1e-2, ybc="follow",
                  wall_min_gap=12, wall_w_factor=4.0, window=True, seed=8, kernel_vb=vb),
             [1, 3, 40, 200])
    assert d["y_wall"] > 0


def test_fp64_d2q7_periodic_from_set_state():
    L, H = 40, 24
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.3, 1.6, (H, L))
    f = d2q7.equilibrium(rho, rng.uniform(-0.05, 0.05, (H, L)), rng.uniform(-0.05, 0.05, (H, L)))
    cfg = cfg7(L=L, H=H, init_rows=H, ybc="periodic", tau=0.7, sigma=1e-2, growth_rate=1e-3,
               seed=12)
    sim = _sim(cfg)
    o = orc.Oracle(cfg)
    sim.set_populations(f)
    o.set_populations(f)
    _compare_fp64(sim, o, 0)
    sim.step(40)
    o.step(40)
    _compare_fp64(sim, o, 40)
    sim.close()


@pytest.mark.parametrize("law", ["division", "division_density"])
@pytest.mark.parametrize("vb", [0, 1, 16])
def test_fp64_d2q7_division_laws(law, vb):
    d = _run(cfg7(L=96, H=64, init_rows=24, tau=0.8, sigma=1e-2, growth=law, growth_rate=2e-2,
                  seed=21, replica=3, kernel_vb=vb), [1, 2, 15, 60])
    assert d["divisions"] > 100


def _one_step_check7(sim, cfg, prec):
    f0 = sim.populations()
    h0 = sim.front_heights()
    t = sim.last_step
    lam = sim.diagnostics()["lam"]
    sim.step(1)
    f1 = sim.populations()
    o = orc.Oracle(dict(cfg, precision="fp64"))
    o.set_populations(f0)
    o.set_front_heights(h0)
    o.set_step(t)
    o.set_lam(lam)
    o.step(1)
    fr = o.populations()
    H, L = f0.shape[1:]
    rho_s = np.zeros((H, L))
    for j in range(H):
        for x in range(L):
            rho_s[j, x] = orc.pull_site(o.p, f0, x, j).sum()
    near = np.abs(rho_s - cfg["rho_c"]) < 1e-5
    W = np.zeros(7)
    if prec == "fp16":
        W = (d2q7.W * cfg.get("rho_ref", 1.0)).astype(np.float32).astype(np.float16).astype(np.float64)
    elif prec == "bf16":
        b = (d2q7.W * cfg.get("rho_ref", 1.0)).astype(np.float32).view(np.uint32)
        b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
        W = b.astype(np.uint32).view(np.float32).astype(np.float64)
    tol = (4e-6 * np.maximum(rho_s, 1.0))[None] + _storage_half_ulp(prec, fr - W[:, None, None]) \
        + 1e-7
    diff = np.abs(f1 - fr)
    bad = (diff > tol) & ~near[None]
    assert not bad.any(), (prec, t, np.argwhere(bad)[:5], diff[bad][:5], tol[bad][:5])
    return float(np.max(diff[:, ~near])) if (~near).any() else 0.0


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_reduced_precision_d2q7_one_step(prec):
    cfg = cfg7(L=160, H=96, init_rows=40, tau=0.8, sigma=1e-3, growth_rate=1e-3,
               region="front_band", region_width=8, precision=prec, seed=1)
    sim = _sim(cfg)
    errs = [_one_step_check7(sim, cfg, prec)]
    sim.step(40)
    errs.append(_one_step_check7(sim, cfg, prec))
    print(prec, "D2Q7 one-step max |diff|", errs)
    sim.close()


@pytest.mark.parametrize("prec,vb", [("fp32", 4), ("fp32", 8), ("fp16", 4), ("fp16", 8),
                                     ("bf16", 4), ("fp64", 16)])
def test_d2q7_vector_form_bitwise_equals_one_column_form(prec, vb):
    """The launch shape never changes results: the vector form against the
    one-column form, bit for bit, with noise, a front band and divisions."""
    for growth in ("bulk", "division_density"):
        base = cfg7(L=256, H=96, init_rows=40, tau=0.8, sigma=1e-2, growth=growth,
                    growth_rate=5e-3, region="front_band", region_width=6, precision=prec,
                    seed=9)
        a = _sim(dict(base, kernel_vb=1))
        b = _sim(dict(base, kernel_vb=vb))
        for n in (1, 10, 40):
            a.step(n)
            b.step(n)
            assert np.array_equal(a.populations(), b.populations()), (prec, vb, growth, n)
            assert np.array_equal(a.front_heights(), b.front_heights())
            da, db = a.diagnostics(), b.diagnostics()
            assert da["divisions"] == db["divisions"] and da["lam"] == db["lam"]
            assert abs(da["mass"] - db["mass"]) <= 1e-9 * da["mass"]
        a.close()
        b.close()


def test_d2q7_populations_round_trip():
    cfg = cfg7(L=64, H=32, init_rows=10, precision="fp32")
    sim = _sim(cfg)
    f = sim.populations()
    assert f.shape == (7, 32, 64)
    assert np.allclose(f[:, :10].sum(0), 1.0, atol=2e-3)
    sim.set_populations(f)
    assert np.array_equal(sim.populations(), f)
    sim.close()


def test_d2q7_batch_members_match_solo_runs_bitwise():
    """D2Q7 members (their own step kernel) batched beside D2Q9 members, with
    per-step launches and with multi-step cooperative launches."""
    from paper_2303_02210_amd import Ensemble
    from tests.test_gpu_batch import _same, _solo
    cfgs = [cfg7(L=128, H=192, init_rows=48, growth_rate=5e-3, sigma=1e-3, precision="fp32", seed=1),
            si.cfg(L=128, H=192, init_rows=48, growth_rate=5e-3, sigma=1e-3, precision="fp32", seed=1),
            cfg7(L=96, H=128, init_rows=60, sigma=1e-2, growth="division_density", growth_rate=1e-2,
                 ybc="follow", wall_min_gap=10, window=True, precision="fp64", seed=2),
            cfg7(L=200, H=96, init_rows=30, growth_rate=1e-3, sigma=1e-3, region="front_band",
                 region_width=6, precision="fp16", seed=3, kernel_ty=3),
            cfg7(L=256, H=128, init_rows=40, growth_rate=2e-3, sigma=1e-3, precision="fp16",
                 seed=4, kernel_vb=4, kernel_ty=4),
            cfg7(L=128, H=96, init_rows=40, growth="division", growth_rate=1e-2, sigma=1e-2,
                 precision="fp64", seed=5, kernel_vb=16)]
    for persistent in (False, True):     # per-step launches; one launch per run
        ens = Ensemble(cfgs, persistent=persistent)
        for n in (8, 8, 13):
            ens.step(n)
        ens.synchronize()
        for i, (c, m) in enumerate(zip(cfgs, ens.members)):
            _same(m, _solo(c, 29), (persistent, i))
        ens.close()


def test_full_size_4096_d2q7_fp32_whole_lattice_parity():
    """4096 x 4096 D2Q7 in its default launch shape: one step checked against
    one oracle step on every site and column."""
    from tests.fullstep import whole_step
    cfg = dict(si.BULK_4096_FP32, lattice="d2q7")
    sim = _sim(cfg)
    sim.step(20)
    stats = whole_step(sim, cfg, lambda: sim.step(1))
    d = sim.diagnostics()
    assert np.all(sim.populations()[:, d["h_hi"] + 1:, :] == 0.0)
    print("d2q7 full-size whole-lattice step", stats)
    sim.close()


@pytest.mark.parametrize("kw", [dict(lattice="d2q7"),
                                dict(growth="division_density", growth_rate=2e-2),
                                dict(lattice="d2q7", growth="division", growth_rate=2e-2,
                                     ybc="follow", wall_min_gap=10, window=True,
                                     division_map=True)])
def test_checkpoint_resume_is_bitwise(kw):
    """A restored run continues bit for bit, division rate, counts and the
    device-driven window included."""
    cfg = si.cfg(**dict(dict(L=96, H=80, init_rows=40, tau=0.8, sigma=1e-2, growth_rate=5e-3,
                             precision="fp32", seed=11), **kw))
    a = _sim(cfg)
    a.step(20)
    blob = a.get_state()
    a.step(30)
    b = _sim(cfg)
    b.set_state(blob)
    b.step(30)
    assert np.array_equal(a.populations(), b.populations())
    assert np.array_equal(a.front_heights(), b.front_heights())
    assert a.diagnostics() == b.diagnostics()
    a.close()
    b.close()
