"""GPU parity: the gfx950 library (through its C ABI) against the FP64 oracle.

Float64 runs must match the oracle to a relative error of 1e-12 (the same
operation order is used on both sides, so they are expected to match bit for
bit) with identical front heights.  Reduced-precision runs are checked one step
at a time from the GPU's own state, element by element, within a tolerance
derived from the float32 arithmetic and the storage rounding; sites whose
tissue/void decision sits within rounding of rho_c are checked against both
branches.
"""
import numpy as np
import pytest

import synth_inputs as si
from oracle import oracle as orc
from tests import d2q9

pytestmark = pytest.mark.gpu


def _sim(cfg):
    from paper_2303_02210_amd import Sim
    return Sim(cfg)


def _rel_err(a, b):
    scale = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / scale)


def _compare_fp64(sim, o, where):
    fg = sim.populations()
    fo = o.populations()
    err = _rel_err(fg, fo)
    assert err <= 1e-12, (where, err)
    hg = sim.front_heights()
    ho = o.front_heights()
    assert np.array_equal(hg, ho), (where, np.nonzero(hg != ho))
    dg = sim.diagnostics()
    do = o.diagnostics()
    for k in ("mass", "src_total", "fix_total", "retired"):
        assert abs(dg[k] - do[k]) <= 1e-12 * max(abs(do["mass"]), 1.0), (where, k, dg[k], do[k])
    assert dg["hbar"] == do["hbar"] and dg["W"] == do["W"], where
    assert dg["y_wall"] == do["y_wall"] and dg["h_hi"] == do["h_hi"], (where, dg, do)
    assert dg["status"] == do["status"]
    return err


def _run_fp64(cfg, checkpoints):
    sim = _sim(cfg)
    o = orc.Oracle(cfg)
    _compare_fp64(sim, o, 0)
    t = 0
    errs = []
    for c in checkpoints:
        sim.step(c - t)
        o.step(c - t)
        t = c
        errs.append(_compare_fp64(sim, o, t))
    sim.close()
    return errs


# ---------------------------------------------------------------- float64
def test_fp64_parity_64x64_workload_1000_steps():
    errs = _run_fp64(si.SMALL_FP64, [1, 2, 10, 100, 500, 1000])
    print("max rel err per checkpoint", errs)


@pytest.fixture(params=["vector", "scalar", "staged"])
def kernel_form(request):
    """The three forms of the step kernel: vectors of columns per lane (used
    when the width splits evenly into lanes), one column per lane, and rows
    staged through LDS by asynchronous global-to-LDS loads."""
    return {"vector": {}, "scalar": {"kernel_vb": 1}, "staged": {"kernel_vb": 2}}[request.param]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16"])
@pytest.mark.parametrize("L,H,ty", [(66, 40, 1), (130, 47, 3), (300, 64, 64), (1000, 90, 32),
                                    (2, 24, 2), (7, 30, 5)])
def test_staged_form_bitwise_equals_vector_form(prec, L, H, ty):
    """Every form runs the same per-site arithmetic, so the LDS-staged form
    must reproduce the vector form bit for bit: rows per block from 1 (no
    load ahead) to 64, ragged widths and heights, the wall following the
    front with the sweep window (ring rows), noise and front-band growth."""
    if prec in ("fp16", "bf16") and L % 2:
        pytest.skip("16-bit staged form needs an even width")
    base = si.cfg(L=L, H=H, init_rows=H // 3, tau=0.8, sigma=1e-2, growth_rate=2e-2,
                  region="front_band", region_width=3, precision=prec, seed=11, replica=1)
    for extra in ({}, {"ybc": "follow", "wall_min_gap": 4, "wall_w_factor": 2.0, "window": True}):
        cfg = dict(base, **extra)
        a = _sim(dict(cfg, kernel_vb=2, kernel_ty=ty))
        b = _sim(dict(cfg, kernel_vb=1))
        for n in (1, 2, 5, 40):
            a.step(n)
            b.step(n)
            fa, fb = a.populations(), b.populations()
            assert np.array_equal(fa, fb), (prec, L, H, ty, extra, n, np.argwhere(fa != fb)[:5])
            assert np.array_equal(a.front_heights(), b.front_heights())
        da, db = a.diagnostics(), b.diagnostics()
        for k in ("y_wall", "h_hi", "step", "status"):
            assert da[k] == db[k], k
        for k in ("mass", "src_total", "fix_total"):
            assert abs(da[k] - db[k]) <= 1e-9 * max(1.0, abs(db[k])), k
        a.close()
        b.close()


@pytest.mark.parametrize("L,H", [(300, 96), (130, 70), (7, 40)])
def test_fp64_parity_noise_front_band_ragged(L, H, kernel_form):
    cfg = si.cfg(L=L, H=H, init_rows=20, tau=0.8, sigma=1e-2, growth_rate=5e-3,
                 region="front_band", region_width=4, seed=3, replica=2, **kernel_form)
    _run_fp64(cfg, [1, 7, 50, 200])


def test_fp64_parity_rear_band_and_no_growth():
    _run_fp64(si.cfg(L=96, H=64, init_rows=30, sigma=1e-2, growth_rate=2e-2,
                     region="rear_band", region_width=10), [5, 120])
    _run_fp64(si.cfg(L=64, H=48, init_rows=20, sigma=1e-2, growth="none"), [5, 100])


def test_fp64_parity_follow_wall():
    cfg = si.cfg(L=72, H=128, init_rows=90, sigma=1e-2, growth_rate=1e-2, ybc="follow",
                 wall_min_gap=20, wall_w_factor=10.0, seed=9)
    errs = _run_fp64(cfg, [1, 2, 50, 150, 300])
    assert errs


def test_fp64_parity_window_flag():
    # the exact sweep window changes the work, never the result
    cfg = si.cfg(L=128, H=256, init_rows=40, sigma=1e-2, growth_rate=3e-3, window=True, seed=4)
    _run_fp64(cfg, [1, 3, 100, 300])
    cfg = dict(cfg, ybc="follow", wall_min_gap=10, wall_w_factor=10.0, H=160, init_rows=100)
    _run_fp64(cfg, [1, 3, 100, 300])


def test_fp64_parity_periodic_from_set_state():
    L, H = 70, 40
    rng = np.random.default_rng(5)
    rho = rng.uniform(0.6, 1.4, (H, L))
    f = d2q9.equilibrium(rho, rng.uniform(-0.1, 0.1, (H, L)), rng.uniform(-0.1, 0.1, (H, L)))
    cfg = si.cfg(L=L, H=H, init_rows=H, ybc="periodic", tau=0.7, sigma=1e-2, growth_rate=1e-3)
    sim = _sim(cfg)
    o = orc.Oracle(cfg)
    sim.set_populations(f)
    o.set_populations(f)
    assert np.array_equal(sim.populations(), o.populations())
    sim.step(60)
    o.step(60)
    assert _rel_err(sim.populations(), o.populations()) <= 1e-12


def test_fp64_parity_random_fronts_8x8():
    # brute force: random mixtures of tissue, sub-threshold and empty sites
    rng = np.random.default_rng(6)
    for trial in range(12):
        # 8 x 8 random rows under two empty rows (tissue in the last row
        # would end the run with DOMAIN_FULL)
        L, H = 8, 10
        cfg = si.cfg(L=L, H=H, init_rows=0, tau=0.8, sigma=1e-2, growth_rate=1e-2,
                     region="front_band", region_width=2, seed=trial)
        kind = rng.integers(0, 3, (H, L))
        kind[8:] = 2
        rho = np.where(kind == 0, rng.uniform(0.6, 1.4, (H, L)),
                       np.where(kind == 1, rng.uniform(0.0, 0.4, (H, L)), 0.0))
        f = np.maximum(d2q9.equilibrium(rho, rng.uniform(-.1, .1, (H, L)),
                                        rng.uniform(-.1, .1, (H, L))), 0.0)
        h0 = rng.integers(0, H + 1, L).astype(np.int32)
        sim = _sim(cfg)
        o = orc.Oracle(cfg)
        for s in (sim, o):
            s.set_populations(f)
            s.set_front_heights(h0)
        sim.step(1)
        o.step(1)
        assert np.array_equal(sim.populations(), o.populations()), trial
        assert np.array_equal(sim.front_heights(), o.front_heights()), trial
        sim.close()


# ---------------------------------------------------------------- reduced precision
_ULP_BITS = {"fp16": 10, "bf16": 7}


def _storage_half_ulp(prec, v):
    """Half an ulp of v in the 16-bit storage format (0 for fp32 storage)."""
    if prec not in _ULP_BITS:
        return np.zeros_like(v)
    a = np.maximum(np.abs(v), 2.0 ** -24 if prec == "fp16" else 2.0 ** -126)
    e = np.floor(np.log2(a))
    if prec == "fp16":
        e = np.maximum(e, -14)
    return 0.5 * 2.0 ** (e - _ULP_BITS[prec])


def _one_step_check(sim, cfg, prec):
    """One GPU step against the oracle's step from the GPU's own state."""
    f0 = sim.populations()
    h0 = sim.front_heights()
    t = sim.last_step
    lam = sim.diagnostics()["lam"]
    sim.step(1)
    f1 = sim.populations()
    h1 = sim.front_heights()
    o = orc.Oracle(dict(cfg, precision="fp64"))
    o.set_populations(f0)
    o.set_front_heights(h0)
    o.set_step(t)
    o.set_lam(lam)
    o.step(1)
    fr = o.populations()
    rho_s = d2q9.stream_pull(f0).sum(0)
    near = np.abs(rho_s - cfg["rho_c"]) < 1e-5
    # storage offsets W_i = w_i rho_ref in the storage type
    if prec in ("fp16", "bf16"):
        import numpy as _np
        W = d2q9.W * cfg.get("rho_ref", 1.0)
        if prec == "fp16":
            W = W.astype(_np.float32).astype(_np.float16).astype(_np.float64)
        else:
            b = W.astype(_np.float32).view(_np.uint32)
            b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
            W = b.astype(_np.uint32).view(_np.float32).astype(_np.float64)
    else:
        W = np.zeros(9)
    tol = (4e-6 * np.maximum(rho_s, 1.0))[None] + _storage_half_ulp(prec, fr - W[:, None, None]) \
        + 1e-7
    diff = np.abs(f1 - fr)
    bad = (diff > tol) & ~near[None]
    assert not bad.any(), (prec, t, np.argwhere(bad)[:5], diff[bad][:5], tol[bad][:5])
    # near-threshold sites: the GPU took one of the two branches
    for y, x in np.argwhere(near):
        fs = orc.pull_site(o.p, f0, int(x), int(y))
        ok = False
        for force in (0, 1):
            out, _, _, _ = orc.update_site(o.p, fs, t, int(x), int(y), int(h0[x]), 0, force, lam)
            ok = ok or np.all(np.abs(f1[:, y, x] - out) <= tol[:, y, x] + 1e-6)
        assert ok, (prec, t, y, x)
    cols = ~near.any(0)
    assert np.array_equal(h1[cols], o.front_heights()[cols])
    return float(np.max(diff[:, ~near])) if (~near).any() else 0.0


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("L", [200, 1000, 98])
def test_reduced_precision_one_step_parity(prec, L, kernel_form):
    cfg = si.cfg(L=L, H=160, init_rows=64, tau=0.8, sigma=1e-3, growth_rate=1e-3,
                 region="front_band", region_width=8, precision=prec, seed=1, **kernel_form)
    sim = _sim(cfg)
    sim.front_heights()
    errs = [_one_step_check(sim, cfg, prec)]
    sim.step(40)
    sim.front_heights()
    errs.append(_one_step_check(sim, cfg, prec))
    sim.step(200)
    sim.front_heights()
    errs.append(_one_step_check(sim, cfg, prec))
    print(prec, "max one-step |diff|", errs)


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_reduced_precision_void_is_exactly_empty(prec):
    cfg = si.cfg(L=128, H=128, init_rows=40, sigma=1e-3, growth_rate=1e-3, precision=prec)
    sim = _sim(cfg)
    sim.step(100)
    f = sim.populations()
    d = sim.diagnostics()
    assert np.all(f[:, d["h_hi"] + 1:, :] == 0.0)
    # mass balance closes to the storage rounding
    m0 = orc.Oracle(dict(cfg, precision="fp64")).diagnostics()["mass"]
    drift = d["mass"] - m0 - d["src_total"] - d["fix_total"]
    print(prec, "mass drift over 100 steps", drift, "relative", drift / d["mass"])
    limit = {"fp32": 1e-5, "fp16": 5e-3, "bf16": 5e-2}[prec]
    assert abs(drift) <= limit * d["mass"]


# ---------------------------------------------------------------- full size
def test_full_size_4096_fp32_whole_lattice_parity():
    """The throughput workload at its full size and launch configuration:
    one step checked against one oracle step on every site and column, plus
    the exactly empty void."""
    from tests.fullstep import whole_step
    cfg = dict(si.BULK_4096_FP32)
    sim = _sim(cfg)
    sim.step(20)
    stats = whole_step(sim, cfg, lambda: sim.step(1))
    d = sim.diagnostics()
    assert np.all(sim.populations()[:, d["h_hi"] + 1:, :] == 0.0)
    print("full-size whole-lattice step", stats)
    sim.close()


def test_rows_swept_counts_the_sweep_window():
    """lbm_diag.rows_swept: with the sweep window each step updates the rows
    up to the highest front so far plus one (the initial rows plus two on
    the first step); without it every step updates all H rows."""
    cfg = si.cfg(L=64, H=96, init_rows=20, sigma=1e-2, growth_rate=3e-2, window=True,
                 precision="fp32", seed=4)
    sim = _sim(cfg)
    assert sim.diagnostics()["rows_swept"] == 0
    want, hi = 0, None
    for k in range(60):
        want += min(cfg["H"], cfg["init_rows"] + 2 if k == 0 else max(1, hi + 2))
        sim.step(1)
        d = sim.diagnostics()
        assert d["rows_swept"] == want, (k, d["rows_swept"], want)
        hi = d["h_hi"]
    assert hi > cfg["init_rows"] + 2, "the front must move"
    sim.close()
    plain = _sim(dict(cfg, window=False))
    plain.step(7)
    assert plain.diagnostics()["rows_swept"] == 7 * cfg["H"]
    plain.close()


# ---------------------------------------------------------------- ABI behaviour
def test_domain_full_is_latched():
    from paper_2303_02210_amd import LbmError
    cfg = si.cfg(L=64, H=24, init_rows=20, growth_rate=5e-2)
    sim = _sim(cfg)
    sim.step(400)
    with pytest.raises(LbmError, match="DOMAIN_FULL"):
        sim.front_heights()
    with pytest.raises(LbmError, match="STATE"):
        sim.step(1)
    assert sim.diagnostics()["status"] & 1
    assert "top row" in sim.last_error()


def test_nonfinite_is_latched():
    from paper_2303_02210_amd import LbmError
    cfg = si.cfg(L=64, H=32, init_rows=10)
    sim = _sim(cfg)
    f = sim.populations()
    f[0, 3, 5] = np.nan
    sim.set_populations(f)
    sim.step(2)
    d = sim.diagnostics()
    assert d["status"] & 2
    with pytest.raises(LbmError):
        sim.front_heights()


def test_checkpoint_resume_is_bitwise():
    cfg = si.cfg(L=96, H=80, init_rows=30, tau=0.8, sigma=1e-2, growth_rate=5e-3,
                 precision="fp32", seed=11)
    a = _sim(cfg)
    a.step(20)
    blob = a.get_state()
    a.step(30)
    b = _sim(cfg)
    b.set_state(blob)
    b.step(30)
    assert np.array_equal(a.populations(), b.populations())
    assert np.array_equal(a.front_heights(), b.front_heights())
    da, db = a.diagnostics(), b.diagnostics()
    assert da == db


def test_front_heights_async_matches():
    import torch
    cfg = si.cfg(L=256, H=128, init_rows=30, sigma=1e-3, growth_rate=1e-3, precision="fp32")
    sim = _sim(cfg)
    dst = torch.empty(256, dtype=torch.int32).pin_memory()
    dev = torch.empty(256, dtype=torch.int32, device="cuda")
    sim.step(25)
    sim.front_heights_async(dst)
    sim.front_heights_async(dev)
    torch.cuda.synchronize()
    h = sim.front_heights()
    assert np.array_equal(dst.numpy(), h) and np.array_equal(dev.cpu().numpy(), h)
