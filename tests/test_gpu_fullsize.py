"""Parity at the throughput workloads' full sizes, in the launch shapes the
benchmark times (library defaults and the shipped tuned shapes): one GPU step
from the GPU's own state against one oracle step from the same state, on
every site and every column (``tests/fullstep.py``: float64 bit for bit; the
reduced precisions within the float32-arithmetic bound plus the storage
rounding, with the mean and r.m.s. of the differences checked for bias).

The largest accepted lattice (2^31 populations, 17 GB per float64 copy) is
checked on sampled sites and every live row of sampled columns instead
(``_sampled_step``), with the same per-element tolerance.
"""
import numpy as np
import pytest

import synth_inputs as si
from oracle import oracle as orc
from tests.fullstep import U32, whole_step

pytestmark = pytest.mark.gpu

_ULP_BITS = {"fp16": 10, "bf16": 7}
_W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
_W7 = np.array([1 / 2] + [1 / 12] * 6)


def _storage_offsets(cfg):
    """W_i = w_i rho_ref rounded to the storage format (0 for fp32/fp64)."""
    prec = cfg.get("precision", "fp32")
    w = _W7 if cfg.get("lattice", "d2q9") == "d2q7" else _W9
    W = w * cfg.get("rho_ref", 1.0)
    if prec == "fp16":
        return W.astype(np.float32).astype(np.float16).astype(np.float64)
    if prec == "bf16":
        b = W.astype(np.float32).view(np.uint32)
        b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
        return b.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.zeros_like(W)


def _half_ulp(prec, v):
    if prec not in _ULP_BITS:
        return np.zeros_like(v)
    a = np.maximum(np.abs(v), 2.0 ** -24 if prec == "fp16" else 2.0 ** -126)
    e = np.floor(np.log2(a))
    if prec == "fp16":
        e = np.maximum(e, -14)
    return 0.5 * 2.0 ** (e - _ULP_BITS[prec])


def _sampled_step(sim, cfg, advance, nsites=3000, ncols=4, seed=0, extra=(), round_ulps=0.5):
    """Step once with `advance()` and check the step against the oracle
    (on sampled sites, the sites in `extra`, and every live row of sampled
    columns).  round_ulps: the storage rounding allowed (half an ulp to
    nearest, one ulp stochastically)."""
    prec = cfg.get("precision", "fp32")
    f0 = sim.populations()
    h0 = sim.front_heights()
    t = sim.last_step
    lam = sim.diagnostics()["lam"]
    advance()
    f1 = sim.populations()
    h1 = sim.front_heights()
    assert sim.last_step == t + 1
    p = orc.make_params(dict(cfg, precision="fp64"))
    q = orc.q_of(p)
    W = _storage_offsets(cfg)
    rng = np.random.default_rng(seed)
    L, H = cfg["L"], cfg["H"]
    # rows that can hold tissue after the step: up to two above the highest
    # row with any mass (sub-threshold mass above the front can cross rho_c)
    massive = np.nonzero(f0.any(axis=(0, 2)))[0]
    top = min(H, int(massive.max()) + 3 if massive.size else 2)
    sites = [(int(rng.integers(0, top)), int(rng.integers(0, L))) for _ in range(nsites)]
    sites += [(int(rng.integers(0, H)), int(rng.integers(0, L))) for _ in range(nsites // 6)]
    sites += list(extra)
    cols = sorted({0, L - 1, *[int(v) for v in rng.integers(0, L, ncols)]})
    for x in cols:
        sites += [(y, x) for y in range(top)]
    worst = 0.0
    for y, x in sites:
        fs = orc.pull_site(p, f0, x, y)
        rho_s = fs.sum()
        got = f1[:, y, x]
        if prec == "fp64":
            out = orc.update_site(p, fs, t, x, y, int(h0[x]), 0, -1, lam)[0][:q]
            assert np.array_equal(got, out), (cfg.get("name"), y, x, got - out)
            continue
        branches = (-1,) if abs(rho_s - cfg["rho_c"]) >= 1e-5 else (0, 1)
        ok = False
        for force in branches:
            out = orc.update_site(p, fs, t, x, y, int(h0[x]), 0, force, lam)[0][:q]
            tol = 32 * U32 * max(rho_s, 1.0) + 1e-7 + 2 * round_ulps * _half_ulp(prec, out - W)
            d = np.abs(got - out)
            if np.all(d <= tol):
                ok = True
                if force == -1:
                    worst = max(worst, float(d.max()))
                break
        assert ok, (cfg.get("name"), prec, y, x, got, out)
    for x in cols:
        rows = [y for y in range(top) if orc.pull_site(p, f0, x, y).sum() >= cfg["rho_c"]]
        near = any(abs(orc.pull_site(p, f0, x, y).sum() - cfg["rho_c"]) < 1e-5
                   for y in range(top))
        if not near:
            assert h1[x] == (max(rows) + 1 if rows else 0), (x, h1[x])
    d = sim.diagnostics()
    assert d["status"] == 0
    if cfg.get("ybc", "fixed") != "periodic":   # periodic rows wrap mass to the top
        assert np.all(f1[:, d["h_hi"] + 1:, :] == 0.0)
    return worst


def _tuned(cfg):
    from paper_2303_02210_amd import autotune
    c = autotune.apply(cfg)
    assert "kernel_vb" in c, ("no tuned shape shipped for", autotune.key(cfg))
    return c


_EDGE = si.EDGE_2048x8192
_BULK = si.BULK_4096_FP32
_CASES = {
    "edge_fp32": dict(_EDGE, precision="fp32"),
    "edge_fp32_tuned": ("tuned", dict(_EDGE, precision="fp32")),
    "edge_fp16": dict(_EDGE, precision="fp16"),
    "edge_fp16_tuned": ("tuned", dict(_EDGE, precision="fp16")),
    "edge_bf16": dict(_EDGE, precision="bf16"),
    "edge_bf16_tuned": ("tuned", dict(_EDGE, precision="bf16")),
    "bulk_fp16": dict(_BULK, precision="fp16"),
    "bulk_bf16": dict(_BULK, precision="bf16"),
    "bulk_fp64": dict(_BULK, precision="fp64"),
    "division_fp32_tuned": ("tuned", dict(_BULK, growth="division")),
    "division_fp16_tuned": ("tuned", dict(_BULK, precision="fp16", growth="division")),
    "division_density_fp32": dict(_BULK, growth="division_density"),
    "d2q7_fp16": dict(_BULK, precision="fp16", lattice="d2q7"),
    "d2q7_fp64": dict(_BULK, precision="fp64", lattice="d2q7"),
    "d2q7_bf16": dict(_BULK, precision="bf16", lattice="d2q7"),
    "d2q7_division_fp32": dict(_BULK, lattice="d2q7", growth="division"),
    "d2q7_division_density_fp64": dict(_BULK, precision="fp64", lattice="d2q7",
                                       growth="division_density"),
    "bulk_fp16_sr_tuned": ("tuned", dict(_BULK, precision="fp16", stochastic_round=True)),
    "edge_bf16_sr_tuned": ("tuned", dict(_EDGE, precision="bf16", stochastic_round=True)),
}


# (the shipped tuned shapes of the 4096 x 4096 bulk workload are the
# library defaults)
_CASES.update({
    "bulk_fp32": dict(_BULK, precision="fp32"),
    "edge_fp16_sr_tuned": ("tuned", dict(_EDGE, precision="fp16", stochastic_round=True)),
    "bulk_bf16_sr_tuned": ("tuned", dict(_BULK, precision="bf16", stochastic_round=True)),
})


@pytest.mark.parametrize("name", list(_CASES))
def test_full_size_whole_lattice_step(name):
    from paper_2303_02210_amd import Sim
    case = _CASES[name]
    cfg = _tuned(case[1]) if isinstance(case, tuple) else case
    sim = Sim(cfg)
    sim.step(20)
    sim.front_heights()
    ulps = 1.0 if cfg.get("stochastic_round") else 0.5
    stats = whole_step(sim, cfg, lambda: sim.step(1), round_ulps=ulps, label=name)
    print(name, {k: cfg.get(k) for k in ("kernel_vb", "kernel_ty")}, stats)
    sim.close()


@pytest.mark.parametrize("lattice,prec", [("d2q9", "fp32"), ("d2q9", "fp64"), ("d2q7", "fp32")])
def test_largest_lattice_sampled_step(lattice, prec):
    """The largest lattice the library accepts (L * H * Q just under 2^31
    populations: the highest offsets of every buffer), tissue nearly to the
    top: one step checked on sampled sites and on the last rows and columns."""
    from paper_2303_02210_amd import Sim
    q = 9 if lattice == "d2q9" else 7
    L = 16384
    H = (1 << 31) // (q * L)
    cfg = si.cfg(name=f"largest_{lattice}_{prec}", lattice=lattice, L=L, H=H, init_rows=H - 40,
                 init_amp=0.1, tau=0.8, sigma=1e-3, growth_rate=1e-4, precision=prec, seed=3)
    sim = Sim(cfg)
    sim.step(3)
    sim.front_heights()
    top = H - 40
    extra = [(y, x) for y in range(top - 6, top + 3) for x in (0, 1, L - 2, L - 1)]
    extra += [(y, x) for y in (0, 1, H // 2) for x in (L - 2, L - 1)]
    worst = _sampled_step(sim, cfg, lambda: sim.step(1), nsites=1500, ncols=1, seed=1,
                          extra=extra)
    print(cfg["name"], L, "x", H, "max |diff|", worst)
    sim.close()


@pytest.mark.parametrize("solo_min_sites", [None, "default"])
def test_full_size_ensemble_whole_members(solo_min_sites):
    """The 256-replica ensemble (476 M sites) in its tuned shapes, stepped as
    one batch (None) or with its large members stepped alone (the default):
    one ensemble step checked on every site of the smallest, a middle and
    the largest member."""
    from paper_2303_02210_amd import Ensemble
    cfgs = [_tuned(c) for c in si.ensemble()]
    ens = Ensemble(cfgs) if solo_min_sites == "default" else Ensemble(cfgs, solo_min_sites=None)
    ens.step(20)
    ens.synchronize()
    picks = [0, 150, len(cfgs) - 1]
    for i in picks:
        m = ens.members[i]
        m.front_heights()
    # each pick steps the whole batch once; the other picks are checked after
    # their own batch step, from their state at that time
    for n, i in enumerate(picks):
        m = ens.members[i]
        m.front_heights()
        stats = whole_step(m, cfgs[i], lambda: (ens.step(1), ens.synchronize()),
                           label=f"member {i}")
        print("member", i, cfgs[i]["L"], "x", cfgs[i]["H"], stats)
    ens.close()
