"""Whole-lattice one-step parity: one GPU step from the GPU's own state,
compared element by element with one oracle step from the same state.

The oracle is given the GPU state before the step (populations decoded to
float64, front heights, step counter and, under a division law, the GPU's
rate lam) and steps once; every population of every site and every column's
front height is then compared with the GPU's step.

Tolerances.  Float64: bit for bit.  Float32 arithmetic: per element
|df| <= 32 u max(rho, 1) + 1e-7 with u = 2^-24 (a site's update chains about
30 rounded operations on values up to rho: density and momentum sums, the
velocity, Eq. 3's polynomial, the relaxation and the noise; each rounding is
at most u of its operand), plus `round_ulps` ulps of the stored offset
f - W_i for the 16-bit storages.  A systematic error that stays inside that
bound is caught by the statistics of the differences over all tissue sites:
their mean must stay within u/4 of zero and their root mean square within
2 u, both relative to the mean tissue density (independent roundings give a
mean of order u / sqrt(n) and an r.m.s. of a few tenths of u).  Sites whose
tissue/void decision lies within 1e-5 of rho_c are checked against both
branches with the oracle's per-site step, and only their columns may have a
different front height.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as orc

U32 = 2.0 ** -24
_ULP_BITS = {"fp16": 10, "bf16": 7}
_W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
_W7 = np.array([1 / 2] + [1 / 12] * 6)


def storage_offsets(cfg):
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


def half_ulp(prec, v):
    """Half an ulp of v in the 16-bit storage format (0 otherwise)."""
    if prec not in _ULP_BITS:
        return np.zeros_like(v)
    a = np.maximum(np.abs(v), 2.0 ** -24 if prec == "fp16" else 2.0 ** -126)
    e = np.frexp(a)[1] - 1                      # floor(log2 a)
    if prec == "fp16":
        e = np.maximum(e, -14)
    return np.ldexp(0.5, e - _ULP_BITS[prec])


def _site_ok(p, cfg, f0, h0, t, lam, y, x, got, round_ulps):
    """A site outside the tolerance is accepted only if its streamed density
    is within 1e-5 of rho_c and the GPU took one of the two branches."""
    prec = cfg.get("precision", "fp32")
    W = storage_offsets(cfg)
    q = orc.q_of(p)
    fs = orc.pull_site(p, f0, x, y)
    rho_s = float(fs.sum())
    if abs(rho_s - cfg["rho_c"]) >= 1e-5:
        return False
    for force in (0, 1):
        out = orc.update_site(p, fs, t, x, y, int(h0[x]), 0, force, lam)[0][:q]
        tol = 32 * U32 * max(rho_s, 1.0) + 1e-7 + 2 * round_ulps * half_ulp(prec, out - W)
        if np.all(np.abs(got - out) <= tol):
            return True
    return False


def whole_step(sim, cfg, advance, round_ulps=0.5, label=None):
    """Step the GPU once with advance() and compare the whole lattice with
    one oracle step.  Returns a dict of difference statistics."""
    prec = cfg.get("precision", "fp32")
    label = label or cfg.get("name")
    f0 = sim.populations()
    h0 = sim.front_heights()
    t = sim.last_step
    d0 = sim.diagnostics()
    assert d0["y_wall"] == 0, "whole_step compares fixed-wall states"
    advance()
    f1 = sim.populations()
    h1 = sim.front_heights()
    assert sim.last_step == t + 1

    o = orc.Oracle(dict(cfg, precision="fp64"))
    o.set_populations(f0)
    o.set_front_heights(h0)
    o.set_step(t)
    if cfg.get("growth") in ("division", "division_density"):
        o.set_lam(d0["lam"])
    o.step(1)
    fo = o.populations()
    ho = o.front_heights()
    o.close()
    p = orc.make_params(dict(cfg, precision="fp64"))
    stats = {"case": label, "sites": int(f0.shape[1] * f0.shape[2])}

    if prec == "fp64":
        bad = np.nonzero(np.any(f1 != fo, axis=0))
        assert bad[0].size == 0, (label, "float64 sites differ", list(zip(*bad))[:10])
        assert np.array_equal(h1, ho), (label, np.nonzero(h1 != ho)[0][:10])
        stats.update(max_abs_diff=0.0, bitwise=True)
        return stats

    W = storage_offsets(cfg)
    rho = fo.sum(axis=0)
    scale = 32 * U32 * np.maximum(rho, 1.0) + 1e-7
    tissue = rho >= cfg["rho_c"]
    worst, s1, s2, n, sh = 0.0, 0.0, 0.0, 0, 0.0
    off_sites = set()
    for i in range(f0.shape[0]):
        d = f1[i] - fo[i]
        hu = half_ulp(prec, fo[i] - W[i])
        tol = scale + 2 * round_ulps * hu
        over = np.abs(d) > tol
        if np.any(over):
            ys, xs = np.nonzero(over)
            off_sites.update(zip(ys.tolist(), xs.tolist()))
            d = np.where(over, 0.0, d)
        worst = max(worst, float(np.max(np.abs(d))))
        dt = d[tissue]
        sh += float(hu[tissue].sum())
        s1 += float(dt.sum())
        s2 += float(np.dot(dt, dt))
        n += dt.size
    assert len(off_sites) <= 1000, (label, "sites outside the tolerance", len(off_sites),
                                   sorted(off_sites)[:10])
    near_cols = set()
    for y, x in sorted(off_sites):
        assert _site_ok(p, cfg, f0, h0, t, d0["lam"], y, x, f1[:, y, x], round_ulps), \
            (label, prec, "site", y, x, f1[:, y, x], fo[:, y, x])
        near_cols.add(x)
    # front heights: only columns holding a site decided within rounding of
    # rho_c may differ
    diff_cols = set(np.nonzero(h1 != ho)[0].tolist())
    if diff_cols - near_cols:
        # a site at the threshold can also round to the same branch on both
        # sides but with the other classification in the front height
        for x in sorted(diff_cols - near_cols):
            rows = range(min(f0.shape[1], max(int(h1[x]), int(ho[x])) + 2))
            near = any(abs(orc.pull_site(p, f0, x, y).sum() - cfg["rho_c"]) < 1e-5 for y in rows)
            assert near, (label, "front height differs", x, h1[x], ho[x])
    mean_rho = float(rho[tissue].mean()) if n else 1.0
    mean = s1 / max(n, 1)
    rms = (s2 / max(n, 1)) ** 0.5
    mean_half_ulp = sh / max(n, 1)
    stats.update(max_abs_diff=worst, mean_diff=mean, rms_diff=rms, mean_rho=mean_rho,
                 mean_half_ulp=mean_half_ulp, off_tolerance_sites=len(off_sites),
                 tissue_values=n, front_height_mismatches=len(diff_cols))
    # no systematic error: the float32 arithmetic's mean error stays within
    # u/4 of the density scale, and the storage rounding (to nearest or
    # stochastic, both unbiased) within a tenth of the stored values' mean
    # half ulp; the r.m.s. stays within 2 u plus the rounding's own spread
    assert abs(mean) <= 0.25 * U32 * mean_rho + 0.1 * mean_half_ulp, (label, "biased", stats)
    assert rms <= 2 * U32 * mean_rho + 2 * round_ulps * mean_half_ulp, (label, "rms", stats)
    return stats
