"""The paper's own proliferation procedure (Sec. II; Eq. 5) in the oracle, and
what separates it from the per-site form the GPU library computes.

Sec. II: n_s = g m_tot / rho_cell cells divide per step, m_tot the total mass;
sites are drawn at random with replacement until that many divisions have
happened; under the density-dependent law a drawn site divides with
probability p_div of Eq. 5.  The oracle's selection mode
(``division_mode="selection"``) runs exactly that, with n_s rounded to an
integer stochastically.

Pins of the selection mode, each against a closed form or a distribution the
procedure must have: a single occupied site takes every division; each step
makes floor(n_s) or ceil(n_s) divisions, n_s on average; the divisions of a
step fall on the occupied sites multinomially (equal shares for the uniform
law, shares proportional to Eq. 5's p_div for the density law, none where
p_div is 0); the axes are uniform; each division puts rho_cell / 2 on both
directions of its axis.

Per-site form against the selection: the same mean number of divisions per
site and step, but the per-site form's total per step is Poisson (variance
n_s, sites independent) where the selection's is fixed (variance at most
1/4, each pair of sites correlated by -n_s / N^2 under the uniform law); the
fronts' h-bar(t) and w(t) of the two forms agree within their spread over
seeds.
"""
import math

import numpy as np
import pytest
from scipy import stats

import synth_inputs as si
from oracle import oracle as orc

from tests import d2q9


def _uniform_state(L, H, rho=1.0):
    r = np.full((H, L), rho)
    return d2q9.equilibrium(r, np.zeros_like(r), np.zeros_like(r))


def _steps_from(o, f, t):
    """One step of oracle o from populations f at step t."""
    o.set_populations(f)
    o.set_step(t)
    o.step(1)


def test_selection_draws_are_uniform():
    us, ua, ax = [], [], []
    for a in range(20000):
        u, v, b = orc.selection_draws(7, 3, 11, a)
        us.append(u)
        ua.append(v)
        ax.append((b * 4) >> 32)
        assert 0.0 < u < 1.0 and 0.0 < v < 1.0
    assert stats.kstest(us, "uniform").pvalue > 1e-4
    assert stats.kstest(ua, "uniform").pvalue > 1e-4
    assert stats.chisquare(np.bincount(ax, minlength=4)).pvalue > 1e-4
    r = [orc.selection_round_uniform(7, 3, t) for t in range(5000)]
    assert stats.kstest(r, "uniform").pvalue > 1e-4


def test_single_occupied_site_takes_every_division():
    """One site of density 1 in an empty lattice: after streaming only its
    rest population (4/9) stays, the neighbours receive 1/9 or 1/36; with
    rho_c = 0.2 it is the only occupied site, so all n_s = g m_tot / rho_cell
    divisions happen there and its mass grows by n_s rho_cell."""
    L, H = 9, 9
    f = np.zeros((9, H, L))
    f[:, 4, 4] = d2q9.W * 1.0
    g, rc = 0.5, 0.1                                      # n_s = 0.5 * 1 / 0.1 = 5
    cfg = si.cfg(L=L, H=H, init_rows=0, rho_c=0.2, growth="division", growth_rate=g,
                 rho_cell=rc, sigma=0.0, mu=0.0, division_mode="selection", seed=2)
    o = orc.Oracle(cfg)
    for t in range(20):
        _steps_from(o, f, t)
        c = o.selection_counts()
        assert c.sum() == 5 and c[4, 4].sum() == 5, (t, np.argwhere(c.sum(axis=2)))
        m = o.division_map(clear=True)
        assert m[4, 4] == 5 and m.sum() == 5
        fo = o.populations()
        assert fo[:, 4, 4].sum() == pytest.approx(4 / 9 + 5 * rc, rel=1e-14)
        assert fo.sum() == pytest.approx(1.0 + 5 * rc, rel=1e-14)
    o.close()


def test_count_per_step_is_n_s_rounded_and_unbiased():
    """A growing tissue with a fixed wall: the streamed state holds the mass
    of the state before it, so step t makes floor(n_s) or ceil(n_s)
    divisions, n_s = g M(t-1) / rho_cell, and n_s on average."""
    g, rc = 3e-3, 0.1
    cfg = si.cfg(L=24, H=64, init_rows=12, growth="division", growth_rate=g, rho_cell=rc,
                 sigma=1e-3, division_mode="selection", seed=5)
    o = orc.Oracle(cfg)
    dev, var = [], []
    for _ in range(300):
        d0 = o.diagnostics()
        ns = g * d0["mass"] / rc
        o.step(1)
        n = o.diagnostics()["divisions"] - d0["divisions"]
        assert n in (math.floor(ns), math.ceil(ns)), (n, ns)
        fr = ns - math.floor(ns)
        dev.append(n - ns)
        var.append(fr * (1 - fr))
    assert abs(sum(dev)) <= 4 * math.sqrt(sum(var)) + 1e-9, (sum(dev), math.sqrt(sum(var)))
    d = o.diagnostics()
    assert d["status"] == 0
    assert d["src_total"] == pytest.approx(d["divisions"] * rc, rel=1e-12)
    o.close()


def _trials(cfg, f, T):
    """Per-site divisions of T independent steps from the same state
    (selection counts summed over axes, or the division map)."""
    o = orc.Oracle(cfg)
    out = np.zeros((T,) + f.shape[1:], np.int64)
    for t in range(T):
        _steps_from(o, f, t)
        out[t] = o.division_map(clear=True)
    o.close()
    return out


def test_uniform_selection_is_multinomial_and_per_site_form_is_poisson():
    """64 occupied sites (periodic, uniform density 1), n_s = 16 per step.
    Selection: every step makes exactly 16 divisions, spread multinomially
    (per-site variance 16/64 (1 - 1/64), pair covariance -16/64^2).  Per-site
    form: independent Poisson counts of mean 1/4 (the total varies with
    variance 16; pairs uncorrelated).  Same mean per site."""
    L = H = 8
    N = L * H
    f = _uniform_state(L, H)
    base = si.cfg(L=L, H=H, init_rows=0, ybc="periodic", growth="division", growth_rate=0.025,
                  rho_cell=0.1, sigma=0.0, mu=0.0, seed=3)
    T = 3000
    sel = _trials(dict(base, division_mode="selection"), f, T).reshape(T, N)
    per = _trials(dict(base, division_mode="per_site"), f, T).reshape(T, N)
    n = 16
    assert np.all(sel.sum(axis=1) == n)
    # equal shares: chi-square of the pooled counts over the sites
    assert stats.chisquare(sel.sum(axis=0)).pvalue > 1e-4
    v_sel = sel.var(axis=0, ddof=1).mean()
    v_per = per.var(axis=0, ddof=1).mean()
    p = 1.0 / N
    assert v_sel == pytest.approx(n * p * (1 - p), rel=0.05)
    assert v_per == pytest.approx(n * p, rel=0.05)
    c_sel = np.cov(sel, rowvar=False)
    c_per = np.cov(per, rowvar=False)
    off = ~np.eye(N, dtype=bool)
    # mean pair covariance: -n/N^2 (selection) against 0 (per site); its
    # standard error over T steps and N(N-1) pairs is about var/(N sqrt(T))
    se = n * p / (N * math.sqrt(T))
    assert abs(c_sel[off].mean() + n / N ** 2) <= 5 * se, c_sel[off].mean()
    assert abs(c_per[off].mean()) <= 5 * se, c_per[off].mean()
    # totals: fixed against Poisson(16)
    tot = per.sum(axis=1)
    assert abs(tot.mean() - n) <= 5 * math.sqrt(n / T)
    assert tot.var(ddof=1) == pytest.approx(n, rel=0.12)
    assert abs(per.mean() - sel.mean()) <= 5 * math.sqrt(n * p / (T * N))


def test_density_selection_shares_follow_eq5():
    """A random density field (some sites below rho_c, some above rho0): each
    streamed site's share of the divisions is p_div / sum p_div with Eq. 5's
    p_div = 1 - rho*/rho0 above rho_c (0 otherwise, and 0 once rho* >= rho0);
    sites with p_div = 0 never divide."""
    L, H = 12, 10
    rng = np.random.default_rng(8)
    rho = rng.uniform(0.3, 1.8, size=(H, L))
    f = d2q9.equilibrium(rho, np.zeros_like(rho), np.zeros_like(rho))
    cfg = si.cfg(L=L, H=H, init_rows=0, ybc="periodic", growth="division_density",
                 growth_rate=0.01, rho_cell=0.1, rho0=1.5, rho_c=0.5, sigma=0.0, mu=0.0,
                 division_mode="selection", seed=6)
    p = orc.make_params(cfg)
    rho_s = np.array([[orc.pull_site(p, f, x, j).sum() for x in range(L)] for j in range(H)])
    pdiv = np.where(rho_s > 0.5, np.maximum(1.0 - rho_s / 1.5, 0.0), 0.0)
    T = 1500
    counts = _trials(cfg, f, T).sum(axis=0)
    assert np.all(counts[pdiv == 0.0] == 0)
    want = counts.sum() * pdiv / pdiv.sum()
    live = pdiv > 0
    assert stats.chisquare(counts[live], want[live]).pvalue > 1e-4
    # and every step's total is n_s rounded (m_tot of the streamed state)
    n_s = 0.01 * rho_s.sum() / 0.1
    assert abs(counts.sum() / T - n_s) <= 1.0


@pytest.mark.parametrize("lattice", ["d2q9", "d2q7"])
def test_selection_injects_half_a_cell_on_both_directions_of_uniform_axes(lattice):
    """With tau huge the update keeps the streamed populations (plus a
    relaxation of order 1/tau), so each direction's change is the injection:
    rho_cell / 2 times the divisions along its axis; the axes are uniform."""
    L, H = 10, 8
    q = 9 if lattice == "d2q9" else 7
    cfg = si.cfg(L=L, H=H, init_rows=0, ybc="periodic", lattice=lattice, tau=1e9, mu=0.0,
                 growth="division", growth_rate=0.05, rho_cell=0.1, sigma=0.0,
                 division_mode="selection", seed=9)
    if lattice == "d2q9":
        f = _uniform_state(L, H)
        axes = [(1, 3), (2, 4), (5, 7), (6, 8)]
    else:
        f = np.zeros((7, H, L))
        f[0] = 0.5
        f[1:] = 1.0 / 12.0
        axes = [(1, 4), (2, 5), (3, 6)]
    p = orc.make_params(cfg)
    o = orc.Oracle(cfg)
    per_axis = np.zeros(len(axes), np.int64)
    for t in range(60):
        _steps_from(o, f, t)
        c = o.selection_counts()
        fo = o.populations()
        per_axis += c.sum(axis=(0, 1))
        for j in range(H):
            for x in range(L):
                fs = orc.pull_site(p, f, x, j)
                dlt = fo[:, j, x] - fs[:q]
                want = np.zeros(q)
                for a, (i1, i2) in enumerate(axes):
                    want[i1] += c[j, x, a] * 0.05
                    want[i2] += c[j, x, a] * 0.05
                assert np.allclose(dlt, want, atol=1e-8), (t, j, x, dlt, want)
    o.close()
    assert stats.chisquare(per_axis).pvalue > 1e-4, per_axis


def _front_curves(cfg, seeds, steps, every):
    hb, ww = [], []
    for s in seeds:
        o = orc.Oracle(dict(cfg, seed=s, replica=s))
        h, w = [], []
        for _ in range(steps // every):
            o.step(every)
            d = o.diagnostics()
            h.append(d["hbar"])
            w.append(d["W"])
        assert o.diagnostics()["status"] == 0, "the run must stay inside its lattice"
        o.close()
        hb.append(h)
        ww.append(w)
    return np.array(hb), np.array(ww)


@pytest.mark.parametrize("law", ["division", "division_density"])
def test_per_site_form_and_selection_grow_the_same_fronts(law):
    """A tissue growing by discrete divisions (g = 0.01; rho0 = 4 rho_init,
    above the density at which the front advances), 8 seeds per form: the
    mean front height and width over seeds agree within 4 standard errors at
    every sampled time."""
    cfg = si.cfg(L=32, H=128, init_rows=12, tau=1.0, growth=law, growth_rate=1e-2,
                 rho_cell=0.1, rho0=4.0, sigma=1e-3, init_amp=0.1)
    seeds = range(8)
    steps, every = 300, 50
    hs, ws = _front_curves(dict(cfg, division_mode="selection"), seeds, steps, every)
    hp, wp = _front_curves(dict(cfg, division_mode="per_site"), seeds, steps, every)
    assert hs[:, -1].mean() > cfg["init_rows"] + 40, "the fronts must move"
    for a, b, name in ((hs, hp, "hbar"), (ws, wp, "W")):
        se = np.sqrt(a.var(axis=0, ddof=1) / a.shape[0] + b.var(axis=0, ddof=1) / b.shape[0])
        diff = np.abs(a.mean(axis=0) - b.mean(axis=0))
        assert np.all(diff <= 4 * se + 1e-9), (name, diff, se)


def test_per_site_form_stalls_where_the_eligible_weight_collapses():
    """The regime where the two forms part (stated, not hidden): with rho0 =
    2.5 rho_init the bulk reaches rho0 before the front can advance (about 3
    rho_init), so the weight sum q of the eligible sites collapses onto a few
    sites.  The selection procedure still makes n_s divisions per step there,
    all of them on those sites, and the fronts go on growing; the per-site
    form, whose mean per site is capped at 8 and whose rate is normalised by
    the previous step's weights, loses most of n_s and its fronts stop."""
    cfg = si.cfg(L=32, H=128, init_rows=12, tau=1.0, growth="division_density",
                 growth_rate=1e-2, rho_cell=0.1, rho0=2.5, sigma=1e-3, init_amp=0.1)
    seeds = range(8)
    hs, _ = _front_curves(dict(cfg, division_mode="selection"), seeds, 300, 100)
    hp, _ = _front_curves(dict(cfg, division_mode="per_site"), seeds, 300, 100)
    assert np.all(hp[:, -1] <= cfg["init_rows"] + 1)
    assert np.sum(hs[:, -1] > cfg["init_rows"] + 20) >= 4, hs[:, -1]
