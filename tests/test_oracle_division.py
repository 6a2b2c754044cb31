"""Pins of the oracle's discrete cell-division growth laws (Sec. II; Eq. 5),
each checked against something other than the oracle's own formulas: the
exponential and Poisson laws from scipy, moment conservation, the expected
division count n_s = g m_tot / rho_cell, the acceptance probability of Eq. 5,
and a literal replay of the paper's selection of sites with replacement."""
import math

import numpy as np
import pytest
from scipy import stats

import synth_inputs as si
from oracle import oracle as orc

from tests import d2q9


def test_exp_neg_matches_exp():
    assert orc.exp_neg(0.0) == 1.0
    for lam in np.concatenate([np.linspace(0.0, 8.0, 801), [1e-12, 1e-6, 0.0625, 7.999999]]):
        want = math.exp(-lam)
        assert abs(orc.exp_neg(lam) - want) <= 4e-15 * want, lam


@pytest.mark.parametrize("lam", [0.01, 0.3, 1.0, 2.5, 7.9])
def test_poisson_inversion_reproduces_the_pmf(lam):
    # an even grid of U: each k takes exactly a pmf(k)-long piece of (0, 1)
    n = 200_000
    ks = np.array([orc.poisson_k((i + 0.5) / n, lam) for i in range(n)])
    kmax = int(ks.max())
    freq = np.bincount(ks, minlength=kmax + 1) / n
    pmf = stats.poisson.pmf(np.arange(kmax + 1), lam)
    assert np.all(np.abs(freq - pmf) <= 1.0 / n + 1e-12), (freq[:6], pmf[:6])
    # and pointwise against scipy's quantile function away from the jumps
    rng = np.random.default_rng(1)
    cdf = stats.poisson.cdf(np.arange(40), lam)
    for U in rng.random(2000):
        if np.min(np.abs(cdf - U)) < 1e-9:
            continue
        assert orc.poisson_k(U, lam) == int(stats.poisson.ppf(U, lam)), (U, lam)


def test_poisson_count_is_capped():
    assert orc.poisson_k(1.0 - 2.0 ** -52, 8.0) <= 32
    assert orc.poisson_k(0.5, 0.0) == 0


def test_division_draws_are_uniform():
    U = []
    fields = []
    for x in range(100):
        for y in range(100):
            u, ax = orc.division_draws(3, 1, 17, x, y)
            U.append(u)
            fields.append([(ax >> (2 * d)) & 3 for d in range(4)])
            n = u * 2.0 ** 52 - 0.5
            assert n == int(n) and 0 <= n < 2 ** 52
    assert stats.kstest(U, "uniform").pvalue > 1e-4
    # every one of the 52 bits of U's numerator is a fair coin
    nums = np.array([int(u * 2.0 ** 52 - 0.5) for u in U], dtype=np.uint64)
    for b in range(52):
        ones = float(((nums >> np.uint64(b)) & np.uint64(1)).mean())
        assert 0.45 < ones < 0.55, (b, ones)
    f = np.array(fields)
    for d in range(4):
        assert stats.chisquare(np.bincount(f[:, d], minlength=4)).pvalue > 1e-4
    # neighbouring counters give unrelated draws
    assert abs(np.corrcoef(U[:-1], U[1:])[0, 1]) < 0.05


def test_division_injects_cell_mass_on_opposite_pairs():
    """With tau huge the relaxation leaves the populations (almost) alone,
    so the update is the injection itself: rho_cell / 2 on both directions of
    each drawn axis, no momentum, mass k rho_cell."""
    cfg = si.cfg(L=8, H=8, growth="division", growth_rate=1e-2, rho_cell=0.1, tau=1e12, mu=0.0,
                 sigma=0.0, seed=5, replica=2)
    p = orc.make_params(cfg)
    opp, w = d2q9.OPP, d2q9.W
    rng = np.random.default_rng(2)
    seen = 0
    for trial in range(200):
        fstar = w * rng.uniform(0.8, 1.2) + rng.uniform(0.0, 0.01, 9)
        t, x, y = int(rng.integers(0, 1000)), int(rng.integers(0, 8)), int(rng.integers(0, 8))
        out, tissue, S, dfix, k, wfx = orc.update_site_ex(p, fstar, t, x, y, 0, 0, -1, lam=2.0)
        assert tissue and dfix == 0.0 and wfx == 1
        U, axes = orc.division_draws(5, 2, t, x, y)
        assert k == int(stats.poisson.ppf(U, 2.0)) or abs(stats.poisson.cdf(k, 2.0) - U) < 1e-12
        assert S == pytest.approx(k * 0.1, abs=1e-15)
        add = out - fstar
        counts = np.bincount([(axes >> (2 * d)) & 3 for d in range(k)], minlength=4)
        for a, i in enumerate((1, 2, 5, 6)):           # E-W, N-S, NE-SW, NW-SE
            assert add[i] == pytest.approx(counts[a] * 0.05, abs=1e-9)
            assert add[opp[i]] == pytest.approx(counts[a] * 0.05, abs=1e-9)
        assert add[0] == pytest.approx(0.0, abs=1e-9)
        assert add.sum() == pytest.approx(k * 0.1, abs=1e-9)
        jx, jy = d2q9.momentum(add[:, None, None])
        assert abs(jx.item()) < 1e-9 and abs(jy.item()) < 1e-9
        seen += k
    assert seen > 200


def test_density_law_stops_at_the_threshold():
    """Eq. 5 gives no division at rho = rho_c exactly (a tissue site, since
    tissue is rho >= rho_c) and none at or above rho0; just above rho_c it
    does divide."""
    cfg = si.cfg(L=8, H=8, growth="division_density", growth_rate=1e-2, rho_cell=0.1,
                 rho_c=0.5, rho0=1.5, sigma=0.0, seed=1)
    p = orc.make_params(cfg)
    at_c = np.zeros(9)
    at_c[0] = 0.5                                       # rho* = rho_c exactly, at rest
    above = at_c.copy()
    above[0] = 0.5 + 2.0 ** -20
    at_0 = np.zeros(9)
    at_0[0] = 1.5
    tot_above = 0
    for t in range(200):
        _, tissue, S, _, k, w = orc.update_site_ex(p, at_c, t, 3, 4, 0, 0, -1, lam=5.0)
        assert tissue and k == 0 and S == 0.0 and w == 0
        _, tissue, _, _, k, w = orc.update_site_ex(p, at_0, t, 3, 4, 0, 0, -1, lam=5.0)
        assert tissue and k == 0 and w == 0
        _, tissue, _, _, k, w = orc.update_site_ex(p, above, t, 3, 4, 0, 0, -1, lam=5.0)
        assert tissue and w == int((1.0 - (0.5 + 2.0 ** -20) / 1.5) * 2 ** 24)
        tot_above += k
    assert tot_above > 0


def test_uniform_division_rate_matches_n_s():
    """All-tissue periodic lattice: per step the paper adds n_s = g m_tot /
    rho_cell cells; the total over many steps matches the sum of n_s within
    Poisson fluctuations, and the mass balance closes on the cell mass."""
    L, H = 32, 32
    cfg = si.cfg(L=L, H=H, init_rows=H, ybc="periodic", growth="division", growth_rate=1e-2,
                 rho_cell=0.1, sigma=0.0, seed=7)
    o = orc.Oracle(cfg)
    d0 = o.diagnostics()
    expect, got = 0.0, 0
    m_prev = d0["mass"]
    for _ in range(60):
        lam = o.diagnostics()["lam"]
        # all L*H sites eligible: lam = n_s / (L H)
        assert lam * L * H == pytest.approx(0.01 * m_prev / 0.1, rel=1e-6)
        n0 = o.diagnostics()["divisions"]
        o.step(1)
        d = o.diagnostics()
        got += d["divisions"] - n0
        expect += 0.01 * m_prev / 0.1
        m_prev = d["mass"]
    assert abs(got - expect) <= 5 * math.sqrt(expect), (got, expect)
    d = o.diagnostics()
    assert d["src_total"] == pytest.approx(d["divisions"] * 0.1, rel=1e-12)
    assert d["mass"] - d0["mass"] == pytest.approx(d["src_total"] + d["fix_total"], rel=1e-9)
    o.close()


def _banded_state(rhos, L=8):
    H = len(rhos)
    rho = np.repeat(np.asarray(rhos, float)[:, None], L, axis=1)
    return d2q9.equilibrium(rho, np.zeros_like(rho), np.zeros_like(rho)), rho


def test_density_law_acceptance_follows_eq5():
    """Rows of fixed density: lam spreads n_s over sum(1 - rho/rho0) of the
    eligible sites (rho_c < rho < rho0), and each site divides at the rate
    lam (1 - rho/rho0); none below rho_c or above rho0."""
    rhos = [0.4, 0.8, 1.1, 1.4, 1.6, 0.45, 1.0, 1.2]
    f, rho = _banded_state(rhos)
    L, H = rho.shape[1], rho.shape[0]
    cfg = si.cfg(L=L, H=H, init_rows=0, ybc="periodic", growth="division_density",
                 growth_rate=5e-2, rho_cell=0.1, rho0=1.5, rho_c=0.5, sigma=0.0, seed=9)
    o = orc.Oracle(cfg)
    o.set_populations(f)
    q = np.where((rho > 0.5) & (rho < 1.5), 1.0 - rho / 1.5, 0.0)
    lam = o.diagnostics()["lam"]
    m_tot = float(rho.sum())
    assert lam == pytest.approx(0.05 * m_tot / 0.1 / q.sum(), rel=1e-6)
    p = orc.make_params(cfg)
    counts = np.zeros((H, L))
    T = 400
    for t in range(T):
        for j in range(H):
            for x in range(L):
                # the site's own band populations as its streamed input
                fs = f[:, j, x]
                _, _, _, _, k, wfx = orc.update_site_ex(p, fs, t, x, j, 0, 0, -1, lam=lam)
                counts[j, x] += k
                assert (wfx > 0) == (q[j, x] > 0)
    mean = counts.mean(axis=1) / T
    want = lam * q[:, 0]
    for j in range(H):
        if q[j, 0] == 0.0:
            assert mean[j] == 0.0
        else:
            se = math.sqrt(want[j] / (T * L))
            assert abs(mean[j] - want[j]) <= 5 * se, (rhos[j], mean[j], want[j])
    o.close()


@pytest.mark.parametrize("law", ["division", "division_density"])
def test_poisson_counts_match_literal_selection_with_replacement(law):
    """The paper's procedure, replayed literally on a small lattice: draw
    sites uniformly with replacement (accepting each with probability q under
    Eq. 5) until n_s cells have divided.  Its mean count per site equals the
    oracle's per-site Poisson mean lam q."""
    rhos = [0.7, 0.9, 1.2, 1.45, 0.3, 1.0]
    f, rho = _banded_state(rhos, L=4)
    H, L = rho.shape
    g, rc = 0.2, 0.1
    cfg = si.cfg(L=L, H=H, init_rows=0, ybc="periodic", growth=law, growth_rate=g,
                 rho_cell=rc, rho0=1.5, sigma=0.0, seed=4)
    o = orc.Oracle(cfg)
    o.set_populations(f)
    lam = o.diagnostics()["lam"]
    o.close()
    tissue = rho >= 0.5
    if law == "division":
        q = np.where(tissue, 1.0, 0.0)
    else:
        q = np.where((rho > 0.5) & (rho < 1.5), 1.0 - rho / 1.5, 0.0)
    n_s = g * rho.sum() / rc                            # cells per step, Sec. II
    sites = np.argwhere(tissue)
    rng = np.random.default_rng(11)
    trials = 4000
    counts = np.zeros_like(rho)
    n_int = int(round(n_s))
    for _ in range(trials):
        made = 0
        while made < n_int:
            j, x = sites[rng.integers(0, len(sites))]
            if rng.random() < q[j, x]:
                counts[j, x] += 1
                made += 1
    literal = counts / trials * (n_s / n_int)           # per unit of the exact n_s
    for j in range(H):
        for x in range(L):
            want = lam * q[j, x]
            se = math.sqrt(max(want, 1e-12) / trials)
            assert abs(literal[j, x] - want) <= 5 * se + 1e-12, (j, x, literal[j, x], want)


def test_division_map_counts_every_division_where_it_happened():
    """The per-site map adds up to the division count, holds nothing outside
    the tissue, and clears."""
    cfg = si.cfg(L=24, H=32, init_rows=12, growth="division", growth_rate=2e-2, sigma=1e-2,
                 region="front_band", region_width=3, seed=9)
    o = orc.Oracle(cfg)
    o.step(20)
    m = o.division_map()
    d = o.diagnostics()
    assert m.sum() == d["divisions"] > 0
    h = o.front_heights()
    rows = np.arange(cfg["H"])[:, None]
    assert np.all(m[rows >= h[None, :]] == 0)                       # above the front
    assert np.all(m[rows < h[None, :] - 3 - 1] == 0)                # below the band
    o.division_map(clear=True)
    assert o.division_map().sum() == 0
    o.step(1)
    assert o.division_map().sum() == o.diagnostics()["divisions"] - d["divisions"]
    o.close()
