"""Pins of the oracle's D2Q7 lattice (the paper's own, Sec. II) against its
geometry and the mathematics of the lattice, not against the oracle's own
formulas: equilibrium moments (Eq. 3 with c_s^2 = 1/4), streaming checked
site by site against positions and direction vectors, the rear-wall
bounce-back, conservation laws, the shear-wave decay rate (tau - 1/2)/4 k^2,
Eq. 4's noise statistics over seven directions, a flat front's first step in
closed form, mirror symmetry, the step-7 fix, and the division injection on
the three axes."""
import numpy as np
import pytest

import synth_inputs as si
from oracle import oracle as orc
from tests import d2q7


def cfg7(**kw):
    return si.cfg(lattice="d2q7", **kw)


# ---------------------------------------------------------------- lattice
def test_lattice_moments_of_the_paper():
    # w_0 = 1/2, w_i = 1/12 (Sec. II): isotropic to fourth order with c_s^2 = 1/4
    W, EX, EY = d2q7.W, d2q7.EX, d2q7.EY
    assert np.isclose(W.sum(), 1.0)
    assert np.isclose((W * EX).sum(), 0) and np.isclose((W * EY).sum(), 0)
    assert np.isclose((W * EX * EX).sum(), 0.25) and np.isclose((W * EY * EY).sum(), 0.25)
    assert np.isclose((W * EX * EY).sum(), 0.0)
    assert np.isclose((W * EX ** 4).sum(), 3 / 16) and np.isclose((W * EX ** 2 * EY ** 2).sum(), 1 / 16)
    assert list(d2q7.OPP) == [0, 4, 5, 6, 1, 2, 3]


@pytest.mark.parametrize("rho,ux,uy", [(1.0, 0.0, 0.0), (0.7, 0.05, -0.02), (1.3, -0.08, 0.11)])
def test_equilibrium_moments_closed_form(rho, ux, uy):
    f = orc.fss7(rho, ux, uy)
    EX, EY = d2q7.EX, d2q7.EY
    assert np.isclose(f.sum(), rho, rtol=1e-14)
    assert np.isclose((f * EX).sum(), rho * ux, rtol=1e-13, atol=1e-16)
    assert np.isclose((f * EY).sum(), rho * uy, rtol=1e-13, atol=1e-16)
    # second moment: rho (c_s^2 delta + u u)
    assert np.isclose((f * EX * EX).sum(), rho * (0.25 + ux * ux), rtol=1e-13)
    assert np.isclose((f * EY * EY).sum(), rho * (0.25 + uy * uy), rtol=1e-13)
    assert np.isclose((f * EX * EY).sum(), rho * ux * uy, rtol=1e-12, atol=1e-15)
    # and the whole distribution against the geometric form of Eq. 3
    g = d2q7.equilibrium(np.array([[rho]]), np.array([[ux]]), np.array([[uy]]))[:, 0, 0]
    assert np.allclose(f, g, rtol=1e-14, atol=1e-17)


# ---------------------------------------------------------------- streaming
@pytest.mark.parametrize("y_wall", [0, 1])
def test_pull_matches_geometry(y_wall):
    """Each pulled population comes from the site at position(x, y) - e_i
    (periodic in x), for both parities of the absolute row; below the rear
    wall it is the site's own reverse population; above the top it is 0."""
    L, H = 5, 6
    rng = np.random.default_rng(7)
    f = rng.uniform(0.1, 1.0, (7, H, L))
    c = cfg7(L=L, H=H, init_rows=H)
    p = orc.make_params(c)
    for j in range(H):
        y_abs = y_wall + j
        for x in range(L):
            fs = orc.pull_site(p, f, x, j, y_abs)
            px, py = d2q7.position(x, y_abs)
            for i in range(7):
                src = d2q7.site_at(px - d2q7.EX[i], py - d2q7.EY[i], L)
                assert src is not None
                xs, ys = src
                js = ys - y_wall
                if js < 0:
                    want = f[d2q7.OPP[i], j, x]
                elif js >= H:
                    want = 0.0
                else:
                    want = f[i, js, xs]
                assert fs[i] == want, (x, j, y_abs, i)


def test_pull_periodic_rows():
    L, H = 4, 6
    rng = np.random.default_rng(8)
    f = rng.uniform(0.1, 1.0, (7, H, L))
    p = orc.make_params(cfg7(L=L, H=H, init_rows=H, ybc="periodic"))
    for j in range(H):
        for x in range(L):
            fs = orc.pull_site(p, f, x, j)
            px, py = d2q7.position(x, j)
            for i in range(7):
                xs, ys = d2q7.site_at(px - d2q7.EX[i], py - d2q7.EY[i], L)
                assert fs[i] == f[i, ys % H, xs]


def test_periodic_odd_height_is_rejected():
    with pytest.raises(ValueError):
        orc.Oracle(cfg7(L=8, H=7, init_rows=7, ybc="periodic"))


# ---------------------------------------------------------------- conservation
def _rand_state(rng, L, H, lo=0.8, hi=1.2, u=0.08):
    rho = rng.uniform(lo, hi, (H, L))
    return d2q7.equilibrium(rho, rng.uniform(-u, u, (H, L)), rng.uniform(-u, u, (H, L)))


def test_mass_and_momentum_conserved():
    L, H = 12, 10
    rng = np.random.default_rng(2)
    f = _rand_state(rng, L, H)
    c = cfg7(L=L, H=H, init_rows=H, ybc="periodic", mu=0.0, growth_rate=0.0, sigma=0.0, tau=0.8)
    o = orc.Oracle(c)
    o.set_populations(f)
    j0 = np.array([v.sum() for v in d2q7.momentum(f)])
    m0 = f.sum()
    scale = np.abs(np.stack(d2q7.momentum(f))).sum()
    for _ in range(40):
        o.step(1)
        g = o.populations()
        j = np.array([v.sum() for v in d2q7.momentum(g)])
        assert abs(g.sum() - m0) <= 1e-13 * m0
        assert np.all(np.abs(j - j0) <= 1e-13 * scale)


@pytest.mark.parametrize("tau", [1.0, 0.7])
def test_friction_decay_closed_form(tau):
    L, H, mu = 6, 4, 0.01
    f = d2q7.equilibrium(np.ones((H, L)), 0.04 * np.ones((H, L)), -0.03 * np.ones((H, L)))
    o = orc.Oracle(cfg7(L=L, H=H, init_rows=H, ybc="periodic", mu=mu, growth_rate=0.0,
                        sigma=0.0, tau=tau))
    o.set_populations(f)
    P0 = np.array([v.sum() for v in d2q7.momentum(f)])
    for t in range(1, 61):
        o.step(1)
        P = np.array([v.sum() for v in d2q7.momentum(o.populations())])
        assert np.allclose(P, P0 * (1.0 - mu / tau) ** t, rtol=1e-12, atol=0), t


def _shear_rate(L, tau, U=1e-3):
    # u_y(x) = U sin(k x) along the rows: positions x + (y mod 2)/2
    H = 2
    k = 2 * np.pi / L
    px = np.array([[d2q7.position(x, y)[0] for x in range(L)] for y in range(H)])
    f = d2q7.equilibrium(np.ones((H, L)), np.zeros((H, L)), U * np.sin(k * px))
    o = orc.Oracle(cfg7(L=L, H=H, init_rows=H, ybc="periodic", mu=0.0, growth_rate=0.0,
                        sigma=0.0, tau=tau))
    o.set_populations(f)
    nu = (tau - 0.5) * d2q7.CS2
    T = 1.0 / (nu * k * k)
    t0, t1 = int(0.1 * T), int(0.6 * T)

    def amp():
        _, jy = d2q7.momentum(o.populations())
        return float((jy * np.sin(k * px)).sum() / (np.sin(k * px) ** 2).sum())

    o.step(t0)
    a0 = amp()
    o.step(t1 - t0)
    a1 = amp()
    return -np.log(a1 / a0) / (t1 - t0), nu * k * k


@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_shear_wave_decay_converges_second_order(tau):
    errs = []
    for L in (16, 32, 64):
        rate, expect = _shear_rate(L, tau)
        errs.append(abs(rate - expect) / expect)
    assert errs[-1] < 3e-3, errs
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


# ---------------------------------------------------------------- noise
def test_noise_statistics_eq4_seven_directions():
    L, H, sigma = 256, 256, 0.01
    o = orc.Oracle(cfg7(L=L, H=H, init_rows=H, ybc="periodic", mu=0.0, growth_rate=0.0,
                        sigma=sigma, tau=1.0, init_amp=0.0))
    f0 = o.populations()
    o.step(1)
    eta = (o.populations() - f0).reshape(7, -1)
    n = eta.shape[1]
    assert np.max(np.abs(eta.sum(0))) < 1e-15 * 7
    cov = np.cov(eta)
    # eta_i = eta~_i - mean of 7: variance (6/7) sigma^2/3, covariance -sigma^2/21
    for i in range(7):
        assert abs(cov[i, i] / (2 * sigma ** 2 / 7) - 1) < 5 * np.sqrt(2.0 / n)
        for j in range(i + 1, 7):
            assert abs(cov[i, j] / (-sigma ** 2 / 21) - 1) < 0.06


# ---------------------------------------------------------------- front rule
@pytest.mark.parametrize("rho_c,advances", [(0.5, False), (1.0 / 6.0 - 1e-9, True)])
def test_flat_front_first_step_closed_form(rho_c, advances):
    # the first empty row pulls NE and NW from the row below: 2/12 = 1/6 of
    # rho = 1, tissue only if rho_c <= 1/6
    L, H = 8, 12
    o = orc.Oracle(cfg7(L=L, H=H, init_rows=5, init_amp=0.0, growth_rate=0.0, sigma=0.0,
                        tau=1.0, rho_c=rho_c))
    assert np.all(o.front_heights() == 5)
    o.step(1)
    assert np.all(o.front_heights() == (6 if advances else 5))
    f = o.populations()
    row = f[:, 5, :]
    if not advances:
        want = np.zeros(7)
        want[5] = want[6] = 1.0 / 12.0      # reversed: SW and SE
        assert np.all(row == want[:, None])
    assert np.all(f[:, 6:, :] == 0.0)


def test_void_update_reverses_pairs():
    rng = np.random.default_rng(4)
    c = cfg7(L=4, H=4)
    for _ in range(20):
        fs = rng.uniform(0, 0.05, 7)
        a, tissue, S, dfix = orc.update_site(c, fs, 0, 0, 0, 0, force=0)
        assert not tissue
        assert np.array_equal(a, fs[d2q7.OPP])


# ---------------------------------------------------------------- symmetry
def test_mirror_equivariance():
    # x -> -x maps site (x, y) to column (-x - (y mod 2)) mod L and swaps
    # E <-> W, NE <-> NW, SW <-> SE
    L, H = 10, 12
    rng = np.random.default_rng(5)
    f = _rand_state(rng, L, H, u=0.05)
    perm = [0, 4, 3, 2, 1, 6, 5]
    g = np.zeros_like(f)
    for y in range(H):
        for x in range(L):
            g[:, y, (-x - (y % 2)) % L] = f[perm, y, x]
    c = cfg7(L=L, H=H, init_rows=H, ybc="periodic", mu=1e-3, growth_rate=1e-3, sigma=0.0, tau=0.9)
    a, b = orc.Oracle(c), orc.Oracle(c)
    a.set_populations(f)
    b.set_populations(g)
    a.step(5)
    b.step(5)
    fa, fb = a.populations(), b.populations()
    ga = np.zeros_like(fa)
    for y in range(H):
        for x in range(L):
            ga[:, y, (-x - (y % 2)) % L] = fa[perm, y, x]
    assert np.allclose(ga, fb, rtol=1e-12, atol=1e-15)


def test_translation_by_two_rows_and_one_column():
    L, H = 8, 10
    rng = np.random.default_rng(6)
    f = _rand_state(rng, L, H)
    c = cfg7(L=L, H=H, init_rows=H, ybc="periodic", mu=1e-3, growth_rate=0.0, sigma=0.0, tau=0.9)
    a, b = orc.Oracle(c), orc.Oracle(c)
    a.set_populations(f)
    b.set_populations(np.roll(np.roll(f, 2, axis=1), 1, axis=2))
    a.step(4)
    b.step(4)
    assert np.array_equal(np.roll(np.roll(a.populations(), 2, axis=1), 1, axis=2), b.populations())


# ---------------------------------------------------------------- growth, fix
def test_bulk_growth_adds_g_rho_without_momentum():
    rng = np.random.default_rng(9)
    c = cfg7(L=4, H=4, growth_rate=1e-2, tau=1e12, mu=0.0, sigma=0.0)
    for _ in range(20):
        fs = d2q7.equilibrium(np.array([[1.0]]), np.array([[0.02]]), np.array([[-0.01]]))[:, 0, 0]
        fs = fs * rng.uniform(0.9, 1.1, 7)
        out, tissue, S, _ = orc.update_site(c, fs, 0, 0, 0, 0)
        assert tissue and S == pytest.approx(1e-2 * fs.sum(), rel=1e-14)
        add = out - fs
        assert add[0] == pytest.approx(0.0, abs=1e-12)
        assert np.allclose(add[1:], S / 6, rtol=1e-6)
        assert abs((add * d2q7.EX).sum()) < 1e-12 and abs((add * d2q7.EY).sum()) < 1e-12


def test_division_injects_cell_mass_on_three_axes():
    c = cfg7(L=8, H=8, growth="division", growth_rate=1e-2, rho_cell=0.1, tau=1e12, mu=0.0,
             sigma=0.0, seed=5, replica=2)
    p = orc.make_params(c)
    rng = np.random.default_rng(2)
    seen = 0
    for _ in range(200):
        fs = d2q7.W * rng.uniform(0.8, 1.2) + rng.uniform(0.0, 0.01, 7)
        t, x, y = int(rng.integers(0, 1000)), int(rng.integers(0, 8)), int(rng.integers(0, 8))
        out, tissue, S, dfix, k, wfx = orc.update_site_ex(p, fs, t, x, y, 0, 0, -1, lam=2.0)
        assert tissue and wfx == 1
        _, axes = orc.division_draws(5, 2, t, x, y)
        digits = []
        n = axes
        for _ in range(k):
            digits.append(n % 3)
            n //= 3
        counts = np.bincount(digits, minlength=3)
        add = out - fs
        for a in range(3):                      # axes E-W, NE-SW, NW-SE
            assert add[a + 1] == pytest.approx(counts[a] * 0.05, abs=1e-9)
            assert add[a + 4] == pytest.approx(counts[a] * 0.05, abs=1e-9)
        assert S == pytest.approx(k * 0.1, abs=1e-15)
        assert abs((add * d2q7.EX).sum()) < 1e-9 and abs((add * d2q7.EY).sum()) < 1e-9
        seen += k
    assert seen > 200
    # each axis is drawn with probability 1/3
    tallies = np.zeros(3)
    for s in range(3000):
        _, axes = orc.division_draws(1, 0, s, 3, 4)
        tallies[axes % 3] += 1
    assert np.all(np.abs(tallies / 3000 - 1 / 3) < 0.04)


def test_negative_fix_closed_form():
    # rest negative: zero it and rescale to keep the density; moving negative:
    # its magnitude goes to the reverse direction
    c = cfg7(L=4, H=4, growth_rate=0.0, tau=1e12, mu=0.0, sigma=0.0)
    fs = np.array([-0.02, 0.2, 0.1, 0.15, 0.05, 0.12, 0.08])
    out, tissue, S, dfix = orc.update_site(c, fs, 0, 0, 0, 0)
    rho_pre = fs.sum()
    g = fs.copy()
    g[0] = 0.0
    g = g * (rho_pre / g.sum())
    assert np.allclose(out, g, rtol=1e-9)
    fs2 = np.array([0.3, 0.2, -0.01, 0.15, 0.05, 0.12, 0.08])
    out2, _, _, dfix2 = orc.update_site(c, fs2, 0, 0, 0, 0)
    want = fs2.copy()
    want[5] += 0.01
    want[2] = 0.0
    assert np.allclose(out2, want, rtol=1e-9, atol=1e-12)
    assert dfix2 == pytest.approx(0.02, rel=1e-6)


def test_initial_state_weights():
    o = orc.Oracle(cfg7(L=6, H=8, init_rows=3, init_amp=0.1, seed=4))
    f = o.populations()
    rho = f.sum(0)
    assert np.all(rho[3:] == 0) and np.all((rho[:3] >= 0.9) & (rho[:3] <= 1.1))
    assert np.allclose(f[:, :3], d2q7.W[:, None, None] * rho[None, :3], rtol=1e-15)
    assert np.all(o.front_heights() == 3)
