"""Pins of the FP64 oracle against facts fixed by the paper and by the
mathematics of the D2Q9 lattice -- not against the oracle itself.

Each test names the property it pins and where it comes from:
  * equilibrium moments (Eq. 3 with the D2Q9 lattice identities),
  * mass balance (Eq. 2 conserves mass; Eq. 4's noise is zero-sum; growth adds
    exactly the injected mass),
  * momentum conservation without friction or growth, and the closed-form
    friction decay of u* = (1 - mu) u,
  * the textbook shear-wave decay rate nu k^2, nu = c_s^2 (tau - 1/2),
  * the noise statistics implied by Eq. 4,
  * the empty void beyond the front (Sec. II, two-step bounce-back),
  * a closed-form first step of a flat front, and streaming by array shifts,
  * translation and mirror symmetry.
"""
import numpy as np
import pytest

import synth_inputs as si
from oracle import oracle as orc
from tests import d2q9


def _ones_state(L, H, rho, ux, uy):
    f = d2q9.equilibrium(rho * np.ones((H, L)), ux * np.ones((H, L)), uy * np.ones((H, L)))
    return f


# ---------------------------------------------------------------- lattice
def test_lattice_tables_match_d2q9():
    cx, cy, opp, w = orc.lattice()
    assert np.array_equal(cx, d2q9.C[:, 0]) and np.array_equal(cy, d2q9.C[:, 1])
    assert np.array_equal(opp, d2q9.OPP)
    assert np.allclose(w, d2q9.W, rtol=0, atol=1e-17)
    # reverse directions really are reversed, and the weights are isotropic
    assert np.array_equal(d2q9.C[opp], -d2q9.C)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose((w[:, None, None] * d2q9.C[:, :, None] * d2q9.C[:, None, :]).sum(0),
                       np.eye(2) / 3.0, atol=1e-16)


# ---------------------------------------------------------------- P1 Eq. 3 moments
def test_equilibrium_moments_closed_form():
    rng = np.random.default_rng(1)
    for _ in range(500):
        rho = rng.uniform(0.05, 3.0)
        ux, uy = rng.uniform(-0.3, 0.3, 2)
        f = orc.fss(rho, ux, uy)
        m0 = f.sum()
        jx, jy = d2q9.momentum(f)
        pxx, pxy, pyy = d2q9.second_moment(f)
        tol = 1e-14 * rho
        assert abs(m0 - rho) <= tol
        assert abs(jx - rho * ux) <= tol and abs(jy - rho * uy) <= tol
        assert abs(pxx - (rho / 3 + rho * ux * ux)) <= tol
        assert abs(pyy - (rho / 3 + rho * uy * uy)) <= tol
        assert abs(pxy - rho * ux * uy) <= tol
        # and it is the textbook D2Q9 equilibrium
        assert np.allclose(f, d2q9.equilibrium(rho, ux, uy), rtol=1e-14, atol=1e-16)


# ---------------------------------------------------------------- P2 mass balance
@pytest.mark.parametrize("extra", [
    dict(),                                                       # the 64x64 FP64 workload
    dict(sigma=1e-2, tau=0.8, growth_rate=5e-3, region="front_band", region_width=3),
    dict(sigma=1e-2, H=128, init_rows=80, ybc="follow", wall_min_gap=20, wall_w_factor=10.0),
])
def test_mass_balance_every_step(extra):
    c = dict(si.SMALL_FP64)
    c.update(extra)
    o = orc.Oracle(c)
    d0 = o.diagnostics()
    m0 = d0["mass"]
    prev = d0
    for t in range(300):
        assert o.step(1) == 0
        d = o.diagnostics()
        dm = d["mass"] - prev["mass"]
        booked = ((d["src_total"] - prev["src_total"]) + (d["fix_total"] - prev["fix_total"])
                  - (d["retired"] - prev["retired"]))
        assert abs(dm - booked) <= 1e-13 * d["mass"], (t, dm, booked)
        prev = d
    assert d["src_total"] > 0
    total = d["mass"] - m0
    assert abs(total - (d["src_total"] + d["fix_total"] - d["retired"])) <= 1e-12 * d["mass"]
    if c["ybc"] == "follow":
        assert d["y_wall"] > 0 and d["retired"] > 0


def test_bulk_growth_rate_is_g_times_tissue_mass():
    # with the whole window tissue and periodic rows, every site injects
    # g rho*, so the total mass grows exactly by a factor (1 + g) per step
    c = si.cfg(L=16, H=16, init_rows=16, ybc="periodic", growth_rate=1e-2, sigma=0.0)
    o = orc.Oracle(c)
    m = [o.diagnostics()["mass"]]
    for _ in range(20):
        o.step(1)
        m.append(o.diagnostics()["mass"])
    m = np.array(m)
    assert np.allclose(m[1:] / m[:-1], 1.01, rtol=1e-13, atol=0)


# ---------------------------------------------------------------- P3 momentum
def test_momentum_conserved_without_friction_growth_noise():
    L, H = 24, 20
    rng = np.random.default_rng(2)
    rho = rng.uniform(0.8, 1.2, (H, L))
    ux = rng.uniform(-0.1, 0.1, (H, L))
    uy = rng.uniform(-0.1, 0.1, (H, L))
    f = d2q9.equilibrium(rho, ux, uy)
    c = si.cfg(L=L, H=H, init_rows=H, ybc="periodic", mu=0.0, growth_rate=0.0,
               sigma=0.0, tau=0.8)
    o = orc.Oracle(c)
    o.set_populations(f)
    j0 = np.array([v.sum() for v in d2q9.momentum(f)])
    scale = np.abs(np.stack(d2q9.momentum(f))).sum()
    m0 = f.sum()
    for _ in range(50):
        o.step(1)
        g = o.populations()
        j = np.array([v.sum() for v in d2q9.momentum(g)])
        assert np.all(np.abs(j - j0) <= 1e-13 * scale)
        assert abs(g.sum() - m0) <= 1e-13 * m0


# ---------------------------------------------------------------- P4 friction
@pytest.mark.parametrize("tau", [1.0, 0.8, 1.7])
def test_friction_decay_closed_form(tau):
    # uniform flow: streaming changes nothing, and relaxing towards
    # f^SS(rho, (1 - mu) u) removes a fraction mu / tau of the momentum
    L, H, mu = 8, 6, 0.01
    f = _ones_state(L, H, 1.0, 0.05, -0.03)
    c = si.cfg(L=L, H=H, init_rows=H, ybc="periodic", mu=mu, growth_rate=0.0,
               sigma=0.0, tau=tau)
    o = orc.Oracle(c)
    o.set_populations(f)
    P0 = np.array([v.sum() for v in d2q9.momentum(f)])
    for t in range(1, 101):
        o.step(1)
        P = np.array([v.sum() for v in d2q9.momentum(o.populations())])
        expect = P0 * (1.0 - mu / tau) ** t
        assert np.allclose(P, expect, rtol=1e-12, atol=0), t


# ---------------------------------------------------------------- P5 shear wave
def _shear_rate(L, tau, mu=0.0, U=1e-3, t0=None, t1=None):
    H = 2
    k = 2 * np.pi / L
    x = np.arange(L)
    uy = U * np.sin(k * x)[None, :] * np.ones((H, 1))
    f = d2q9.equilibrium(np.ones((H, L)), np.zeros((H, L)), uy)
    c = si.cfg(L=L, H=H, init_rows=H, ybc="periodic", mu=mu, growth_rate=0.0,
               sigma=0.0, tau=tau)
    o = orc.Oracle(c)
    o.set_populations(f)
    nu = (tau - 0.5) / 3.0
    T = 1.0 / (nu * k * k)
    t0 = int(0.1 * T) if t0 is None else t0
    t1 = int(0.6 * T) if t1 is None else t1

    def amp():
        _, jy = d2q9.momentum(o.populations())
        return float((jy.mean(0) * np.sin(k * x)).sum() / (np.sin(k * x) ** 2).sum())

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
    assert errs[-1] < 2e-3, errs
    # relative error falls like k^2: about a factor 4 per doubling of L
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


def test_shear_wave_with_friction():
    # friction adds -ln(1 - mu/tau) per step on top of viscous decay
    L, tau, mu = 64, 1.0, 2e-3
    rate, visc = _shear_rate(L, tau, mu=mu)
    expect = visc - np.log(1 - mu / tau)
    assert abs(rate - expect) / expect < 5e-3


# ---------------------------------------------------------------- P6 noise statistics
def test_noise_statistics_eq4():
    L, H, sigma = 512, 512, 0.01
    c = si.cfg(L=L, H=H, init_rows=H, ybc="periodic", mu=0.0, growth_rate=0.0,
               sigma=sigma, tau=1.0, init_amp=0.0)
    o = orc.Oracle(c)
    f0 = o.populations()
    o.step(1)
    eta = (o.populations() - f0).reshape(9, -1)      # at rest: f = f^SS + eta
    n = eta.shape[1]
    # zero sum at every site (to rounding)
    assert np.max(np.abs(eta.sum(0))) < 1e-15 * 9
    var_t = sigma ** 2 / 3.0
    cov = np.cov(eta)
    for i in range(9):
        se_mean = np.sqrt(8 / 9 * var_t / n)
        assert abs(eta[i].mean()) < 5 * se_mean
        # variance 8 sigma^2 / 27; sampling error of a variance ~ sqrt(2/n)
        # (uniform has smaller kurtosis, this bound is conservative)
        assert abs(cov[i, i] / (8 * sigma ** 2 / 27) - 1) < 5 * np.sqrt(2.0 / n)
        for j in range(i + 1, 9):
            assert abs(cov[i, j] / (-sigma ** 2 / 27) - 1) < 0.05
    # each eta~_i is uniform on [-sigma, sigma]: recover it and check the range
    assert np.max(np.abs(eta)) < 2 * sigma


def test_noise_uniforms_chi_square():
    rng = np.random.default_rng(3)
    n = 20000
    u = np.stack([orc.noise_uniforms(0, 0, int(t), int(x), int(y))
                  for t, x, y in rng.integers(0, 10 ** 6, (n, 3))])
    assert np.all((u > 0) & (u < 1))
    bins = 20
    for i in range(9):
        hist, _ = np.histogram(u[:, i], bins=bins, range=(0, 1))
        chi2 = ((hist - n / bins) ** 2 / (n / bins)).sum()
        assert chi2 < 50.0, (i, chi2)      # 19 dof: p ~ 1e-4 at 43.8
    cc = np.corrcoef(u.T)
    assert np.max(np.abs(cc - np.eye(9))) < 0.04


# ---------------------------------------------------------------- P7 empty void
def test_void_beyond_front_stays_exactly_empty():
    c = dict(si.SMALL_FP64, sigma=1e-2, tau=0.8)
    o = orc.Oracle(c)
    for t in range(400):
        o.step(1)
        d = o.diagnostics()
        f = o.populations()
        hi = int(d["h_hi"])
        assert hi < c["H"]
        assert np.all(f[:, hi + 1:, :] == 0.0), t
        # the front layer itself holds mass below threshold only
        h = o.front_heights()
        for x in range(0, c["L"], 7):
            if h[x] < c["H"]:
                assert f[:, h[x], x].sum() < c["rho_c"] + 1e-12


def test_void_update_is_an_involution():
    rng = np.random.default_rng(4)
    c = si.SMALL_FP64
    for _ in range(50):
        fs = rng.uniform(0, 0.05, 9)
        a, tissue, S, dfix = orc.update_site(c, fs, 0, 0, 0, 0, force=0)
        b, _, _, _ = orc.update_site(c, a, 0, 0, 0, 0, force=0)
        assert not tissue and S == 0 and dfix == 0
        assert np.array_equal(b, fs)
        assert np.array_equal(a, fs[d2q9.OPP])


# ---------------------------------------------------------------- P8 front rule
@pytest.mark.parametrize("rho_c,expect_h", [(0.5, 16), (0.1, 17)])
def test_flat_front_first_step_closed_form(rho_c, expect_h):
    # flat front of uniform rho = 1 at rest, no growth or noise, tau = 1: the
    # first empty row receives the N, NE and NW populations of the row below,
    # 1/9 + 1/36 + 1/36 = 1/6, and is tissue only if rho_c <= 1/6
    c = si.cfg(L=32, H=32, init_rows=16, init_amp=0.0, growth_rate=0.0, sigma=0.0,
               tau=1.0, rho_c=rho_c)
    o = orc.Oracle(c)
    assert np.all(o.front_heights() == 16)
    o.step(1)
    f = o.populations()
    assert np.all(o.front_heights() == expect_h)
    row = f[:, 16, :]
    if expect_h == 16:
        # reversed: the mass now points back down
        want = np.zeros(9)
        want[4] = 1.0 / 9.0
        want[7] = 1.0 / 36.0
        want[8] = 1.0 / 36.0
        assert np.all(row == want[:, None])
    else:
        # tissue now: it relaxes with u_y close to 1, and the negative-value
        # fix of step 7 books the mass it adds; otherwise mass is conserved
        d = o.diagnostics()
        assert d["fix_total"] > 0
        assert np.allclose(row.sum(0), 1.0 / 6.0 + d["fix_total"] / 32, rtol=1e-14)
    assert np.all(f[:, 17:, :] == 0.0)


def _rand_front_state(rng, L, H):
    """Random state with tissue, sub-threshold and empty sites mixed."""
    kind = rng.integers(0, 3, (H, L))
    rho = np.where(kind == 0, rng.uniform(0.6, 1.4, (H, L)),
                   np.where(kind == 1, rng.uniform(0.0, 0.4, (H, L)), 0.0))
    ux = rng.uniform(-0.1, 0.1, (H, L))
    uy = rng.uniform(-0.1, 0.1, (H, L))
    f = d2q9.equilibrium(rho, ux, uy)
    f = np.where(f > 0, f, 0.0) * rng.uniform(0.7, 1.3, f.shape)
    return f


@pytest.mark.parametrize("ybc", ["fixed", "periodic"])
def test_step_equals_shift_streaming_plus_site_update(ybc):
    # brute force on 8x8 lattices: streaming by array shifts, then the
    # per-site update, then h by a direct column scan; compared bitwise with
    # the oracle's own step
    rng = np.random.default_rng(5)
    L = H = 8
    seen_masks = set()
    for trial in range(48):
        c = si.cfg(L=L, H=H, init_rows=0, sigma=1e-2, tau=0.8, growth_rate=1e-2,
                   region="front_band", region_width=2, ybc=ybc, seed=trial)
        o = orc.Oracle(c)
        f = _rand_front_state(rng, L, H)
        h_prev = rng.integers(0, H + 1, L).astype(np.int32)
        o.set_populations(f)
        o.set_front_heights(h_prev)
        fstar = d2q9.stream_pull(f, ybc)
        tissue = fstar.sum(0) >= c["rho_c"]
        for y in range(H):
            for x in range(L):
                m = 0
                for k, (dx, dy) in enumerate([(a, b) for b in (-1, 0, 1) for a in (-1, 0, 1)]):
                    if tissue[(y + dy) % H, (x + dx) % L]:
                        m |= 1 << k
                seen_masks.add(m)
        want = np.zeros_like(f)
        h_want = np.zeros(L, np.int32)
        for y in range(H):
            for x in range(L):
                out, tis, _, _ = orc.update_site(c, fstar[:, y, x], 0, x, y, int(h_prev[x]))
                assert tis == bool(tissue[y, x])
                want[:, y, x] = out
                if tis:
                    h_want[x] = y + 1
        o.step(1)
        assert np.array_equal(o.populations(), want)
        assert np.array_equal(o.front_heights(), h_want)
    assert len(seen_masks) > 400


# ---------------------------------------------------------------- P9 symmetry
def _mirror_x(f):
    # x -> L-1-x swaps E<->W, NE<->NW, SE<->SW
    perm = [0, 3, 2, 1, 4, 6, 5, 8, 7]
    return f[perm][:, :, ::-1]


def test_translation_equivariance_bitwise():
    rng = np.random.default_rng(6)
    L = H = 16
    c = si.cfg(L=L, H=H, init_rows=0, sigma=0.0, tau=0.8, growth_rate=1e-2)
    f = _rand_front_state(rng, L, H)
    f[:, H // 2:, :] = 0.0
    a = orc.Oracle(c)
    b = orc.Oracle(c)
    a.set_populations(f)
    b.set_populations(np.roll(f, 5, axis=2))
    a.set_front_heights(np.full(L, H // 2, np.int32))
    b.set_front_heights(np.full(L, H // 2, np.int32))
    a.step(20)
    b.step(20)
    assert np.array_equal(np.roll(a.populations(), 5, axis=2), b.populations())
    assert np.array_equal(np.roll(a.front_heights(), 5), b.front_heights())


def test_mirror_equivariance():
    rng = np.random.default_rng(7)
    L = H = 16
    c = si.cfg(L=L, H=H, init_rows=0, sigma=0.0, tau=1.0, growth_rate=1e-2)
    f = _rand_front_state(rng, L, H)
    f[:, H // 2:, :] = 0.0
    a = orc.Oracle(c)
    b = orc.Oracle(c)
    a.set_populations(f)
    b.set_populations(_mirror_x(f))
    a.step(10)
    b.step(10)
    assert np.allclose(_mirror_x(a.populations()), b.populations(), rtol=0, atol=1e-14)


# ---------------------------------------------------------------- init
def test_initial_state_appendix_a():
    c = dict(si.SMALL_FP64)
    o = orc.Oracle(c)
    f = o.populations()
    rho = f.sum(0)
    assert np.all(f[:, 16:, :] == 0)
    r = rho[:16]
    assert np.all(np.abs(r - 1.0) <= 1e-3 + 1e-15)
    assert r.std() > 1e-4
    # at rest: populations are w_i rho
    assert np.allclose(f[:, :16, :], d2q9.W[:, None, None] * r[None], rtol=1e-15, atol=0)
    assert np.all(o.front_heights() == 16)
    # uniform draw: mean 1/2, variance 1/12 over many sites
    u = np.array([orc.init_uniform(0, 0, x, y) for x in range(64) for y in range(64)])
    assert abs(u.mean() - 0.5) < 0.02 and abs(u.var() - 1 / 12) < 0.01


def test_domain_full_is_reported():
    c = si.cfg(L=8, H=20, init_rows=16, growth_rate=5e-2)
    o = orc.Oracle(c)
    rc = 0
    for _ in range(400):
        rc = o.step(1)
        if rc:
            break
    assert rc == -4
    assert o.diagnostics()["status"] & orc.ST_DOMAIN_FULL
    assert o.step(1) == -4


def test_invalid_params_rejected():
    for bad in (dict(tau=0.5), dict(rho_c=0.0), dict(L=0), dict(sigma=-1.0),
                dict(growth_rate=-1e-3), dict(init_rows=100)):
        c = dict(si.SMALL_FP64)
        c.update(bad)
        with pytest.raises(ValueError):
            orc.Oracle(c)


# ---------------------------------------------------------------- growth adds no momentum
@pytest.mark.parametrize("mu", [0.0, 0.01])
def test_growth_injects_mass_but_no_momentum(mu):
    # proliferation puts equal mass on opposite directions (Sec. II), so with
    # bulk growth a uniform flow still loses momentum only to friction:
    # P(t) = P(0) (1 - mu/tau)^t while the mass grows by (1 + g) per step
    L, H, g, tau = 8, 6, 0.02, 0.9
    f = _ones_state(L, H, 1.0, 0.04, 0.02)
    c = si.cfg(L=L, H=H, init_rows=H, ybc="periodic", mu=mu, growth_rate=g,
               sigma=0.0, tau=tau)
    o = orc.Oracle(c)
    o.set_populations(f)
    P0 = np.array([v.sum() for v in d2q9.momentum(f)])
    for t in range(1, 41):
        o.step(1)
        fp = o.populations()
        P = np.array([v.sum() for v in d2q9.momentum(fp)])
        assert np.allclose(P, P0 * (1.0 - mu / tau) ** t, rtol=1e-12, atol=0), t
        assert np.isclose(fp.sum(), f.sum() * (1 + g) ** t, rtol=1e-12)


# ---------------------------------------------------------------- growth regions
@pytest.mark.parametrize("region,width", [("all", 0), ("front_band", 3), ("rear_band", 4)])
def test_source_counts_tissue_mass_in_region(region, width):
    # the injected mass of one step is g times the streamed density summed
    # over tissue sites in the region; region membership is evaluated here
    # from the definitions (front band: y >= h_prev(x) - ell; rear band:
    # y < wall + d)
    rng = np.random.default_rng(21)
    L, H, g = 12, 16, 0.01
    c = si.cfg(L=L, H=H, init_rows=0, sigma=0.0, growth_rate=g, region=region,
               region_width=width)
    for trial in range(5):
        f = _rand_front_state(rng, L, H)
        h_prev = rng.integers(0, H + 1, L).astype(np.int32)
        o = orc.Oracle(c)
        o.set_populations(f)
        o.set_front_heights(h_prev)
        rho_star = d2q9.stream_pull(f).sum(0)
        y = np.arange(H)[:, None] * np.ones((1, L), int)
        if region == "front_band":
            inreg = y >= h_prev[None, :] - width
        elif region == "rear_band":
            inreg = y < width
        else:
            inreg = np.ones((H, L), bool)
        want = g * rho_star[(rho_star >= c["rho_c"]) & inreg].sum()
        o.step(1)
        assert np.isclose(o.diagnostics()["src_total"], want, rtol=1e-13, atol=0)


# ---------------------------------------------------------------- rear wall rule
@pytest.mark.parametrize("gap,factor", [(20, 0.0), (4, 10.0)])
def test_rear_wall_keeps_required_gap_and_follows(gap, factor):
    # Appendix A: the wall stays at least max(gap, 10 w) behind the mean front,
    # and advances with it (it is never further back than one row more)
    c = dict(si.SMALL_FP64, sigma=1e-2, H=128, init_rows=90, ybc="follow",
             wall_min_gap=gap, wall_w_factor=factor, growth_rate=1e-2)
    o = orc.Oracle(c)
    moved = 0
    prev = o.diagnostics()["y_wall"]
    for t in range(300):
        o.step(1)
        d = o.diagnostics()
        need = max(float(gap), factor * d["W"])
        h = o.front_heights().astype(float)
        hbar = h.mean()
        assert hbar - d["y_wall"] >= need - 1e-9 or d["y_wall"] == prev
        if d["y_wall"] > prev:
            moved += 1
            # it moved as far as the rule allows, no further
            assert hbar - (d["y_wall"] + 1) < need + 1e-9
        assert d["y_wall"] >= prev
        prev = d["y_wall"]
    assert moved > 5


# ---------------------------------------------------------------- init amplitude
def test_initial_density_uniform_in_band():
    # Appendix A: rho uniform on [(1 - a) rho_init, (1 + a) rho_init]
    a = 0.1
    c = si.cfg(L=128, H=64, init_rows=64, init_amp=a, rho_init=0.1, rho_c=0.05)
    rho = orc.Oracle(c).populations().sum(0).ravel()
    n = rho.size
    assert rho.min() >= 0.09 - 1e-12 and rho.max() <= 0.11 + 1e-12
    assert rho.min() < 0.0901 and rho.max() > 0.1099
    sd = 0.1 * a / np.sqrt(3)
    assert abs(rho.mean() - 0.1) < 5 * sd / np.sqrt(n)
    assert abs(rho.var() / sd ** 2 - 1) < 0.05


# ---------------------------------------------------------------- step 7
def test_negative_fix_closed_form():
    # tau = 1, no noise or growth: the relaxed populations are the textbook
    # equilibrium at u* = (1 - mu) j/rho.  A fast flow makes some of them
    # negative.  Step 7: a negative rest population is zeroed and all nine
    # rescaled to the old total; then each negative moving population is
    # zeroed and its magnitude added to the reverse direction.
    cases = [
        [0.01, 1.0, 0.05, 0.0, 0.05, 0.1, 0.0, 0.0, 0.1],      # fast east: f_0 < 0
        [0.02, 0.0, 0.0, 0.05, 0.9, 0.0, 0.0, 0.12, 0.1],      # fast south: f_0 < 0
        [0.1, 0.5, 0.4, 0.0, 0.0, 0.3, 0.0, 0.0, 0.02],        # north-east: moving < 0
        [0.09, 0.05, 0.08, 0.7, 0.0, 0.0, 0.2, 0.14, 0.03],    # west
        [0.46, 0.3, 0.23, 0.04, 0.05, 0.12, 0.02, 0.015, 0.04],  # slow: no fix
    ]
    c = si.cfg(L=4, H=4, mu=0.0, tau=1.0, sigma=0.0, growth_rate=0.0, rho_c=0.1)
    n_rest_fix = 0
    for fs in cases:
        fs = np.array(fs)
        r0 = fs.sum()
        jx, jy = d2q9.momentum(fs)
        eq = d2q9.equilibrium(r0, jx / r0, jy / r0)      # what relaxation gives
        want = eq.copy()
        if want[0] < 0:
            n_rest_fix += 1
            tot = want.sum()
            want[0] = 0.0
            want = want * (tot / want.sum())
        for i in range(1, 9):
            if want[i] < 0:
                want[d2q9.OPP[i]] += -want[i]
                want[i] = 0.0
        out, tissue, S, dfix = orc.update_site(c, fs, 0, 0, 0, 0)
        assert tissue
        assert np.allclose(out, want, rtol=1e-12, atol=1e-15), (fs, out, want)
        assert np.all(out >= 0)
        assert np.isclose(dfix, out.sum() - eq.sum(), rtol=1e-10, atol=1e-15)
    assert n_rest_fix >= 2


def test_width_is_population_std_of_heights():
    # w(t) of Sec. III with the 1/L normalisation: numpy's population std
    c = dict(si.SMALL_FP64, sigma=2e-2, tau=0.8)
    o = orc.Oracle(c)
    for _ in range(5):
        o.step(40)
        h = o.front_heights().astype(float)
        d = o.diagnostics()
        assert abs(d["hbar"] - h.mean()) <= 1e-12 * h.mean()
        assert abs(d["W"] - h.std()) <= 1e-12 * max(h.std(), 1.0)
