"""The analysis functions of the scaling pipeline against curves whose
exponents, amplitudes and rates are known by construction (Family-Vicsek
scaling with alpha = 1/2, beta = 1/3, z = 3/2 as for KPZ; pure Fourier
modes; exponential growth; the dispersion relation of Eq. 7), and the
extreme-region division count against a direct loop."""
import numpy as np
import pytest

from paper_2303_02210_amd import scaling as sc


def _fv_curves(alpha=0.5, beta=1 / 3, z=1.5, Ls=(32, 64, 128, 256), s=3.0, noise=0.0, seed=0):
    rng = np.random.default_rng(seed)
    curves = {}
    for L in Ls:
        t = np.logspace(0, np.log10(60 * L ** z), 400)
        u = t / L ** z
        F = (u ** (-beta * s) + 1.0) ** (-1.0 / s)
        w = L ** alpha * F * (1 + noise * rng.standard_normal(t.size))
        curves[L] = (t, w)
    return curves


def test_exponents_recovered_from_family_vicsek_curves():
    fit = sc.fit_exponents(_fv_curves())
    assert fit["alpha"] == pytest.approx(0.5, abs=0.01)
    assert fit["beta"] == pytest.approx(1 / 3, abs=0.03)
    assert fit["z"] == pytest.approx(1.5, abs=0.02)
    assert fit["alpha_over_beta"] == pytest.approx(1.5, abs=0.15)


def test_exponents_of_another_class():
    # Edwards-Wilkinson in 1+1 dimensions: alpha 1/2, beta 1/4, z 2
    fit = sc.fit_exponents(_fv_curves(alpha=0.5, beta=0.25, z=2.0, Ls=(16, 32, 64, 128)))
    assert fit["alpha"] == pytest.approx(0.5, abs=0.01)
    assert fit["beta"] == pytest.approx(0.25, abs=0.03)
    assert fit["z"] == pytest.approx(2.0, abs=0.03)


def test_collapse_measures_the_right_exponents():
    curves = _fv_curves(noise=0.01, seed=3)
    _, good = sc.collapse(curves, 0.5, 1.5)
    _, bad_a = sc.collapse(curves, 0.3, 1.5)
    _, bad_z = sc.collapse(curves, 0.5, 1.0)
    assert good < 0.02 and bad_a > 5 * good and bad_z > 5 * good


def test_saturation_of_a_noisy_plateau():
    rng = np.random.default_rng(1)
    t = np.arange(1000.0)
    w = 3.0 + 0.1 * rng.standard_normal(1000)
    m, se = sc.saturation(t, w)
    assert m == pytest.approx(3.0, abs=4 * 0.1 / np.sqrt(300))
    assert 0 < se < 0.05


def test_mode_amplitude_and_growth_rate():
    L = 128
    x = np.arange(L)
    for n, A in ((1, 2.0), (3, 0.7), (10, 0.05)):
        h = 50.0 + A * np.cos(2 * np.pi * n * x / L + 0.4) + 0.3 * np.cos(2 * np.pi * 17 * x / L)
        assert sc.mode_amplitude(h, n) == pytest.approx(A, rel=1e-12)
    t = np.arange(0, 500, 10.0)
    assert sc.growth_rate(t, 0.3 * np.exp(-2.5e-3 * t)) == pytest.approx(-2.5e-3, rel=1e-9)


def test_dispersion_fit_of_eq7():
    q = 2 * np.pi * np.arange(1, 9) / 256
    om = 4e-4 - 0.3 * q ** 2
    fit = sc.fit_dispersion(q, om)
    assert fit["k"] == pytest.approx(4e-4, rel=1e-9)
    assert fit["gamma"] == pytest.approx(0.3, rel=1e-9)
    assert fit["L_c"] == pytest.approx(np.sqrt(0.3 / 4e-4), rel=1e-9)
    assert fit["q_c"] == pytest.approx(np.sqrt(4e-4 / 0.3), rel=1e-9)


def test_division_difference_against_a_direct_count():
    rng = np.random.default_rng(5)
    L, H, y_wall = 64, 80, 37
    for _ in range(20):
        dm = rng.integers(0, 4, (H, L))
        h = y_wall + rng.integers(25, 75, L)
        got = sc.division_difference(dm, h, y_wall)
        want = []
        for xc in (int(np.argmax(h)), int(np.argmin(h))):
            tot = 0
            for dx in range(-10, 11):
                x = (xc + dx) % L
                for y in range(int(h[x]) - 20, int(h[x])):
                    j = y - y_wall
                    if 0 <= j < H:
                        tot += int(dm[j, x])
            want.append(tot)
        assert got == want[0] - want[1]
