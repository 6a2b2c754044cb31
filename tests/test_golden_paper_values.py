"""The oracle and the input recipe against values the paper prints
(`tests/golden/paper_values.json`, each entry with its citation): the D2Q7
weights and the coefficients of Eq. 3, the divisor of Eq. 4's zero-sum
noise and the range of its draws, the reverse directions of the bounce-back
rule, App. A's parameters, initial density band and rear-wall rule, App. B's
proliferating band, and the KPZ exponents the scaling pipeline recovers.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import synth_inputs as si
from oracle import oracle as orc
from paper_2303_02210_amd import scaling as sc
from tests import d2q7

_GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _num(v):
    return float(Fraction(v)) if isinstance(v, str) else float(v)


def _cfg7(**kw):
    return si.cfg(lattice="d2q7", **kw)


def test_weights_are_the_printed_ones():
    g = _GOLD["lattice_weights"]
    w = np.array([_num(g["w0"])] + [_num(g["w_moving"])] * 6)
    for rho in (1.0, 0.37, 2.5):
        # at rest Eq. 3 reduces to w_i rho
        assert np.array_equal(orc.fss7(rho, 0.0, 0.0), w * rho)


@pytest.mark.parametrize("rho,ux,uy", [(1.0, 0.03, -0.01), (0.6, -0.12, 0.05), (1.7, 0.0, 0.2)])
def test_steady_state_has_the_printed_coefficients(rho, ux, uy):
    g = _GOLD["steady_state_coefficients"]
    c = _num(_GOLD["appendix_a_parameters"]["c"])
    w = np.array([_num(_GOLD["lattice_weights"]["w0"])]
                 + [_num(_GOLD["lattice_weights"]["w_moving"])] * 6)
    eu = (d2q7.EX * ux + d2q7.EY * uy) / c
    want = w * rho * (1 + g["linear"] * eu + g["quadratic"] * eu * eu
                      + g["speed_squared"] * (ux * ux + uy * uy) / (c * c))
    assert np.allclose(orc.fss7(rho, ux, uy), want, rtol=1e-14, atol=1e-17)


def test_noise_subtracts_the_mean_over_seven_printed_draws():
    """One bulk tissue site stepped with and without noise: the difference is
    eta_i = eta~_i - (1/7) sum eta~, with eta~_i = sigma (2 U_i - 1) on
    [-sigma, sigma] from the site's draws."""
    g = _GOLD["noise"]
    sigma = 0.05
    p_on = orc.make_params(_cfg7(L=8, H=8, init_rows=8, sigma=sigma, tau=0.8))
    p_off = orc.make_params(_cfg7(L=8, H=8, init_rows=8, sigma=0.0, tau=0.8))
    fs = orc.fss7(1.0, 0.02, -0.01)
    for t, x, y in [(0, 1, 2), (5, 3, 7), (91, 6, 0)]:
        on = orc.update_site(p_on, fs, t, x, y, 8)[0][:7]
        off = orc.update_site(p_off, fs, t, x, y, 8)[0][:7]
        U = orc.noise_uniforms(p_on.seed, p_on.replica, t, x, y)[:7]
        raw = sigma * (2.0 * U - 1.0)
        assert np.all(np.abs(raw) <= sigma)
        eta = raw - raw.sum() / g["mean_divisor"]
        assert np.allclose(on - off, eta, rtol=0, atol=1e-15)
        assert abs((on - off).sum()) < 1e-15


def test_void_site_reverses_the_printed_pairs():
    pairs = _GOLD["reverse_pairs"]["pairs"]
    rev = {0: 0}
    for a, b in pairs:
        rev[a], rev[b] = b, a
    c = _cfg7(L=8, H=8, init_rows=0, rho_c=0.5)
    fs = np.array([0.01, 0.02, 0.03, 0.04, 0.05, 0.06, 0.07])   # sum 0.28 < rho_c
    out = orc.update_site(c, fs, 3, 2, 2, 0)[0][:7]
    for i in range(7):
        assert out[i] == fs[rev[i]], i


def test_paper_inputs_are_appendix_a_rescaled():
    """The paper's runs use App. A's parameters with every density scaled by
    rho_init -> 1 (sigma and rho_cell are densities too)."""
    g = _GOLD["appendix_a_parameters"]
    s = si.PAPER_BASE["rho_init"] / g["rho_init"]
    pb = si.PAPER_BASE
    assert pb["lattice"] == "d2q7"
    assert pb["tau"] == g["tau"] and pb["mu"] == g["mu"] and pb["growth_rate"] == g["g"]
    for key, gk in (("rho_c", "rho_c"), ("sigma", "sigma"), ("rho_cell", "rho_cell"),
                    ("rho0", "rho0")):
        assert pb[key] == pytest.approx(g[gk] * s, rel=1e-12), key
    band = _GOLD["initial_density"]["band"]
    assert 1 - pb["init_amp"] == pytest.approx(band[0]) and 1 + pb["init_amp"] == pytest.approx(band[1])
    wall = _GOLD["rear_wall"]
    assert pb["ybc"] == "follow"
    assert pb["wall_min_gap"] == wall["min_gap"] and pb["wall_w_factor"] == wall["w_factor"]
    b = _GOLD["appendix_b_band"]
    rear = [r for r in si.appendix_b(2) if r["region"] == "rear_band"]
    assert rear and all(r["region_width"] == b["rows_from_rear_wall"] and r["L"] == b["L"]
                        for r in rear)


def test_initial_density_fills_the_printed_band():
    band = _GOLD["initial_density"]["band"]
    c = _cfg7(L=64, H=32, init_rows=20, init_amp=0.1, rho_init=1.0, sigma=0.0)
    o = orc.Oracle(c)
    rho = o.populations().sum(0)[:20]
    assert rho.min() >= band[0] and rho.max() <= band[1]
    assert rho.min() < band[0] + 0.01 and rho.max() > band[1] - 0.01
    # at rest: f_i = w_i rho (Eq. 3 with u = 0)
    w = np.array([0.5] + [1 / 12] * 6)
    assert np.allclose(o.populations()[:, :20, :], w[:, None, None] * rho[None], rtol=1e-15)
    o.close()


def test_rear_wall_rule_uses_the_printed_gap():
    """With App. A's rule the wall sits max(50, 10 w) behind the mean front
    once it has moved (flat front: the 50-row floor decides)."""
    wall = _GOLD["rear_wall"]
    c = _cfg7(L=16, H=160, init_rows=120, init_amp=0.0, sigma=0.0, ybc="follow",
              wall_min_gap=wall["min_gap"], wall_w_factor=float(wall["w_factor"]))
    o = orc.Oracle(c)
    o.step(1)
    d = o.diagnostics()
    need = max(float(wall["min_gap"]), wall["w_factor"] * d["W"])
    assert d["y_wall"] == int(np.floor(d["hbar"] - need))
    assert d["y_wall"] > 0
    o.close()


def test_scaling_pipeline_recovers_the_printed_kpz_exponents():
    g = _GOLD["kpz_exponents"]
    a, b, z = _num(g["alpha"]), _num(g["beta"]), _num(g["z"])
    assert z == pytest.approx(a / b)
    curves = {}
    for L in (32, 64, 128, 256):
        t = np.logspace(0, np.log10(60 * L ** z), 400)
        F = ((t / L ** z) ** (-b * 3.0) + 1.0) ** (-1.0 / 3.0)
        curves[L] = (t, L ** a * F)
    fit = sc.fit_exponents(curves)
    assert fit["alpha"] == pytest.approx(a, abs=0.01)
    assert fit["beta"] == pytest.approx(b, abs=0.03)
    assert fit["z"] == pytest.approx(z, abs=0.02)
