"""The paper's observables from the engine's output (Sec. III and IV):

* the interface width w(L, t), its growth exponent beta (w ~ t^beta before
  saturation), saturated width w_inf ~ L^alpha and crossover time
  t_inf ~ L^z, and the collapse of w / L^alpha against t / L^z (Fig. 2);
* the difference between the divisions near the most and the least advanced
  parts of the front (Fig. 3c): 21 columns (10 either side) around h_max and
  around h_min, each 20 rows into the tissue below its own front;
* the growth rate omega(q) of a sinusoidal front perturbation and the fit of
  the dispersion relation omega = k - gamma q^2 of Eq. 7.

Host-side numpy only; the curves, front heights and division maps come from
the GPU library (``Sim``, ``Ensemble``).
"""
from __future__ import annotations

import numpy as np


# --------------------------------------------------------------------- w(L, t)
def saturation(t, w, tail: float = 0.3):
    """w_inf: the mean of w over the last `tail` fraction of the run's time,
    and its standard error over that window (blocks of 10 samples)."""
    t = np.asarray(t, float)
    w = np.asarray(w, float)
    seg = w[t >= t[-1] - tail * (t[-1] - t[0])]
    nb = max(1, len(seg) // 10)
    blocks = np.array([b.mean() for b in np.array_split(seg, nb)])
    se = blocks.std(ddof=1) / np.sqrt(nb) if nb > 1 else 0.0
    return float(seg.mean()), float(se)


def growth_exponent(t, w, t_max: float | None = None, t_min: float | None = None):
    """beta: least-squares slope of log w against log t over (t_min, t_max]
    (default: from the first positive sample to a third of the crossover,
    estimated as where w first reaches half of its saturated value)."""
    t = np.asarray(t, float)
    w = np.asarray(w, float)
    if t_max is None:
        w_inf, _ = saturation(t, w)
        reach = np.nonzero(w >= 0.5 * w_inf)[0]
        t_max = t[reach[0]] if reach.size else t[-1]
    lo = t_min if t_min is not None else 0.0
    m = (t > lo) & (t <= t_max) & (w > 0)
    if m.sum() < 3:
        return float("nan")
    return float(np.polyfit(np.log(t[m]), np.log(w[m]), 1)[0])


def crossover_time(t, w, beta: float | None = None):
    """t_inf: where the early power law A t^beta reaches w_inf."""
    t = np.asarray(t, float)
    w = np.asarray(w, float)
    w_inf, _ = saturation(t, w)
    reach = np.nonzero(w >= 0.5 * w_inf)[0]
    t_hi = t[reach[0]] if reach.size else t[-1]
    m = (t > 0) & (t <= t_hi) & (w > 0)
    if m.sum() < 3:
        return float("nan")
    b, logA = np.polyfit(np.log(t[m]), np.log(w[m]), 1)
    if beta is not None:
        b = beta
        logA = float(np.mean(np.log(w[m]) - b * np.log(t[m])))
    return float(np.exp((np.log(w_inf) - logA) / b))


def fit_exponents(curves: dict):
    """curves: {L: (t, w)} with w averaged over runs.  Returns alpha (slope
    of log w_inf on log L), beta (mean growth exponent over the sizes), z
    from t_inf ~ L^z, the ratio alpha / beta, and the per-size figures."""
    Ls = np.array(sorted(curves), float)
    per = {}
    for L in Ls:
        t, w = curves[int(L)] if int(L) in curves else curves[L]
        w_inf, se = saturation(t, w)
        b = growth_exponent(t, w)
        per[int(L)] = {"w_inf": w_inf, "w_inf_se": se, "beta": b}
    beta = float(np.nanmean([per[int(L)]["beta"] for L in Ls]))
    for L in Ls:
        t, w = curves[int(L)] if int(L) in curves else curves[L]
        per[int(L)]["t_inf"] = crossover_time(t, w, beta)
    alpha = float(np.polyfit(np.log(Ls), np.log([per[int(L)]["w_inf"] for L in Ls]), 1)[0])
    z = float(np.polyfit(np.log(Ls), np.log([per[int(L)]["t_inf"] for L in Ls]), 1)[0])
    return {"alpha": alpha, "beta": beta, "z": z, "alpha_over_beta": alpha / beta,
            "sizes": per}


def collapse(curves: dict, alpha: float, z: float, bins: int = 24):
    """Rescale each curve to (t / L^z, w / L^alpha) and measure how well they
    fall on one curve: the mean over log-spaced bins of the spread (std / mean)
    of the rescaled widths of the sizes present in the bin."""
    out = {}
    xs, ys, labels = [], [], []
    for L, (t, w) in curves.items():
        t = np.asarray(t, float)
        w = np.asarray(w, float)
        m = (t > 0) & (w > 0)
        x = t[m] / float(L) ** z
        y = w[m] / float(L) ** alpha
        out[int(L)] = (x, y)
        xs.append(x)
        ys.append(y)
        labels.append(np.full(x.size, int(L)))
    x = np.concatenate(xs)
    y = np.concatenate(ys)
    lab = np.concatenate(labels)
    edges = np.logspace(np.log10(x.min()), np.log10(x.max()), bins + 1)
    spreads = []
    for a, b in zip(edges[:-1], edges[1:]):
        sel = (x >= a) & (x < b)
        if len(np.unique(lab[sel])) < 2:
            continue
        means = [y[sel & (lab == L)].mean() for L in np.unique(lab[sel])]
        spreads.append(np.std(means) / np.mean(means))
    return out, float(np.mean(spreads)) if spreads else float("nan")


# ----------------------------------------------------- divisions near extremes
def extreme_regions(h, half_width: int = 10, depth: int = 20):
    """The two regions of Fig. 3c for front heights h(x) (periodic in x): the
    columns within half_width of the column of h_max (h_min), each taken
    `depth` rows into the tissue below its own front height.  Returns
    (cols, row_lo, row_hi) for the maximum and for the minimum, with per-column
    absolute rows [row_lo, row_hi)."""
    h = np.asarray(h)
    L = h.size
    out = []
    for xc in (int(np.argmax(h)), int(np.argmin(h))):
        cols = (xc + np.arange(-half_width, half_width + 1)) % L
        top = h[cols].astype(np.int64)
        out.append((cols, top - depth, top))
    return tuple(out)


def division_difference(div_map, h, y_wall: int, half_width: int = 10, depth: int = 20):
    """Divisions in the region around h_max minus those in the region around
    h_min.  div_map[j, x] counts divisions at window row j (absolute row
    y_wall + j)."""
    div_map = np.asarray(div_map)
    H = div_map.shape[0]
    tot = []
    for cols, lo, hi in extreme_regions(h, half_width, depth):
        n = 0
        for x, a, b in zip(cols, lo, hi):
            j0 = max(int(a) - y_wall, 0)
            j1 = min(int(b) - y_wall, H)
            if j1 > j0:
                n += int(div_map[j0:j1, x].sum())
        tot.append(n)
    return tot[0] - tot[1]


# ---------------------------------------------------------------- dispersion
def mode_amplitude(h, n: int) -> float:
    """|c_n|: the amplitude of the n-th Fourier mode of the front h(x)
    (h = h_bar + A cos(2 pi n x / L + phase) gives A)."""
    h = np.asarray(h, float)
    L = h.size
    c = np.fft.rfft(h - h.mean())
    return float(2.0 * np.abs(c[n]) / L)


def growth_rate(t, amp):
    """omega: least-squares slope of log amplitude against t."""
    t = np.asarray(t, float)
    a = np.asarray(amp, float)
    m = a > 0
    return float(np.polyfit(t[m], np.log(a[m]), 1)[0])


def fit_dispersion(q, omega):
    """k and gamma of omega = k - gamma q^2 (Eq. 7) by least squares, the
    marginal wavenumber q_c = sqrt(k / gamma) and the paper's critical length
    L_c = sqrt(gamma / k)."""
    q = np.asarray(q, float)
    om = np.asarray(omega, float)
    A = np.stack([np.ones_like(q), -q * q], axis=1)
    (k, gamma), *_ = np.linalg.lstsq(A, om, rcond=None)
    ok = k > 0 and gamma > 0
    return {"k": float(k), "gamma": float(gamma),
            "q_c": float(np.sqrt(k / gamma)) if ok else float("nan"),
            "L_c": float(np.sqrt(gamma / k)) if ok else float("nan")}
