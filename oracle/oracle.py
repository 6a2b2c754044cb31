"""ctypes wrapper around the FP64 CPU oracle (``liblbm_oracle.so``).

TEST INFRASTRUCTURE ONLY: the oracle is the plain reference the GPU library is
checked against.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product package never does.

The oracle follows Appendix A of arXiv 2303.02210 (steps 1-7 per site, then
the front heights, the width of Sec. III and the rear-wall rule), on the
square D2Q9 lattice or on the paper's triangular D2Q7 lattice; see
``lbm_oracle.c`` for the per-step citations.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.environ.get("LBM_ORACLE_LIB") or os.path.join(_HERE, "liblbm_oracle.so")

GROWTH = {"none": 0, "bulk": 1, "division": 2, "division_density": 3}
REGION = {"all": 0, "front_band": 1, "rear_band": 2}
YBC = {"fixed": 0, "follow": 1, "periodic": 2}
LATTICE = {"d2q9": 0, "d2q7": 1}
# how the division laws pick their sites: "per_site" (a Poisson count per
# eligible site, the GPU library's form) or "selection" (Sec. II literally)
DIVISION_MODE = {"per_site": 0, "selection": 1}
Q = {"d2q9": 9, "d2q7": 7}
ST_DOMAIN_FULL = 1
ST_NONFINITE = 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc: no fast-math, no FMA contraction."""
    if os.environ.get("LBM_ORACLE_LIB"):
        return _LIB
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32), ("H", ctypes.c_int32),
        ("tau", ctypes.c_double), ("mu", ctypes.c_double), ("rho_c", ctypes.c_double),
        ("rho_init", ctypes.c_double), ("init_amp", ctypes.c_double),
        ("init_rows", ctypes.c_int32),
        ("growth", ctypes.c_int32), ("growth_rate", ctypes.c_double),
        ("region", ctypes.c_int32), ("region_width", ctypes.c_int32),
        ("sigma", ctypes.c_double),
        ("ybc", ctypes.c_int32), ("wall_min_gap", ctypes.c_int32),
        ("wall_w_factor", ctypes.c_double),
        ("seed", ctypes.c_uint32), ("replica", ctypes.c_uint32),
        ("rho_cell", ctypes.c_double), ("rho0", ctypes.c_double),
        ("lattice", ctypes.c_int32), ("division_mode", ctypes.c_int32),
    ]


class _Diag(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("src_total", ctypes.c_double),
        ("fix_total", ctypes.c_double), ("retired", ctypes.c_double),
        ("hbar", ctypes.c_double), ("W", ctypes.c_double),
        ("step", ctypes.c_int64), ("y_wall", ctypes.c_int64), ("h_hi", ctypes.c_int64),
        ("status", ctypes.c_uint32),
        ("lam", ctypes.c_double), ("divisions", ctypes.c_int64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        L = _lib
        dp = ctypes.POINTER(ctypes.c_double)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_noise_bits.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64,
                                     ctypes.c_int32, ctypes.c_int64, u32p]
        L.orc_noise_uniforms.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64,
                                         ctypes.c_int32, ctypes.c_int64, dp]
        L.orc_init_uniform.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int32,
                                       ctypes.c_int64]
        L.orc_init_uniform.restype = ctypes.c_double
        L.orc_lattice.argtypes = [i32p, i32p, i32p, dp]
        L.orc_fss.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.orc_pull_site.argtypes = [ctypes.POINTER(_Params), dp, ctypes.c_int32,
                                    ctypes.c_int32, dp]
        L.orc_pull_site_abs.argtypes = [ctypes.POINTER(_Params), dp, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int64, dp]
        L.orc_fss7.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.orc_q.argtypes = [ctypes.POINTER(_Params)]
        L.orc_q.restype = ctypes.c_int
        L.orc_update_site.argtypes = [ctypes.POINTER(_Params), dp, ctypes.c_int64,
                                      ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_int64, ctypes.c_int, ctypes.c_double, dp, dp, dp,
                                      i32p, ctypes.POINTER(ctypes.c_int64)]
        L.orc_update_site.restype = ctypes.c_int
        L.orc_selection_draws.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64,
                                          ctypes.c_int64, dp, dp, u32p]
        L.orc_selection_round_uniform.argtypes = [ctypes.c_uint32, ctypes.c_uint32,
                                                  ctypes.c_int64]
        L.orc_selection_round_uniform.restype = ctypes.c_double
        L.orc_division_draws.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64,
                                         ctypes.c_int32, ctypes.c_int64, dp,
                                         ctypes.POINTER(ctypes.c_uint64)]
        L.orc_exp_neg.argtypes = [ctypes.c_double]
        L.orc_exp_neg.restype = ctypes.c_double
        L.orc_poisson_k.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_poisson_k.restype = ctypes.c_int
        L.orc_create.argtypes = [ctypes.POINTER(_Params)]
        L.orc_create.restype = ctypes.c_void_p
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.orc_step.restype = ctypes.c_int
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_diagnostics.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Diag)]
        L.orc_front_heights.argtypes = [ctypes.c_void_p, i32p]
        L.orc_get_populations.argtypes = [ctypes.c_void_p, dp]
        L.orc_set_populations.argtypes = [ctypes.c_void_p, dp]
        L.orc_set_front_heights.argtypes = [ctypes.c_void_p, i32p]
        L.orc_set_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.orc_set_lam.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.orc_division_map.argtypes = [ctypes.c_void_p, i32p]
        L.orc_clear_division_map.argtypes = [ctypes.c_void_p]
        L.orc_selection_counts.argtypes = [ctypes.c_void_p, i32p]
        L.orc_selection_counts.restype = ctypes.c_int
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def make_params(cfg: dict) -> _Params:
    """Map a workload dict (see ``synth_inputs``) to the oracle's struct."""
    p = _Params()
    p.L = int(cfg["L"])
    p.H = int(cfg["H"])
    p.tau = float(cfg.get("tau", 1.0))
    p.mu = float(cfg.get("mu", 1e-3))
    p.rho_c = float(cfg.get("rho_c", 0.5))
    p.rho_init = float(cfg.get("rho_init", 1.0))
    p.init_amp = float(cfg.get("init_amp", 1e-3))
    p.init_rows = int(cfg.get("init_rows", 0))
    p.growth = GROWTH[cfg.get("growth", "bulk")]
    p.growth_rate = float(cfg.get("growth_rate", 0.0))
    p.region = REGION[cfg.get("region", "all")]
    p.region_width = int(cfg.get("region_width", 0))
    p.sigma = float(cfg.get("sigma", 0.0))
    p.ybc = YBC[cfg.get("ybc", "fixed")]
    p.wall_min_gap = int(cfg.get("wall_min_gap", 50))
    p.wall_w_factor = float(cfg.get("wall_w_factor", 10.0))
    p.seed = int(cfg.get("seed", 0)) & 0xFFFFFFFF
    p.replica = int(cfg.get("replica", 0)) & 0xFFFFFFFF
    p.rho_cell = float(cfg.get("rho_cell", 0.1))
    p.rho0 = float(cfg.get("rho0", 1.5))
    p.lattice = LATTICE[cfg.get("lattice", "d2q9")]
    p.division_mode = DIVISION_MODE[cfg.get("division_mode", "per_site")]
    return p


def q_of(p: _Params) -> int:
    """Populations per site of the lattice p names."""
    return 7 if p.lattice == LATTICE["d2q7"] else 9


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                            _ptr(out, ctypes.c_uint32))
    return out


def noise_bits(seed, replica, t, x, y) -> np.ndarray:
    out = np.zeros(9, dtype=np.uint32)
    lib().orc_noise_bits(seed, replica, t, x, y, _ptr(out, ctypes.c_uint32))
    return out


def noise_uniforms(seed, replica, t, x, y) -> np.ndarray:
    out = np.zeros(9, dtype=np.float64)
    lib().orc_noise_uniforms(seed, replica, t, x, y, _ptr(out, ctypes.c_double))
    return out


def init_uniform(seed, replica, x, y) -> float:
    return float(lib().orc_init_uniform(seed, replica, x, y))


def division_draws(seed, replica, t, x, y):
    """(U, axes): the Poisson uniform and the 64 axis bits of one site."""
    U = ctypes.c_double()
    ax = ctypes.c_uint64()
    lib().orc_division_draws(seed, replica, t, x, y, ctypes.byref(U), ctypes.byref(ax))
    return U.value, ax.value


def selection_draws(seed, replica, t, a):
    """(U_site, U_acc, axis_bits) of attempt a of the selection procedure."""
    us, ua = ctypes.c_double(), ctypes.c_double()
    bits = ctypes.c_uint32()
    lib().orc_selection_draws(seed, replica, t, a, ctypes.byref(us), ctypes.byref(ua),
                              ctypes.byref(bits))
    return us.value, ua.value, bits.value


def selection_round_uniform(seed, replica, t) -> float:
    return float(lib().orc_selection_round_uniform(seed, replica, t))


def exp_neg(lam: float) -> float:
    return float(lib().orc_exp_neg(float(lam)))


def poisson_k(U: float, lam: float) -> int:
    return int(lib().orc_poisson_k(float(U), float(lam)))


def lattice():
    cx = np.zeros(9, np.int32)
    cy = np.zeros(9, np.int32)
    opp = np.zeros(9, np.int32)
    w = np.zeros(9, np.float64)
    lib().orc_lattice(_ptr(cx, ctypes.c_int32), _ptr(cy, ctypes.c_int32),
                      _ptr(opp, ctypes.c_int32), _ptr(w, ctypes.c_double))
    return cx, cy, opp, w


def fss(rho, ux, uy) -> np.ndarray:
    out = np.zeros(9, np.float64)
    lib().orc_fss(float(rho), float(ux), float(uy), _ptr(out, ctypes.c_double))
    return out


def fss7(rho, ux, uy) -> np.ndarray:
    out = np.zeros(7, np.float64)
    lib().orc_fss7(float(rho), float(ux), float(uy), _ptr(out, ctypes.c_double))
    return out


def pull_site(cfg_or_params, f: np.ndarray, x: int, j: int, y_abs: int | None = None) -> np.ndarray:
    """Step 1 at window row j (absolute row y_abs, default j)."""
    p = cfg_or_params if isinstance(cfg_or_params, _Params) else make_params(cfg_or_params)
    q = q_of(p)
    f = np.ascontiguousarray(f, dtype=np.float64)
    assert f.shape == (q, p.H, p.L)
    out = np.zeros(9, np.float64)
    lib().orc_pull_site_abs(ctypes.byref(p), _ptr(f, ctypes.c_double), x, j,
                            j if y_abs is None else int(y_abs), _ptr(out, ctypes.c_double))
    return out[:q]


def update_site_ex(cfg_or_params, fstar, t, x, y_abs, h_prev_x, y_wall=0, force=-1, lam=0.0):
    """Steps 2-7 at one site.  Returns (f_out[Q], tissue, S, dfix, ndiv, wfx)."""
    p = cfg_or_params if isinstance(cfg_or_params, _Params) else make_params(cfg_or_params)
    q = q_of(p)
    fs = np.zeros(9, np.float64)
    fs[:q] = np.asarray(fstar, dtype=np.float64)[:q]
    out = np.zeros(9, np.float64)
    S = ctypes.c_double()
    dfix = ctypes.c_double()
    nd = ctypes.c_int32()
    wfx = ctypes.c_int64()
    tissue = lib().orc_update_site(ctypes.byref(p), _ptr(fs, ctypes.c_double), int(t),
                                   int(x), int(y_abs), int(h_prev_x), int(y_wall), int(force),
                                   float(lam), _ptr(out, ctypes.c_double), ctypes.byref(S),
                                   ctypes.byref(dfix), ctypes.byref(nd), ctypes.byref(wfx))
    return out[:q], bool(tissue), S.value, dfix.value, nd.value, wfx.value


def update_site(cfg_or_params, fstar, t, x, y_abs, h_prev_x, y_wall=0, force=-1, lam=0.0):
    """Steps 2-7 at one site.  Returns (f_out[Q], tissue, S, dfix)."""
    return update_site_ex(cfg_or_params, fstar, t, x, y_abs, h_prev_x, y_wall, force, lam)[:4]


class Oracle:
    """One FP64 CPU simulation: same life cycle as the GPU handle."""

    def __init__(self, cfg: dict):
        self.cfg = dict(cfg)
        self.p = make_params(cfg)
        self._h = lib().orc_create(ctypes.byref(self.p))
        if not self._h:
            raise ValueError("invalid oracle parameters")
        self.L = self.p.L
        self.H = self.p.H
        self.Q = q_of(self.p)

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1) -> int:
        return int(lib().orc_step(self._h, int(n)))

    def diagnostics(self) -> dict:
        d = _Diag()
        lib().orc_diagnostics(self._h, ctypes.byref(d))
        return {k: getattr(d, k) for k, _ in _Diag._fields_}

    def front_heights(self) -> np.ndarray:
        out = np.zeros(self.L, np.int32)
        lib().orc_front_heights(self._h, _ptr(out, ctypes.c_int32))
        return out

    def set_front_heights(self, h) -> None:
        a = np.ascontiguousarray(h, dtype=np.int32)
        assert a.shape == (self.L,)
        lib().orc_set_front_heights(self._h, _ptr(a, ctypes.c_int32))

    def populations(self) -> np.ndarray:
        out = np.zeros((self.Q, self.H, self.L), np.float64)
        lib().orc_get_populations(self._h, _ptr(out, ctypes.c_double))
        return out

    def set_populations(self, f) -> None:
        a = np.ascontiguousarray(f, dtype=np.float64)
        assert a.shape == (self.Q, self.H, self.L)
        lib().orc_set_populations(self._h, _ptr(a, ctypes.c_double))

    def set_step(self, t: int) -> None:
        lib().orc_set_step(self._h, int(t))

    def set_lam(self, lam: float) -> None:
        lib().orc_set_lam(self._h, float(lam))

    def selection_counts(self) -> np.ndarray:
        """The selection procedure's divisions of the last step, [H][L][axes]."""
        na = 3 if self.p.lattice == LATTICE["d2q7"] else 4
        out = np.zeros((self.H, self.L, na), np.int32)
        if lib().orc_selection_counts(self._h, _ptr(out, ctypes.c_int32)) == 0:
            raise ValueError("not a selection-procedure run")
        return out

    def division_map(self, clear: bool = False) -> np.ndarray:
        out = np.zeros((self.H, self.L), np.int32)
        lib().orc_division_map(self._h, _ptr(out, ctypes.c_int32))
        if clear:
            lib().orc_clear_division_map(self._h)
        return out
