"""ctypes declarations of ``include/lbmgrow.h`` and the in-tree library loader.

Argument marshalling only: every step of the simulation runs in the gfx950
kernels of ``liblbmgrow.so``.  If the library has not been built, importing
this module raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbmgrow.so")

ABI_VERSION = 4

OK = 0
E_INVALID, E_NOMEM, E_DEVICE, E_DOMAIN_FULL, E_NONFINITE, E_UNSUPPORTED, E_STATE = (
    -1, -2, -3, -4, -5, -6, -7)
ERROR_NAMES = {0: "OK", -1: "LBM_E_INVALID", -2: "LBM_E_NOMEM", -3: "LBM_E_DEVICE",
               -4: "LBM_E_DOMAIN_FULL", -5: "LBM_E_NONFINITE", -6: "LBM_E_UNSUPPORTED",
               -7: "LBM_E_STATE"}

PRECISION = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3}
STORAGE_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}
LATTICE = {"d2q9": 0, "d2q7": 1}
Q = {"d2q9": 9, "d2q7": 7}
GROWTH = {"none": 0, "bulk": 1, "division": 2, "division_density": 3}
REGION = {"all": 0, "front_band": 1, "rear_band": 2}
YBC = {"fixed": 0, "follow": 1, "periodic": 2}
FLAG_WINDOW = 1
FLAG_DIVISION_MAP = 2
FLAG_STOCHASTIC_ROUND = 4
FLAG_BATCH_TABLE = 8
FLAG_BATCH_OWN = 16
ST_DOMAIN_FULL = 1
ST_NONFINITE = 2
ST_SYNC_LOST = 4


class Params(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32), ("struct_size", ctypes.c_uint32),
        ("L", ctypes.c_int32), ("H", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("growth", ctypes.c_int32),
        ("tau", ctypes.c_double), ("mu", ctypes.c_double), ("rho_c", ctypes.c_double),
        ("rho_init", ctypes.c_double), ("init_amp", ctypes.c_double),
        ("init_rows", ctypes.c_int32), ("region", ctypes.c_int32),
        ("growth_rate", ctypes.c_double),
        ("region_width", ctypes.c_int32), ("ybc", ctypes.c_int32),
        ("sigma", ctypes.c_double),
        ("wall_min_gap", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("wall_w_factor", ctypes.c_double), ("rho_ref", ctypes.c_double),
        ("seed", ctypes.c_uint32), ("replica", ctypes.c_uint32),
        ("kernel_vb", ctypes.c_int32), ("kernel_ty", ctypes.c_int32),
        ("rho_cell", ctypes.c_double), ("rho0", ctypes.c_double),
        ("lattice", ctypes.c_int32), ("kernel_order", ctypes.c_int32),
    ]


class Diag(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("src_total", ctypes.c_double),
        ("fix_total", ctypes.c_double), ("retired", ctypes.c_double),
        ("hbar", ctypes.c_double), ("W", ctypes.c_double),
        ("step", ctypes.c_int64), ("y_wall", ctypes.c_int64), ("h_hi", ctypes.c_int64),
        ("status", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
        ("lam", ctypes.c_double), ("divisions", ctypes.c_int64),
        ("rows_swept", ctypes.c_int64),
    ]


# (name, restype, argtypes) of every entry point in include/lbmgrow.h
_VP = ctypes.c_void_p
_SIGS = [
    ("lbm_version", ctypes.c_char_p, []),
    ("lbm_workspace_bytes", ctypes.c_size_t, [ctypes.POINTER(Params)]),
    ("lbm_create", ctypes.c_int, [ctypes.POINTER(Params), _VP, ctypes.c_size_t, _VP,
                                  ctypes.POINTER(_VP)]),
    ("lbm_create_static", ctypes.c_int, [ctypes.POINTER(Params), _VP,
                                         ctypes.POINTER(ctypes.c_size_t), _VP,
                                         ctypes.POINTER(_VP)]),
    ("lbm_step", ctypes.c_int, [_VP, ctypes.c_int64]),
    ("lbm_front_heights", ctypes.c_int, [_VP, _VP, ctypes.POINTER(ctypes.c_int64)]),
    ("lbm_front_heights_async", ctypes.c_int, [_VP, _VP]),
    ("lbm_diagnostics", ctypes.c_int, [_VP, ctypes.POINTER(Diag)]),
    ("lbm_get_populations", ctypes.c_int, [_VP, _VP]),
    ("lbm_set_populations", ctypes.c_int, [_VP, _VP]),
    ("lbm_set_front_heights", ctypes.c_int, [_VP, _VP]),
    ("lbm_division_map", ctypes.c_int, [_VP, _VP, ctypes.c_int]),
    ("lbm_state_bytes", ctypes.c_size_t, [_VP]),
    ("lbm_get_state", ctypes.c_int, [_VP, _VP, ctypes.c_size_t]),
    ("lbm_set_state", ctypes.c_int, [_VP, _VP, ctypes.c_size_t]),
    ("lbm_stream_copy", ctypes.c_int, [_VP, _VP, ctypes.c_size_t, _VP]),
    ("lbm_last_error", ctypes.c_char_p, [_VP]),
    ("lbm_destroy", ctypes.c_int, [_VP]),
    ("lbm_tiles", ctypes.c_int64, [ctypes.POINTER(Params)]),
    ("lbm_batch_workspace_bytes", ctypes.c_size_t, [ctypes.c_int, ctypes.c_int64]),
    ("lbm_batch_create", ctypes.c_int, [_VP, ctypes.c_size_t, ctypes.c_int, ctypes.c_int64, _VP,
                                        ctypes.POINTER(_VP)]),
    ("lbm_batch_add", ctypes.c_int, [_VP, _VP]),
    ("lbm_batch_remove", ctypes.c_int, [_VP, _VP]),
    ("lbm_batch_step", ctypes.c_int, [_VP, ctypes.c_int64]),
    ("lbm_batch_persistent", ctypes.c_int, [_VP, ctypes.c_int]),
    ("lbm_batch_destroy", ctypes.c_int, [_VP]),
]
ENTRY_POINTS = [s[0] for s in _SIGS]

_lib = None


def lib() -> ctypes.CDLL:
    """Load ``liblbmgrow.so`` from the package directory (no fallback)."""
    global _lib
    if _lib is None:
        # torch carries its own copy of the HIP runtime (same soname as the
        # system's): load torch first so that the library binds to that one
        # copy, or the process would hold two runtimes and torch's streams
        # and memory would be foreign to the library's
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; "
                "g.build()' or python paper_2303_02210_amd/build.py)")
        lib_ = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(lib_, name)
            fn.restype = res
            fn.argtypes = args
        check_source(lib_)
        _lib = lib_
    return _lib


def built_source_hash(lib_=None) -> str:
    """The source hash a library reports in lbm_version() (its last word)."""
    v = (lib_ or lib()).lbm_version().decode()
    return v.rsplit(" ", 1)[-1]


def check_source(lib_) -> None:
    """Refuse a library built from other sources than the ones in this tree
    (a stale build would otherwise run silently)."""
    from .build import source_hash
    got, want = built_source_hash(lib_), source_hash()
    if got != want:
        raise ImportError(
            f"{LIB_PATH} was built from sources with hash {got}, but the sources in this "
            f"tree hash to {want}: rebuild it (python paper_2303_02210_amd/build.py)")


def make_params(cfg: dict) -> Params:
    """Fill the C parameter block from a workload dict."""
    p = Params()
    p.abi_version = ABI_VERSION
    p.struct_size = ctypes.sizeof(Params)
    p.L = int(cfg["L"])
    p.H = int(cfg["H"])
    p.precision = PRECISION[cfg.get("precision", "fp64")]
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
    p.rho_ref = float(cfg.get("rho_ref", cfg.get("rho_init", 1.0)))
    p.seed = int(cfg.get("seed", 0)) & 0xFFFFFFFF
    p.replica = int(cfg.get("replica", 0)) & 0xFFFFFFFF
    p.flags = (FLAG_WINDOW if cfg.get("window", False) else 0) | \
        (FLAG_DIVISION_MAP if cfg.get("division_map", False) else 0) | \
        (FLAG_STOCHASTIC_ROUND if cfg.get("stochastic_round", False) else 0) | \
        (FLAG_BATCH_TABLE if cfg.get("batch_table", False) else 0) | \
        (FLAG_BATCH_OWN if cfg.get("batch_own", False) else 0)
    p.kernel_vb = int(cfg.get("kernel_vb", 0))
    p.kernel_ty = int(cfg.get("kernel_ty", 0))
    p.rho_cell = float(cfg.get("rho_cell", 0.1))
    p.rho0 = float(cfg.get("rho0", 1.5))
    p.lattice = LATTICE[cfg.get("lattice", "d2q9")]
    p.kernel_order = int(cfg.get("kernel_order", 0))
    return p


class LbmError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        self.code = code
        super().__init__(f"{where}: {ERROR_NAMES.get(code, code)}"
                         + (f" ({detail})" if detail else ""))
