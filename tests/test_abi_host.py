"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every entry point include/lbmgrow.h declares, lays out its structs as the
header does, and validates parameters before touching the device."""
import ctypes
import os
import re
import subprocess

import pytest

import synth_inputs as si
from paper_2303_02210_amd import _ffi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbmgrow.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _ffi.lib()
    declared = _declared_functions()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(_ffi.ENTRY_POINTS) == declared
    out = subprocess.run(["nm", "-D", "--defined-only", _ffi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (lbm_[a-z_0-9]+)", out))
    assert set(declared) <= exported


def test_struct_layout_matches_header(tmp_path):
    # compile a probe against the header and compare every offset with ctypes
    fields = [f for f, _ in _ffi.Params._fields_]
    dfields = [f for f, _ in _ffi.Diag._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbmgrow.h"', 'int main(void){',
           'printf("%zu %zu\\n", sizeof(lbm_params), sizeof(lbm_diag));']
    for f in fields:
        src.append(f'printf("P {f} %zu\\n", offsetof(lbm_params, {f}));')
    for f in dfields:
        src.append(f'printf("D {f} %zu\\n", offsetof(lbm_diag, {f}));')
    src.append("return 0;}")
    c = tmp_path / "probe.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    sp, sd = (int(v) for v in lines[0].split())
    assert sp == ctypes.sizeof(_ffi.Params) and sd == ctypes.sizeof(_ffi.Diag)
    for line in lines[1:]:
        if not line:
            continue
        kind, name, off = line.split()
        cls = _ffi.Params if kind == "P" else _ffi.Diag
        assert getattr(cls, name).offset == int(off), name


def test_version_string():
    assert b"gfx950" in _ffi.lib().lbm_version()


def _ws(cfg):
    p = _ffi.make_params(cfg)
    return int(_ffi.lib().lbm_workspace_bytes(ctypes.byref(p)))


def test_workspace_bytes_scales_with_precision():
    base = dict(si.BULK_4096_FP32)
    n = {pr: _ws(dict(base, precision=pr)) for pr in ("fp64", "fp32", "fp16", "bf16")}
    pops = 2 * 9 * 4096 * 4096
    for pr, b in (("fp64", 8), ("fp32", 4), ("fp16", 2), ("bf16", 2)):
        assert pops * b <= n[pr] < pops * b + 4 * 2 ** 20
    assert n["fp16"] == n["bf16"]


@pytest.mark.parametrize("bad", [
    dict(tau=0.5), dict(tau=float("nan")), dict(rho_c=0.0), dict(L=1), dict(H=3),
    dict(sigma=-1.0), dict(growth_rate=-1e-3), dict(init_rows=65), dict(mu=1.5),
    dict(init_amp=1.0), dict(region_width=-1), dict(precision="fp64", window=True, ybc="periodic"),
    dict(growth="division", rho_cell=0.0), dict(growth="division_density", rho_cell=float("inf")),
    dict(growth="division_density", rho0=0.5), dict(growth="division_density", rho0=0.4),
    dict(lattice="d2q7", kernel_vb=2),
    dict(lattice="d2q7", ybc="periodic", H=63, init_rows=10),
    dict(precision="fp32", stochastic_round=True), dict(precision="fp64", stochastic_round=True),
    dict(precision="fp16", stochastic_round=True, kernel_vb=2),
])
def test_invalid_parameters_rejected_on_host(bad):
    c = dict(si.SMALL_FP64)
    c.update(bad)
    assert _ws(c) == 0
    p = _ffi.make_params(c)
    h = ctypes.c_void_p()
    rc = _ffi.lib().lbm_create(ctypes.byref(p), ctypes.c_void_p(256), 1 << 30, None, ctypes.byref(h))
    assert rc == _ffi.E_INVALID and not h.value


@pytest.mark.parametrize("lattice,q", [("d2q9", 9), ("d2q7", 7)])
def test_size_limits(lattice, q):
    """L * H * Q <= 2^31 populations and L <= 2^24: the largest lattice is
    accepted, one row more is not, and the workspace holds both buffers."""
    L = 16384
    H = (1 << 31) // (q * L)
    c = dict(si.SMALL_FP64, lattice=lattice, L=L, H=H, init_rows=8, precision="fp32")
    n = _ws(c)
    assert n >= 2 * q * L * H * 4
    assert _ws(dict(c, H=H + 1)) == 0
    assert _ws(dict(c, L=1 << 24, H=4, init_rows=2)) > 0
    assert _ws(dict(c, L=(1 << 24) + 64, H=4, init_rows=2)) == 0


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("lattice", ["d2q9", "d2q7"])
def test_stochastic_rounding_accepted_for_16_bit_storage(prec, lattice):
    c = dict(si.SMALL_FP64, precision=prec, lattice=lattice)
    assert _ws(dict(c, stochastic_round=True)) == _ws(c) > 0


def test_d2q7_workspace_holds_seven_populations():
    base = dict(si.BULK_4096_FP32)
    n9 = _ws(base)
    n7 = _ws(dict(base, lattice="d2q7"))
    pops = 2 * 4096 * 4096 * 4
    assert n9 - n7 >= 2 * pops and n7 >= 7 * pops


def test_abi_version_and_size_checked():
    p = _ffi.make_params(si.SMALL_FP64)
    p.abi_version = 99
    assert _ffi.lib().lbm_workspace_bytes(ctypes.byref(p)) == 0
    p = _ffi.make_params(si.SMALL_FP64)
    p.struct_size = 8
    assert _ffi.lib().lbm_workspace_bytes(ctypes.byref(p)) == 0


def test_create_rejects_bad_workspace_before_device_work():
    p = _ffi.make_params(si.SMALL_FP64)
    n = _ffi.lib().lbm_workspace_bytes(ctypes.byref(p))
    h = ctypes.c_void_p()
    L = _ffi.lib()
    assert L.lbm_create(ctypes.byref(p), None, n, None, ctypes.byref(h)) == _ffi.E_INVALID
    assert L.lbm_create(ctypes.byref(p), ctypes.c_void_p(4096 + 8), n, None,
                        ctypes.byref(h)) == _ffi.E_INVALID          # not 256-byte aligned
    assert L.lbm_create(ctypes.byref(p), ctypes.c_void_p(4096), n - 1, None,
                        ctypes.byref(h)) == _ffi.E_NOMEM
    assert L.lbm_step(None, 1) == _ffi.E_INVALID
    assert L.lbm_destroy(None) == _ffi.E_INVALID


def test_autotune_keys_and_candidates_for_stochastic_rounding(monkeypatch):
    from paper_2303_02210_amd import autotune
    c = dict(si.BULK_4096_FP32, precision="fp16")
    sr = dict(c, stochastic_round=True)
    assert autotune.key(sr) == autotune.key(c) + "/sr"
    assert any(s["kernel_vb"] == 2 for s in autotune.candidates(c))
    assert not any(s["kernel_vb"] == 2 for s in autotune.candidates(sr))
    # no key of its own: the nearest-rounding shape, unless it is the staged form
    monkeypatch.setattr(autotune, "cache", lambda: {autotune.key(c): {"kernel_vb": 4, "kernel_ty": 2}})
    assert autotune.apply(sr)["kernel_vb"] == 4
    monkeypatch.setattr(autotune, "cache", lambda: {autotune.key(c): {"kernel_vb": 2, "kernel_ty": 32}})
    assert "kernel_vb" not in autotune.apply(sr)


def test_autotune_key_separates_front_band_growth():
    """The edge strip (growth in a band at the front) and a bulk-grown lattice
    of the same size have different best shapes, so their keys differ; the
    shipped table holds an entry for each standard workload."""
    from paper_2303_02210_amd import autotune
    edge = dict(si.EDGE_2048x8192, precision="fp32")
    bulk = dict(edge, region="all")
    assert autotune.key(edge) == autotune.key(bulk) + "/band"
    assert autotune.key(dict(edge, precision="fp16", stochastic_round=True)).endswith("/band/sr")
    shipped = autotune._load(autotune.SHIPPED)
    for p in ("fp32", "fp16", "bf16"):
        assert autotune.key(dict(edge, precision=p)) in shipped, p
    for p in ("fp16", "bf16"):
        assert autotune.key(dict(edge, precision=p, stochastic_round=True)) in shipped, p
    for c in si.ensemble():
        assert autotune.key(c) in shipped, c["L"]
