"""lbm_create_static, the entry point for callers that cannot allocate: a
simulation whose scratch (front heights, tallies, device state, diagnostics)
lives in the library's static device array comes out bit for bit as the same
simulation created with lbm_create over a caller workspace, for two calls in
a row on one device (the second on a smaller lattice, which reuses the array
the first one left behind), in every storage type and with the sweep window,
the wall following the front and a division law (the scratch-heavy paths)."""
import ctypes

import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu


def _run(cfg, steps, static):
    from paper_2303_02210_amd import Sim
    s = Sim(cfg, static_scratch=static)
    s.step(steps)
    out = (s.populations(), s.front_heights(), s.diagnostics(), s.get_state())
    s.close()
    return out


def _same(a, b, tag):
    fa, ha, da, _ = a
    fb, hb, db, _ = b
    assert np.array_equal(fa, fb), tag
    assert np.array_equal(ha, hb), tag
    for k, v in da.items():
        assert v == db[k], (tag, k, v, db[k])


CASES = [
    (si.cfg(L=256, H=192, init_rows=60, tau=0.8, sigma=1e-3, growth_rate=2e-3, precision="fp32",
            seed=3),
     si.cfg(L=96, H=64, init_rows=20, sigma=1e-3, growth_rate=2e-3, precision="fp64", seed=4)),
    (si.cfg(L=200, H=160, init_rows=90, sigma=1e-2, growth="division", growth_rate=1e-2,
            ybc="follow", wall_min_gap=10, window=True, precision="fp16", seed=5),
     si.cfg(L=72, H=96, init_rows=40, sigma=1e-2, growth="division_density", growth_rate=1e-2,
            region="front_band", region_width=6, precision="bf16", seed=6)),
    (si.cfg(L=128, H=128, init_rows=40, lattice="d2q7", sigma=1e-3, growth_rate=3e-3,
            window=True, division_map=True, precision="fp64", seed=7),
     si.cfg(L=64, H=32, init_rows=10, sigma=1e-3, growth_rate=3e-3, precision="fp32", seed=8)),
]


@pytest.mark.parametrize("pair", range(len(CASES)))
def test_static_scratch_matches_the_workspace_entry_point(pair):
    first, second = CASES[pair]
    assert first["L"] * first["H"] > second["L"] * second["H"]
    for n, cfg in enumerate((first, second)):      # two calls in a row, the second smaller
        ref = _run(cfg, 37, static=False)
        got = _run(cfg, 37, static=True)
        _same(got, ref, (pair, n))
        assert got[2]["step"] == 37 and got[2]["status"] == 0


def test_one_live_static_handle_per_device_and_size_limit():
    from paper_2303_02210_amd import LbmError, Sim, _ffi
    cfg = si.cfg(L=64, H=64, init_rows=16, growth_rate=1e-3)
    a = Sim(cfg, static_scratch=True)
    with pytest.raises(LbmError, match="NOMEM"):
        Sim(cfg, static_scratch=True)
    a.step(3)
    a.close()
    b = Sim(cfg, static_scratch=True)            # the array is free again
    b.step(3)
    b.close()
    # a lattice whose scratch exceeds the static array is refused up front
    big = si.cfg(L=4096, H=4096, init_rows=16, division_map=True)
    p = _ffi.make_params(big)
    size = ctypes.c_size_t(0)
    assert _ffi.lib().lbm_create_static(ctypes.byref(p), None, ctypes.byref(size), None,
                                        None) == _ffi.E_NOMEM
    # and the size query reports the two population buffers
    p = _ffi.make_params(cfg)
    assert _ffi.lib().lbm_create_static(ctypes.byref(p), None, ctypes.byref(size), None,
                                        None) == 0
    assert size.value >= 2 * 9 * 64 * 64 * 8
