"""Dispatch orders (kernel_order 1-4): the order in which a step's row strips
are handed to the GPU changes nothing in the results.  Every order must
visit every tile of the lattice exactly once, including the strips past the
last whole group of eight (one per XCD) and, for the two-sweep order, an odd
number of groups; so each case's height leaves a ragged tail and an odd
group count.  Each order is compared bit for bit with order 1 (from the wall
up), which the parity tests pin to the oracle."""
import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu


def _run(cfg, steps):
    from paper_2303_02210_amd import Sim
    s = Sim(cfg)
    s.step(steps)
    out = (s.populations(), s.front_heights(), s.diagnostics())
    s.close()
    return out


# (tag, cfg): strips gy = H / ty with gy % 8 != 0 and gy // 8 odd
CASES = [
    ("fp32 vector, 1 row", si.cfg(L=512, H=107, init_rows=40, growth_rate=2e-3, sigma=1e-3,
                                  precision="fp32", seed=11)),
    ("fp16 vector, 2 rows", si.cfg(L=1024, H=154, init_rows=60, growth_rate=2e-3, sigma=1e-3,
                                   precision="fp16", seed=12)),
    ("fp16 one column, 4 rows", si.cfg(L=300, H=172, init_rows=50, tau=0.8, growth_rate=1e-3,
                                       sigma=1e-3, region="front_band", region_width=8,
                                       precision="fp16", kernel_vb=1, kernel_ty=4, seed=13)),
    ("bf16 vector, stochastic rounding", si.cfg(L=512, H=154, init_rows=60, growth_rate=2e-3,
                                                sigma=1e-3, precision="bf16",
                                                stochastic_round=True, seed=14)),
    ("fp64 vector", si.cfg(L=256, H=95, init_rows=30, growth_rate=2e-3, sigma=1e-3,
                           precision="fp64", seed=15)),
    ("fp32 staged", si.cfg(L=256, H=800, init_rows=100, growth_rate=2e-3, sigma=1e-3,
                           precision="fp32", kernel_vb=2, seed=16)),
    ("d2q7 fp32", si.cfg(L=512, H=114, init_rows=40, growth_rate=2e-3, sigma=1e-3,
                         precision="fp32", lattice="d2q7", seed=17)),
    ("fp32 uniform divisions", si.cfg(L=256, H=101, init_rows=40, growth="division",
                                      growth_rate=2e-3, sigma=1e-3, precision="fp32", seed=18)),
    ("fp32 follow wall, window", si.cfg(L=256, H=131, init_rows=100, growth_rate=1e-2, sigma=1e-2,
                                        ybc="follow", wall_min_gap=10, window=True,
                                        precision="fp32", seed=19)),
]


@pytest.mark.parametrize("tag,cfg", CASES, ids=[c[0] for c in CASES])
def test_every_dispatch_order_gives_the_same_result(tag, cfg):
    steps = 25
    f1, h1, d1 = _run(dict(cfg, kernel_order=1), steps)
    for order in (2, 3, 4, 0):
        f, h, d = _run(dict(cfg, kernel_order=order), steps)
        assert np.array_equal(f, f1), (tag, order)
        assert np.array_equal(h, h1), (tag, order)
        for k in ("step", "y_wall", "h_hi", "status", "divisions", "rows_swept", "mass",
                  "src_total", "fix_total", "retired", "hbar", "W"):
            assert d[k] == d1[k], (tag, order, k, d[k], d1[k])
