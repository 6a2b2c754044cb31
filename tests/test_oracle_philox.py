"""The oracle's Philox4x32-10 (Salmon et al., SC'11) against rocRAND's
independent implementation of the same generator, compiled here for the host,
and statistical checks of the 24-bit uniforms the method draws from it."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as orc

_HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_pin(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("philox") / "pin")
    subprocess.run([hipcc, "-O1", os.path.join(_HERE, "philox_rocrand_pin.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(rocrand_pin):
    rng = np.random.default_rng(11)
    rows = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF, 0xFFFFFFFF, 0x3FFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF]]
    for _ in range(300):
        k0, k1, c0, c2, c3 = (int(v) for v in rng.integers(0, 2 ** 32, 5))
        c1 = int(rng.integers(0, 2 ** 30))      # the engine's offset is 4 * (c0 | c1 << 32)
        rows.append([k0, k1, c0, c1, c2, c3])
    text = "\n".join(" ".join("%x" % v for v in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_pin], input=text, capture_output=True, text=True, check=True)
    got = [[int(w, 16) for w in line.split()] for line in out.stdout.strip().splitlines()]
    assert len(got) == len(rows)
    for r, g in zip(rows, got):
        mine = orc.philox4x32_10(r[2:], r[:2]).tolist()
        assert mine == g, (r, mine, g)


def test_noise_bits_layout():
    # words 0-7: the top 24 bits of the two Philox blocks (calls 0 and 1 of
    # the noise stream); word 8: the low bytes of block 0 words 0, 1, 2
    seed, rep, t, x, y = 7, 3, 12345, 17, 901
    a = orc.philox4x32_10([x, y, t, 0], [seed, rep])
    b = orc.philox4x32_10([x, y, t, 1], [seed, rep])
    k = orc.noise_bits(seed, rep, t, x, y)
    assert k[:4].tolist() == (a >> 8).tolist()
    assert k[4:8].tolist() == (b >> 8).tolist()
    assert int(k[8]) == ((int(a[0]) & 0xFF) << 16) | ((int(a[1]) & 0xFF) << 8) | (int(a[2]) & 0xFF)
    u = orc.noise_uniforms(seed, rep, t, x, y)
    assert np.array_equal(u, (k.astype(np.float64) + 0.5) / 2.0 ** 24)


def test_init_uniform_stream():
    # the initial density uses the counter's fourth word 4 (stream 1, call 0), t = 0
    r = orc.philox4x32_10([5, 9, 0, 4], [1, 2])
    assert orc.init_uniform(1, 2, 5, 9) == ((int(r[0]) >> 8) + 0.5) / 2.0 ** 24


def test_noise_factor_exact_in_float32():
    rng = np.random.default_rng(12)
    for t, x, y in rng.integers(0, 10 ** 6, (200, 3)):
        u = orc.noise_uniforms(0, 0, int(t), int(x), int(y))
        # u = (2k + 1) 2^-25 needs 25 bits, but the factor multiplying sigma,
        # 2u - 1 = (2k + 1 - 2^24) 2^-24, fits a float32 significand exactly
        v = 2.0 * u - 1.0
        assert np.array_equal(v.astype(np.float32).astype(np.float64), v)
