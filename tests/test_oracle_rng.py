"""Pins of the oracle's counter-based generator (replaces the paper's
parallel Mersenne Twister, sect. 3.4; the paper asks for tested generators,
sect. 3.5)."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand(orc):
    rng = np.random.default_rng(123)
    cases = rng.integers(0, 2**32, size=(64, 6), dtype=np.uint64).tolist()
    cases += [[0, 0, 0, 0, 0, 0], [2**32 - 1] * 6, [1, 2, 3, 4, 5, 6]]
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "probe")
        subprocess.check_call(["hipcc", "-O1", "-o", exe, os.path.join(HERE, "philox_probe.cpp")],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        inp = "\n".join(" ".join(str(int(v)) for v in c) for c in cases) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [list(map(int, l.split())) for l in out.strip().splitlines()]
    got = [orc.philox(c[:4], c[4:]) for c in cases]
    assert got == ref


def test_u24_open_interval_and_exact(orc):
    for x in [0, 255, 256, 2**32 - 1, 2**31, 12345678]:
        u = orc.u24(x)
        assert 0.0 < u < 1.0
        assert u == ((x >> 8) + 0.5) / 2**24  # exact in FP64 (25 significant bits)
    # 25 bits do not fit FP32: the walk in FP32 draws these uniforms in FP64
    u = orc.u24(2**32 - 1)
    assert float(np.float32(u)) != u and float(np.float32(orc.u24(2**16))) == orc.u24(2**16)
    assert orc.u24(0) == 0.5 / 2**24
    assert orc.u24(2**32 - 1) == 1.0 - 0.5 / 2**24


def test_draw_layout_matches_blocks(orc):
    seed, pid, it, model, tag = 0x1234_5678_9ABC, 0x0000_BEEF_0000_0042, 3, 7, 0
    for d in range(0, 13):
        ctr = [d >> 2, pid & 0xFFFFFFFF, ((pid >> 32) & 0xFFFF) | (it << 16), (model << 8) | tag]
        key = [seed & 0xFFFFFFFF, seed >> 32]
        blk = orc.philox(ctr, key)
        assert orc.draw(seed, pid, it, model, tag, d) == orc.u24(blk[d & 3])


def test_uniformity_and_stream_independence(orc):
    n = 20000
    u = np.array([orc.draw(7, p, 0, 0, 0, 0) for p in range(n)])
    v = np.array([orc.draw(7, p, 0, 0, 0, 1) for p in range(n)])
    w = np.array([orc.draw(7, p, 1, 0, 0, 0) for p in range(n)])  # next iteration
    for a in (u, v, w):
        assert stats.kstest(a, "uniform").pvalue > 1e-4
    hist, _ = np.histogram(u, bins=50, range=(0, 1))
    assert stats.chisquare(hist).pvalue > 1e-4
    for a, b in ((u, v), (u, w)):
        assert abs(np.corrcoef(a, b)[0, 1]) < 5.0 / np.sqrt(n)
