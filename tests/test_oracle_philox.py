"""Pins for the oracle's Philox4x32-10 (Salmon et al., SC'11)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat_rows(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "philox_kat.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([int(t, 16) for t in line.split()])
    return rows


def test_published_known_answers(golden_dir):
    rows = _kat_rows(golden_dir)
    assert len(rows) == 3
    for r in rows:
        out = philox.philox4x32_10(*r[:6])
        assert [int(v) for v in out] == r[6:10]


@pytest.fixture(scope="module")
def rocrand_kat(tmp_path_factory):
    cxx = shutil.which("g++")
    inc = "/opt/rocm/include"
    if cxx is None or not os.path.exists(os.path.join(inc, "rocrand", "rocrand_philox4x32_10.h")):
        pytest.skip("rocRAND headers or g++ not available")
    exe = str(tmp_path_factory.mktemp("kat") / "kat")
    subprocess.run([cxx, "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", inc,
                    os.path.join(HERE, "rocrand_philox_kat.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def test_matches_rocrand_engine(rocrand_kat):
    rng = np.random.Generator(np.random.PCG64(123))
    n = 2000
    c = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64)
    c[:, 1] &= (1 << 30) - 1
    k = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64)
    k[:10] = 0
    c[:10] = np.arange(10)[:, None]
    lines = "\n".join(" ".join("%08x" % int(v) for v in (*c[i], *k[i])) for i in range(n))
    out = subprocess.run([rocrand_kat], input=lines, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for i in range(n):
        ref = [int(t, 16) for t in out[i].split()]
        got = philox.philox4x32_10(*c[i], *k[i])
        assert [int(v) for v in got] == ref, i


def test_vectorised_equals_elementwise():
    blocks = np.arange(37, dtype=np.int64)
    w = philox.draw(0x1234_5678_9ABC_DEF0, philox.XO, 7, 3, blocks)
    for b in (0, 5, 36):
        one = philox.draw(0x1234_5678_9ABC_DEF0, philox.XO, 7, 3, b)
        assert np.array_equal(w[b], one)


def test_streams_differ_by_every_counter_field():
    base = philox.draw(5, philox.SEL, 1, 2, 3)
    for other in (philox.draw(6, philox.SEL, 1, 2, 3), philox.draw(5, philox.XO, 1, 2, 3),
                  philox.draw(5, philox.SEL, 2, 2, 3), philox.draw(5, philox.SEL, 1, 3, 3),
                  philox.draw(5, philox.SEL, 1, 2, 4), philox.draw(5, philox.SEL, 1, 2, 3, run=1)):
        assert not np.array_equal(base, other)


def test_output_bits_uniform():
    w = philox.draw(9, philox.BATCH, 0, 0, np.arange(1 << 16)).reshape(-1)
    bits = ((w[:, None] >> np.arange(32, dtype=np.uint32)) & 1).astype(np.float64)
    frac = bits.mean(axis=0)
    n = w.size
    assert np.all(np.abs(frac - 0.5) < 5 * 0.5 / np.sqrt(n))
    hist = np.bincount((w >> 24).astype(np.int64), minlength=256)
    from scipy.stats import chisquare
    assert chisquare(hist).pvalue > 1e-4
