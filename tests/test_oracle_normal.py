"""Pins for the oracle's float32 Box-Muller sampler against float64 libm,
exact special values and the normal distribution."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from oracle import normal32 as n32
from oracle import philox

F32 = np.float32


def _ulp_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ulp = np.spacing(np.abs(ref).astype(F32)).astype(np.float64)
    return np.abs(got - ref) / ulp


def test_constants_are_nearest_float32():
    for val, exact in ((n32.PIO2, math.pi / 2), (n32.SQRT2, math.sqrt(2.0))):
        lo, hi = np.nextafter(val, F32(0)), np.nextafter(val, F32(10))
        assert abs(float(val) - exact) <= abs(float(lo) - exact)
        assert abs(float(val) - exact) <= abs(float(hi) - exact)
    # two-part ln 2: high part has <= 16 significant bits, sum is ln 2
    assert float(n32.LN2_HI) * 2**16 == int(float(n32.LN2_HI) * 2**16)
    assert abs(float(n32.LN2_HI) + float(n32.LN2_LO) - math.log(2.0)) < 1e-13
    for k, c in n32.LN_C.items():
        assert abs(float(c) - 1.0 / k) <= 0.5 * float(np.spacing(c))
    for k, c in n32.SIN_C.items():
        assert abs(float(c) - (-1) ** ((k - 1) // 2) / math.factorial(k)) <= 0.5 * abs(float(np.spacing(c)))
    for k, c in n32.COS_C.items():
        assert abs(float(c) - (-1) ** (k // 2) / math.factorial(k)) <= 0.5 * abs(float(np.spacing(c)))


def test_f32_nearest_ties_and_exact():
    assert n32.f32_nearest(Fraction(1, 2)) == F32(0.5)
    # 1 + 2^-24 is exactly halfway between 1 and 1 + 2^-23: ties to even -> 1
    assert n32.f32_nearest(1 + Fraction(1, 2**24)) == F32(1.0)
    assert n32.f32_nearest(1 + Fraction(3, 2**24)) == F32(1.0) + F32(2.0**-22)


@pytest.mark.slow
def test_ln32_whole_domain_within_2ulp():
    k = np.arange(1, 2**24 + 1, dtype=np.uint32)
    u = k.astype(F32) * F32(2.0**-24)
    got = n32.ln32(u)
    ref = np.log(u.astype(np.float64))
    nz = ref != 0
    assert np.all(_ulp_err(got[nz], ref[nz]) <= 2.0)
    assert got[-1] == 0.0 and not np.signbit(got[-1])


def test_ln32_special_values():
    for k in range(0, 25):
        u = F32(2.0 ** -k)
        got = float(n32.ln32(np.array([u]))[0])
        assert abs(got + k * math.log(2.0)) <= 1.0 * float(np.spacing(F32(k * math.log(2.0) + 1e-30)))
    u = np.array([0.75, 0.9, 0.5 + 2**-24, 1 - 2**-24], dtype=F32)
    assert np.all(_ulp_err(n32.ln32(u), np.log(u.astype(np.float64))) <= 2.0)


@pytest.mark.slow
def test_sincos_whole_domain():
    fi = np.arange(2**24, dtype=np.uint32)
    for q in range(4):
        b = (np.uint32(q) << np.uint32(30)) | (fi << np.uint32(6))
        c, s = n32.sincos_turn(b)
        ang = (q + fi.astype(np.float64) * 2.0**-24) * (math.pi / 2)
        assert np.max(np.abs(c - np.cos(ang))) < 1.2e-7
        assert np.max(np.abs(s - np.sin(ang))) < 1.2e-7


def test_sincos_exact_points():
    # angle 0 and quarter turns: cos/sin are exactly 0 or +-1
    for q, (cq, sq) in enumerate(((1, 0), (0, 1), (-1, 0), (0, -1))):
        c, s = n32.sincos_turn(np.array([q << 30], dtype=np.uint32))
        assert float(c[0]) == cq and float(s[0]) == sq
    # the low six bits are ignored
    c1, s1 = n32.sincos_turn(np.array([0x12345640], dtype=np.uint32))
    c2, s2 = n32.sincos_turn(np.array([0x1234567F], dtype=np.uint32))
    assert c1[0] == c2[0] and s1[0] == s2[0]


def test_box_muller_radius_and_angle():
    rng = np.random.Generator(np.random.PCG64(5))
    a = rng.integers(0, 2**32, size=100000, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 2**32, size=100000, dtype=np.uint64).astype(np.uint32)
    z0, z1 = n32.normal_pair(a, b)
    u1 = ((a >> 8).astype(np.float64) + 1) * 2.0**-24
    r2 = -2.0 * np.log(u1)
    np.testing.assert_allclose(z0.astype(np.float64)**2 + z1.astype(np.float64)**2, r2,
                               rtol=2e-6, atol=1e-6)
    ang = (b.astype(np.float64) // 64) * 2.0**-24 * (math.pi / 2)
    r = np.sqrt(r2)
    np.testing.assert_allclose(z0, r * np.cos(ang), atol=2e-6)
    np.testing.assert_allclose(z1, r * np.sin(ang), atol=2e-6)


def test_normals_are_standard_normal():
    w = philox.draw(11, philox.MUTNORM, 1, 0, np.arange(1 << 18))
    z = n32.normals4(w).reshape(-1).astype(np.float64)
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    for t in (3.0, 4.0):
        p = 2 * stats.norm.sf(t)
        tail = np.count_nonzero(np.abs(z) > t) / n
        assert abs(tail - p) < 6 * math.sqrt(p / n)
    # the four lanes of one block are uncorrelated
    zz = n32.normals4(w).astype(np.float64)
    cc = np.corrcoef(zz.T)
    assert np.all(np.abs(cc - np.eye(4)) < 6 / math.sqrt(zz.shape[0]))
