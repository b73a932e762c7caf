"""Float32 Box-Muller normal sampler (oracle side), evaluated op by op.

Gaussian mutation (paper section 3.2, the mutation operator) adds sigma times
a standard normal draw to each gene.  The paper names no sampler.  Because
mutated genes must match the device bit for bit, the sampler is defined here
entirely in terms of IEEE float32 operations that are correctly rounded on
every conforming machine (+, -, *, /, sqrt, exact int->float conversions),
evaluated in a fixed order with no fused multiply-add:

Box-Muller (Box & Muller 1958): for two independent 32-bit words (a, b)

    u1    = ((a >> 8) + 1) * 2**-24                  in (0, 1]
    r     = sqrt(-2 * ln32(u1))
    q     = b >> 30                                  quadrant 0..3
    fi    = (b >> 6) & 0xFFFFFF;  f = fi * 2**-24    in [0, 1)
    angle = (q + f) * pi/2
    z0    = r * cos(angle),  z1 = r * sin(angle)

sin/cos of f*pi/2 are taken on [0, pi/4] by symmetry: if f >= 1/2 the
complementary fraction g = 1 - f (exact) is used and the results swapped.

ln32(u): u = m * 2**e with m in (sqrt(1/2), sqrt(2)] (exact split of the
float's exponent and mantissa), s = (m - 1)/(m + 1), and
ln m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ... + s^11/11); then
ln u = e*LN2_HI + (e*LN2_LO + ln m) with a two-part ln 2 whose high part
has 16 significant bits so that e*LN2_HI is exact (Cody & Waite).

sin / cos on [0, pi/4]: Taylor series to x^11 and x^12.

Every coefficient is the float32 nearest to the exact real value (computed
here from exact rationals, and from 50-digit decimal expansions of pi, ln 2
and sqrt 2).

Pins: accuracy of ln32 / sin / cos against float64 libm over their whole
input domains (2**24 points each), exact special values, and the distribution
of the resulting normals (moments, Kolmogorov-Smirnov).
"""

from fractions import Fraction
from math import factorial

import numpy as np

F32 = np.float32

# 50-digit expansions of the irrational constants used below
_PI = Fraction("3.14159265358979323846264338327950288419716939937510")
_LN2 = Fraction("0.69314718055994530941723212145817656807550013436026")
_SQRT2 = Fraction("1.41421356237309504880168872420969807856967187537694")


def f32_nearest(q):
    """The float32 nearest to the exact rational ``q`` (ties to even)."""
    q = Fraction(q)
    d = F32(float(q))
    cands = [np.nextafter(d, F32(-np.inf)), d, np.nextafter(d, F32(np.inf))]
    best = None
    for c in cands:
        err = abs(Fraction(float(c)) - q)
        even = (int(np.array(c, dtype=F32).view(np.uint32)) & 1) == 0
        key = (err, not even)
        if best is None or key < best[0]:
            best = (key, c)
    return F32(best[1])


PIO2 = f32_nearest(_PI / 2)
SQRT2 = f32_nearest(_SQRT2)
LN2_HI = F32(float(Fraction(int(_LN2 * 2**16), 2**16)))   # 16 significant bits
LN2_LO = f32_nearest(_LN2 - Fraction(float(LN2_HI)))
# atanh series 1/3, 1/5, ..., 1/11
LN_C = {k: f32_nearest(Fraction(1, k)) for k in (3, 5, 7, 9, 11)}
# Taylor coefficients (-1)^n/(2n+1)! for sin and (-1)^n/(2n)! for cos
SIN_C = {2 * n + 1: f32_nearest(Fraction((-1) ** n, factorial(2 * n + 1)))
         for n in range(1, 6)}                     # x^3 .. x^11
COS_C = {2 * n: f32_nearest(Fraction((-1) ** n, factorial(2 * n)))
         for n in range(1, 7)}                     # x^2 .. x^12
TWO_M24 = F32(2.0 ** -24)
INV_LN2 = f32_nearest(1 / _LN2)
# Taylor coefficients 1/n! for exp, n = 2..7
EXP_C = {n: f32_nearest(Fraction(1, factorial(n))) for n in range(2, 8)}


def ln32(u):
    """Natural log of float32 ``u`` in (0, 1] (normal numbers), float32 ops."""
    u = np.asarray(u, dtype=F32)
    bits = u.view(np.uint32)
    e = (bits >> np.uint32(23)).astype(np.int32) - np.int32(127)
    m = ((bits & np.uint32(0x7FFFFF)) | np.uint32(0x3F800000)).view(F32)
    big = m > SQRT2
    m = np.where(big, m * F32(0.5), m).astype(F32)
    e = np.where(big, e + np.int32(1), e)
    f = m - F32(1.0)
    t = m + F32(1.0)
    s = f / t
    z = s * s
    p = LN_C[11]
    for k in (9, 7, 5, 3):
        p = p * z
        p = p + LN_C[k]
    sz = s * z
    szp = sz * p
    h = s + szp
    lnm = F32(2.0) * h
    ef = e.astype(F32)
    hi = ef * LN2_HI
    lo = ef * LN2_LO
    lo = lo + lnm
    return (hi + lo).astype(F32)


def sincos_quarter(x):
    """(sin x, cos x) for float32 ``x`` in [0, pi/4], float32 ops."""
    x = np.asarray(x, dtype=F32)
    z = x * x
    ps = SIN_C[11]
    for k in (9, 7, 5, 3):
        ps = ps * z
        ps = ps + SIN_C[k]
    xz = x * z
    s = x + xz * ps
    pc = COS_C[12]
    for k in (10, 8, 6, 4, 2):
        pc = pc * z
        pc = pc + COS_C[k]
    c = F32(1.0) + z * pc
    return s.astype(F32), c.astype(F32)


def sincos_turn(b):
    """(cos, sin) of the angle (q + f) * pi/2 encoded by 32-bit word ``b``."""
    b = np.asarray(b, dtype=np.uint32)
    q = b >> np.uint32(30)
    fi = (b >> np.uint32(6)) & np.uint32(0xFFFFFF)
    swap = fi >= np.uint32(1 << 23)
    f = fi.astype(F32) * TWO_M24
    g = np.where(swap, F32(1.0) - f, f).astype(F32)
    x = g * PIO2
    s0, c0 = sincos_quarter(x)
    s = np.where(swap, c0, s0)
    c = np.where(swap, s0, c0)
    # rotate by q quarter turns: cos(a + q pi/2), sin(a + q pi/2)
    cq = np.select([q == 0, q == 1, q == 2], [c, -s, -c], s)
    sq = np.select([q == 0, q == 1, q == 2], [s, c, -s], -c)
    return cq.astype(F32), sq.astype(F32)


def normal_pair(a, b):
    """Two standard normal float32 draws from uint32 words ``a`` and ``b``."""
    a = np.asarray(a, dtype=np.uint32)
    u1 = ((a >> np.uint32(8)) + np.uint32(1)).astype(F32) * TWO_M24
    lg = ln32(u1)
    r = np.sqrt(F32(-2.0) * lg)
    c, s = sincos_turn(b)
    return (r * c).astype(F32), (r * s).astype(F32)


def normals4(words):
    """Four normals from a Philox output block ``words[..., 0:4]``.

    Normals 0,1 come from the pair (w0, w1); normals 2,3 from (w2, w3).
    """
    words = np.asarray(words, dtype=np.uint32)
    z0, z1 = normal_pair(words[..., 0], words[..., 1])
    z2, z3 = normal_pair(words[..., 2], words[..., 3])
    return np.stack([z0, z1, z2, z3], axis=-1)


def exp32(x):
    """e**x for float32 ``x`` with |x| <= 80, float32 ops (self-adaptive sigma).

    n = rint(x / ln 2) (ties to even), r = (x - n*LN2_HI) - n*LN2_LO (the same
    two-part ln 2 as ln32, n*LN2_HI exact), e**r by its Taylor series to r^7
    (|r| <= 0.35), then an exact scaling by 2**n built from the exponent bits.
    """
    x = np.asarray(x, dtype=F32)
    if np.any(np.abs(x) > F32(80.0)):
        raise ValueError("exp32 domain is |x| <= 80")
    t = x * INV_LN2
    n = np.rint(t).astype(F32)
    hi = n * LN2_HI
    r = x - hi
    lo = n * LN2_LO
    r = r - lo
    p = EXP_C[7]
    for k in (6, 5, 4, 3, 2):
        p = p * r
        p = p + EXP_C[k]
    p = p * r
    p = p + F32(1.0)
    p = p * r
    p = p + F32(1.0)
    scale = ((n.astype(np.int32) + np.int32(127)).astype(np.uint32) << np.uint32(23)).view(F32)
    return (p * scale).astype(F32)
