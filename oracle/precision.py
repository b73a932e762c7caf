"""Reduced-precision evaluation of the population (oracle side; test
infrastructure only).

The paper evaluates in float32.  The reduced-precision variants round the
weights of every layer and the network's input, the batch; the products
accumulate in float32 and the biases, the hidden activations and the
fitness (Eq. 1) stay float32 (float64 here):

* ``bf16``: the batch X and every weight matrix W_l are rounded to
  bfloat16 (8 significant bits, float32's exponent range; round to
  nearest, ties to even).  In the first layer both operands are bfloat16,
  so its products are exact in float32 and the layer is a sum of exact
  products: the device accumulates it in float32, the oracle in float64.
* ``fp8``: OCP FP8 E4M3 (1 sign, 4 exponent bits with bias 7, 3 mantissa
  bits; largest finite value 448, no infinities, subnormals down to 2^-9)
  with power-of-two scales, one per network and layer: W_l of each network
  is divided by 2^e_l and X by 2^e_x, rounded to E4M3 (nearest, ties to
  even), and each layer's sums are multiplied back by 2^(e_l + e_x) (the
  first layer) or 2^e_l (later layers).  e is the smallest integer with
  B <= 448 * 2^e for a bound B of the operand's largest magnitude, so no
  scaled value exceeds 448.  For the batch and for W_2 .. W_L, B is the
  largest magnitude.  For a network's W_1 it is its largest magnitude after
  initialisation or a restore, and for a child the bound its parents give
  (``fp8_child_bounds``), known before the child exists, so that the
  child's FP8 copy can be written as the child is made.  An operand holding
  NaN or an infinity (a non-finite bound) makes the fitness of the affected
  networks NaN.

The hidden activations are not rounded: they are float32 sums whose
summation order differs between any two implementations, and rounding them
to 8 or 3 significant bits would turn that last-bit difference into a
whole rounding step wherever a sum lies near a rounding midpoint.

Scaling by powers of two and products of these short significands are
exact in float64; beyond the quantisation itself the oracle rounds only in
its float64 sums.
"""

import math

import numpy as np

from . import leea as L

BF16 = "bf16"
FP8 = "fp8"
F32 = "f32"
E4M3_MAX = 448.0


def round_bf16(x):
    """Nearest bfloat16 value of each float32 element, ties to even; NaN and
    infinities are kept.  Dropping the low 16 bits of the float32 encoding
    with a round-half-even carry is exactly that rounding (the encoding is
    monotone in the magnitude and the carry may overflow into the exponent,
    which is the correct next binade or infinity)."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).copy()
    nan = np.isnan(a)
    out[nan] = np.nan
    return out


def e4m3_table():
    """The 127 non-negative finite E4M3 values, indexed by their 7-bit code
    (exponent field e, mantissa field m): m * 2^-9 for e = 0 (subnormal),
    (1 + m/8) * 2^(e-7) otherwise; code 127 (e = 15, m = 7) is NaN."""
    vals = []
    for code in range(127):
        e, m = code >> 3, code & 7
        vals.append(m * 2.0**-9 if e == 0 else (1.0 + m / 8.0) * 2.0**(e - 7))
    return np.array(vals, dtype=np.float64)


_E4M3 = e4m3_table()


def round_e4m3_codes(v):
    """E4M3 code (sign bit 7, magnitude code in bits 0..6) of the nearest
    value to each float64 element with |v| <= 448, ties to the even code
    (the one with an even mantissa).  NaN gives code 0x7F."""
    v = np.asarray(v, dtype=np.float64)
    a = np.abs(v)
    nan = np.isnan(v)
    if np.any(a[~nan] > E4M3_MAX):
        raise ValueError("value beyond the E4M3 range after scaling")
    a = np.where(nan, 0.0, a)
    hi = np.searchsorted(_E4M3, a, side="left")          # first table value >= a
    hi = np.minimum(hi, len(_E4M3) - 1)
    lo = np.maximum(hi - 1, 0)
    dlo = a - _E4M3[lo]
    dhi = _E4M3[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    code = np.where(pick_hi, hi, lo)
    code = np.where(a == _E4M3[hi], hi, code)
    sign = (np.signbit(v) & ~nan).astype(np.int64) << 7
    return np.where(nan, 0x7F, code | sign).astype(np.uint8)


def e4m3_value(codes):
    """float64 value of E4M3 codes (0x7F / 0xFF are NaN)."""
    c = np.asarray(codes, dtype=np.int64)
    mag = c & 0x7F
    val = np.where(mag == 0x7F, np.nan, _E4M3[np.minimum(mag, 126)])
    return np.where(c & 0x80, -val, val)


def round_e4m3(v):
    """Nearest E4M3 value (float64) of each element with |v| <= 448."""
    return e4m3_value(round_e4m3_codes(v))


def fp8_exponent(amax):
    """Smallest integer e with amax <= 448 * 2^e (0 for amax = 0).  amax is
    a non-negative finite number; every comparison is exact."""
    amax = float(amax)
    if not math.isfinite(amax) or amax < 0:
        raise ValueError("amax must be finite and non-negative")
    if amax == 0.0:
        return 0
    _, k = math.frexp(amax)                  # amax in [2^(k-1), 2^k)
    e = k - 9                                # 448 * 2^(k-9) < 2^k
    while amax > E4M3_MAX * 2.0**e:
        e += 1
    while amax <= E4M3_MAX * 2.0**(e - 1):
        e -= 1
    return e


MUT_BOUND_FACTOR = np.float32(1.0 + 2.0**-20)
MUT_BOUND_Z = np.float32(6.0)


def amax_w1(pop, widths):
    """Largest |W_1| of every network (float32, exact; NaN if W_1 holds a
    NaN, inf for an infinity)."""
    pop = np.asarray(pop, dtype=np.float32)
    w1 = widths[0] * widths[1]
    a = np.abs(pop[:, :w1])
    out = a.max(axis=1)
    out[np.isnan(a).any(axis=1)] = np.nan
    return out.astype(np.float32)


def fp8_child_bounds(parent_amax, ops, p1, p2, sigma):
    """Bound of each child's largest |W_1| from its parents (float32, each
    operation rounded): an elite has its parent's largest magnitude; every
    gene of a crossover child (uniform: a parent's gene; arithmetic:
    fl(fl(a + b) * 0.5), which lies between them) is bounded by the larger
    parent's; a mutant's genes are fl(t + fl(sigma * z)) with |z| <= 5.78 for
    the float32 Box-Muller sampler (radius sqrt(-2 ln 2^-24) ~= 5.768), so
    fl(fl(a * (1 + 2^-20)) + fl(6 sigma)) covers them with room for every
    rounding."""
    amax = np.asarray(parent_amax, dtype=np.float32)
    ops = np.asarray(ops)
    a1 = amax[np.asarray(p1)]
    a2 = amax[np.asarray(p2)]
    cross = np.where(np.isnan(a1) | np.isnan(a2), np.float32(np.nan), np.maximum(a1, a2))
    mut = (a1 * MUT_BOUND_FACTOR) + (MUT_BOUND_Z * np.float32(sigma))
    out = np.where(ops == L.ELITE, a1, np.where(ops == L.CROSS, cross, mut))
    return out.astype(np.float32)


def quantize_fp8(a, bound=None):
    """(values, e): a (float32) divided by 2^e, rounded to E4M3, as float64
    values still scaled by 2^-e; e from `bound` (default: the operand's
    largest magnitude).  Returns (None, None) if a holds NaN or an infinity
    or the bound is not finite."""
    a = np.asarray(a, dtype=np.float64)
    if not np.all(np.isfinite(a)):
        return None, None
    if bound is None:
        bound = np.max(np.abs(a)) if a.size else 0.0
    if not math.isfinite(float(bound)):
        return None, None
    if a.size and np.max(np.abs(a)) > float(bound):
        raise ValueError("the bound is below the operand's largest magnitude")
    e = fp8_exponent(float(bound))
    return round_e4m3(a * 2.0**-e), e


def layer1_operands(genome, widths, x, dtype, w_bound=None):
    """(Xq, Wq, factor) such that the first layer's product is
    factor * Xq Wq^T exactly; Xq / Wq are None when an fp8 operand is not
    finite (the network's fitness is NaN).  w_bound: the bound the FP8 scale
    of W_1 comes from (default: its largest magnitude)."""
    W1 = L.unpack(np.asarray(genome), widths)[0][0]
    if dtype == BF16:
        return (round_bf16(x).astype(np.float64), round_bf16(W1).astype(np.float64), 1.0)
    if dtype == FP8:
        xq, ex = quantize_fp8(x)
        wq, ew = quantize_fp8(W1, w_bound)
        if xq is None or wq is None:
            return None, None, None
        return xq, wq, 2.0**(ex + ew)
    if dtype == F32:
        return (np.asarray(x, dtype=np.float64), W1.astype(np.float64), 1.0)
    raise ValueError("unknown dtype %r" % (dtype,))


def tail_operand(W, dtype):
    """(Wq, factor) of a weight matrix past the first layer: the layer's
    product with activations h is factor * h Wq^T exactly as in float64;
    Wq is None when an fp8 weight is not finite."""
    W = np.asarray(W, dtype=np.float32)
    if dtype == BF16:
        return round_bf16(W).astype(np.float64), 1.0
    if dtype == FP8:
        wq, e = quantize_fp8(W)
        return (None, None) if wq is None else (wq, 2.0**e)
    if dtype == F32:
        return W.astype(np.float64), 1.0
    raise ValueError("unknown dtype %r" % (dtype,))


def forward_lowp(genome, widths, x, dtype, w_bound=None):
    """Logits (float64) of one network with every layer's weights (and the
    batch) in `dtype`."""
    layers = L.unpack(np.asarray(genome), widths)
    xq, wq, factor = layer1_operands(genome, widths, x, dtype, w_bound)
    n = np.asarray(x).shape[0]
    if xq is None:
        return np.full((n, widths[-1]), np.nan)
    h = factor * (xq @ wq.T) + layers[0][1].astype(np.float64)
    for l, (W, b) in enumerate(layers):
        if l > 0:
            Wq, fac_l = tail_operand(W, dtype)
            if Wq is None:
                return np.full((n, widths[-1]), np.nan)
            h = fac_l * (h @ Wq.T) + b.astype(np.float64)
        if l < len(layers) - 1:
            h = np.maximum(h, 0.0)
    return h


def evaluate_lowp(pop, widths, x, y, dtype, w_bounds=None):
    """Raw fitness and accuracy of every network with its weights and the
    batch in `dtype` (float64 everywhere else); w_bounds: per-network FP8
    bounds of W_1."""
    P = pop.shape[0]
    f = np.empty(P, dtype=np.float64)
    acc = np.empty(P, dtype=np.float64)
    for j in range(P):
        z = forward_lowp(pop[j], widths, x, dtype, None if w_bounds is None else w_bounds[j])
        if np.isnan(z).any():
            f[j], acc[j] = np.nan, np.nan
        else:
            f[j], acc[j] = L.fitness_from_logits(z, y)
    return f, acc
