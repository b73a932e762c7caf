"""Pins for the reduced-precision oracle (weights and batch in bfloat16 or OCP
FP8 E4M3 with power-of-two scales): the roundings against torch's own
casts and against brute force over the formats' value grids, the scale
rule in closed form, and the forward pass against the float64 forward on
inputs that every format represents exactly."""
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import leea as L
from oracle import precision as Q

F32 = np.float32


def _grid_values(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    mant = rng.random(n) + 1.0
    expo = rng.integers(-40, 40, n)
    sign = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    return (sign * mant * 2.0**expo).astype(F32)


def test_round_bf16_matches_torch_cast():
    x = _grid_values(400000, 0)
    # exact ties: low 16 bits 0x8000, both parities of the kept part
    u = _grid_values(2000, 1).view(np.uint32)
    ties = ((u & 0xFFFF0000) | 0x8000).view(F32)
    special = np.array([0.0, -0.0, np.inf, -np.inf, np.finfo(F32).max, np.finfo(F32).tiny,
                        1e-45, 1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-8], dtype=F32)
    for arr in (x, ties, special):
        ref = torch.from_numpy(arr).to(torch.bfloat16).float().numpy()
        got = Q.round_bf16(arr)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    assert np.isnan(Q.round_bf16(np.array([np.nan], dtype=F32))[0])


def test_round_bf16_brute_force_nearest():
    x = _grid_values(300, 2)
    for v in x:
        u = int(np.array([v], dtype=F32).view(np.uint32)[0])
        lo = np.array([u & 0xFFFF0000], dtype=np.uint32).view(F32)[0]
        hi = np.array([(u & 0xFFFF0000) + 0x10000], dtype=np.uint32).view(F32)[0]
        fv, flo, fhi = Fraction(float(v)), Fraction(float(lo)), Fraction(float(hi))
        dlo, dhi = abs(fv - flo), abs(fhi - fv)
        if dlo < dhi:
            want = lo
        elif dhi < dlo:
            want = hi
        else:
            want = lo if ((u >> 16) & 1) == 0 else hi
        assert Q.round_bf16(np.array([v], dtype=F32))[0] == want


def test_e4m3_table_known_values():
    t = Q.e4m3_table()
    assert len(t) == 127
    assert t[0] == 0.0 and t[1] == 2.0**-9 and t[7] == 7 * 2.0**-9
    assert t[8] == 2.0**-6                    # smallest normal
    assert t[0x38] == 1.0
    assert t[126] == 448.0 == Q.E4M3_MAX
    assert np.all(np.diff(t) > 0)
    assert np.isnan(Q.e4m3_value(0x7F)) and np.isnan(Q.e4m3_value(0xFF))
    assert Q.e4m3_value(0x80 | 0x38) == -1.0


def test_round_e4m3_matches_torch_cast():
    t = Q.e4m3_table()
    mids = (t[1:] + t[:-1]) / 2                               # every tie
    rng = np.random.Generator(np.random.PCG64(3))
    dense = rng.uniform(-448, 448, 200000)
    small = rng.uniform(-2.0**-5, 2.0**-5, 50000)             # subnormal range
    for arr in (mids, -mids, dense, small, t, -t):
        arr32 = arr.astype(F32)
        ref = torch.from_numpy(arr32).to(torch.float8_e4m3fn).float().numpy().astype(np.float64)
        got = Q.round_e4m3(arr32.astype(np.float64))
        assert np.array_equal(got, ref)
    with pytest.raises(ValueError):
        Q.round_e4m3(np.array([449.0]))


def test_round_e4m3_brute_force_nearest_even():
    t = Q.e4m3_table()
    rng = np.random.Generator(np.random.PCG64(4))
    vals = np.concatenate([rng.uniform(0, 448, 500), (t[1:] + t[:-1]) / 2])
    for v in vals:
        d = np.abs(t - v)
        best = np.flatnonzero(d == d.min())
        want = best[0] if len(best) == 1 else [c for c in best if c % 2 == 0][0]
        assert Q.round_e4m3_codes(np.array([v]))[0] == want


def test_fp8_exponent_closed_form():
    assert Q.fp8_exponent(0.0) == 0
    assert Q.fp8_exponent(448.0) == 0
    assert Q.fp8_exponent(np.nextafter(448.0, 1e9)) == 1
    assert Q.fp8_exponent(224.0) == -1
    assert Q.fp8_exponent(1.0) == -8          # 448 / 256 = 1.75 >= 1 > 0.875
    rng = np.random.Generator(np.random.PCG64(5))
    for a in np.exp(rng.uniform(-60, 60, 2000)):
        e = Q.fp8_exponent(a)
        assert a <= 448.0 * 2.0**e and a > 448.0 * 2.0**(e - 1)


def test_quantize_fp8_scale_equivariance():
    rng = np.random.Generator(np.random.PCG64(6))
    a = (rng.standard_normal(5000) * 0.05).astype(F32)
    q, e = Q.quantize_fp8(a)
    assert np.max(np.abs(q)) <= 448.0 and np.max(np.abs(q)) > 224.0 - 16.0
    for k in (-5, 3, 20):
        q2, e2 = Q.quantize_fp8((a.astype(np.float64) * 2.0**k).astype(F32))
        assert e2 == e + k and np.array_equal(q2, q)
    assert Q.quantize_fp8(np.array([1.0, np.nan], dtype=F32)) == (None, None)


def _tiny_net(widths, rng, scale):
    c = L.param_count(widths)
    g = np.zeros(c, dtype=F32)
    # dyadic weights with 3 significant bits: exact in bf16 and (scaled) E4M3
    g[:] = (rng.integers(-7, 8, c) * 2.0**-scale).astype(F32)
    return g


def test_forward_lowp_reduces_to_forward_on_representable_values():
    rng = np.random.Generator(np.random.PCG64(7))
    widths = (12, 8, 5, 3)
    g = _tiny_net(widths, rng, 6)
    x = (rng.integers(0, 8, (9, 12)) * 2.0**-3).astype(F32)
    ref = L.forward(g, widths, x)
    for dt in (Q.F32, Q.BF16, Q.FP8):
        assert np.array_equal(Q.forward_lowp(g, widths, x, dt), ref), dt


def test_forward_lowp_error_within_quantisation_bound():
    rng = np.random.Generator(np.random.PCG64(8))
    widths = (64, 16, 4)
    g = (rng.standard_normal(L.param_count(widths)) * 0.1).astype(F32)
    x = rng.random((20, 64)).astype(F32)
    W1 = L.unpack(g, widths)[0][0].astype(np.float64)
    mag = np.abs(x.astype(np.float64)) @ np.abs(W1).T      # sum |x||w| per unit
    exact = x.astype(np.float64) @ W1.T
    for dt, u in ((Q.BF16, 2.0**-8), (Q.FP8, 2.0**-4)):
        xq, wq, fac = Q.layer1_operands(g, widths, x, dt)
        got = fac * (xq @ wq.T)
        # each operand carries relative error <= u (normals); fp8 subnormals
        # add an absolute 2^-10 * 2^e per operand
        bound = mag * (2 * u + u * u)
        if dt == Q.FP8:
            ex = Q.fp8_exponent(np.abs(x).max())
            ew = Q.fp8_exponent(np.abs(W1).max())
            sub = 2.0**-10
            bound += (np.abs(x).sum(1)[:, None] * sub * 2.0**ew
                      + (np.abs(W1).sum(1)[None, :] * sub * 2.0**ex) + 64 * sub * sub * 2.0**(ex + ew)) * 1.01
        assert np.all(np.abs(got - exact) <= bound + 1e-15), dt
        assert np.any(got != exact), dt


def test_tail_weights_rounded_hand_example():
    """A later layer's weight 1 + 2^-9 with an exact first layer: the float32
    logit is 1 + 2^-9; bfloat16 (spacing 2^-7 at 1) rounds the weight to 1;
    FP8 scales it by 2^-(-8) to 256.5, which E4M3 (spacing 32 there) rounds to
    256, i.e. 1 after the scale."""
    widths = (2, 1, 1)
    g = np.zeros(L.param_count(widths), dtype=F32)
    (W1, b1), (W2, b2) = L.unpack(g, widths)
    W1[0, 0] = 1.0
    W2[0, 0] = 1.0 + 2.0**-9
    g = np.concatenate([W1.ravel(), b1, W2.ravel(), b2]).astype(F32)
    x = np.array([[1.0, 0.0]], dtype=F32)
    assert Q.forward_lowp(g, widths, x, Q.F32)[0, 0] == 1.0 + 2.0**-9
    assert Q.forward_lowp(g, widths, x, Q.BF16)[0, 0] == 1.0
    assert Q.fp8_exponent(1.0 + 2.0**-9) == -8
    assert Q.forward_lowp(g, widths, x, Q.FP8)[0, 0] == 1.0


@pytest.mark.parametrize("dt", [Q.BF16, Q.FP8])
def test_tail_layer_scale_is_per_layer(dt):
    """Multiplying the last layer's weights by 2^k (bias zero) multiplies the
    logits by exactly 2^k: the last layer's FP8 scale follows its own largest
    magnitude (a scale taken from another layer would overflow E4M3 at
    2^20 or lose bits at 2^-20), and bfloat16 rounding commutes with powers
    of two."""
    rng = np.random.Generator(np.random.PCG64(11))
    widths = (16, 8, 5)
    g = (rng.standard_normal(L.param_count(widths)) * 0.3).astype(F32)
    (W1, b1), (W2, b2) = L.unpack(g, widths)
    b2[:] = 0.0
    x = rng.random((7, 16)).astype(F32)
    base = np.concatenate([W1.ravel(), b1, W2.ravel(), b2]).astype(F32)
    ref = Q.forward_lowp(base, widths, x, dt)
    for k in (20, -20, 3):
        gk = np.concatenate([W1.ravel(), b1, (W2 * F32(2.0**k)).ravel(), b2]).astype(F32)
        assert np.array_equal(Q.forward_lowp(gk, widths, x, dt), ref * 2.0**k), (dt, k)
    # and the rounding of the later layer is there: it differs from float32
    assert not np.array_equal(ref, Q.forward_lowp(base, widths, x, Q.F32))


def test_tail_product_error_within_quantisation_bound():
    """A later layer's product against the exact one: each weight carries a
    relative error <= 2^-8 (bfloat16) or 2^-4 (E4M3 normals) plus, for FP8,
    an absolute 2^-10 * 2^e for subnormals."""
    rng = np.random.Generator(np.random.PCG64(12))
    W = (rng.standard_normal((10, 32)) * 0.2).astype(F32)
    h = np.abs(rng.standard_normal((20, 32)))
    exact = h @ W.astype(np.float64).T
    mag = h @ np.abs(W.astype(np.float64)).T
    for dt, u in ((Q.BF16, 2.0**-8), (Q.FP8, 2.0**-4)):
        wq, fac = Q.tail_operand(W, dt)
        got = fac * (h @ wq.T)
        bound = mag * u
        if dt == Q.FP8:
            bound += h.sum(1)[:, None] * 2.0**-10 * fac
        assert np.all(np.abs(got - exact) <= bound * 1.0001 + 1e-15), dt
        assert np.any(got != exact), dt


def test_lowp_nan_operands_give_nan_fitness():
    rng = np.random.Generator(np.random.PCG64(9))
    widths = (8, 4, 3)
    pop = (rng.standard_normal((3, L.param_count(widths))) * 0.3).astype(F32)
    pop[1, 5] = np.nan
    x = rng.random((6, 8)).astype(F32)
    y = rng.integers(0, 3, 6)
    for dt in (Q.BF16, Q.FP8):
        f, _ = Q.evaluate_lowp(pop, widths, x, y, dt)
        assert np.isnan(f[1]) and np.isfinite(f[0]) and np.isfinite(f[2])
    # a non-finite weight in a later layer: NaN fitness under FP8 (its scale)
    w2 = widths[0] * widths[1] + widths[1]
    pop[2, w2 + 1] = np.inf
    f, _ = Q.evaluate_lowp(pop, widths, x, y, Q.FP8)
    assert np.isnan(f[2]) and np.isfinite(f[0])


def test_box_muller_radius_bound():
    """The largest normal the float32 sampler can return: u1 = 2^-24 (its
    smallest value) gives the largest radius, sqrt(-2 ln 2^-24) ~= 5.768, and
    the rotated cosine/sine never exceed 1; the FP8 mutation bound uses 6."""
    from oracle.normal32 import normal_pair
    words = np.array([0, 1, 0xFF, 0x3FFFFFFF, 0x40000000, 0x7FFFFFFF, 0x80000000, 0xBFFFFFFF,
                      0xC0000000, 0xFFFFFFFF, 0x12345678], dtype=np.uint32)
    zmax = 0.0
    for b in words:
        for a in (np.uint32(0), np.uint32(0xFF)):          # both give u1 = 2^-24
            z0, z1 = normal_pair(a, b)
            zmax = max(zmax, abs(float(z0)), abs(float(z1)))
    assert 5.76 < zmax <= 5.78
    # every other u1 gives a smaller radius
    rng = np.random.Generator(np.random.PCG64(0))
    for a, b in rng.integers(0, 2**32, (2000, 2), dtype=np.uint64).astype(np.uint32):
        z0, z1 = normal_pair(a, b)
        assert abs(float(z0)) <= zmax and abs(float(z1)) <= zmax


@pytest.mark.parametrize("crossover", ["uniform", "arithmetic"])
def test_fp8_child_bounds_cover_the_children(crossover):
    """Soundness of the parent-derived FP8 bound: for elites it is the
    parent's largest |W_1| exactly; for crossover children and mutants (many
    sigmas and mutation rates, magnitudes from 1e-30 to 1e3) every child's
    largest |W_1| stays at or below it; where sigma is small against the
    weights (the paper's regime) the scale exponent it gives is the exact
    one or one above."""
    widths = (48, 16, 4)
    c = L.param_count(widths)
    rng = np.random.Generator(np.random.PCG64(3))
    for sigma, p_gene, mag in ((0.001, 1.0, 0.08), (0.05, 0.3, 1e-3), (0.0, 1.0, 1.0),
                               (1e-12, 1.0, 2.0), (3.0, 1.0, 1e3), (0.01, 0.1, 1e-30)):
        P = 24
        pop = (rng.standard_normal((P, c)) * mag).astype(np.float32)
        pop[5, :widths[0] * widths[1]] = 0.0
        cfg = L.Config(widths=widths, pop=P, p_elite=0.25, p_cross=0.5, p_mut=0.25, rho=0.5,
                       crossover=crossover, sigma=sigma, p_gene=p_gene, seed=9)
        f = rng.standard_normal(P).astype(np.float32)
        for g in (1, 2, 3):
            ops, p1, p2, _ = L.plan(L.rank(f), f, cfg, g)
            kids = L.vary(pop, ops, p1, p2, cfg, g)
            amax_p = Q.amax_w1(pop, widths)
            bound = Q.fp8_child_bounds(amax_p, ops, p1, p2, sigma)
            amax_k = Q.amax_w1(kids, widths)
            assert np.all(amax_k <= bound), (sigma, p_gene, mag, g)
            el = ops == L.ELITE
            assert np.array_equal(bound[el], amax_p[p1[el]])
            tight = 6 * sigma <= mag / 8
            for j in range(P):
                if amax_k[j] == 0.0:
                    continue
                e_exact = Q.fp8_exponent(float(amax_k[j]))
                e_bound = Q.fp8_exponent(float(bound[j]))
                assert e_bound >= e_exact
                if tight and ops[j] != L.CROSS:
                    assert e_bound <= e_exact + 1, (sigma, mag, j)
            pop = kids


def test_fp8_child_bounds_non_finite_parents():
    amax = np.array([0.5, np.nan, np.inf, 0.25], dtype=np.float32)
    ops = np.array([L.ELITE, L.CROSS, L.CROSS, L.MUT, L.MUT])
    p1 = np.array([1, 0, 0, 2, 3])
    p2 = np.array([1, 1, 2, 2, 3])
    b = Q.fp8_child_bounds(amax, ops, p1, p2, 0.01)
    assert np.isnan(b[0]) and np.isnan(b[1]) and np.isinf(b[2]) and np.isinf(b[3])
    assert b[4] == (np.float32(0.25) * Q.MUT_BOUND_FACTOR) + np.float32(6.0) * np.float32(0.01)


def test_quantize_fp8_with_a_bound():
    a = np.array([0.5, -0.25, 0.125], dtype=np.float32)
    q0, e0 = Q.quantize_fp8(a)
    q1, e1 = Q.quantize_fp8(a, bound=0.5)
    assert e0 == e1 and np.array_equal(q0, q1)
    q2, e2 = Q.quantize_fp8(a, bound=1.0)            # one binade up
    assert e2 == e0 + 1 and np.array_equal(q2 * 2.0**e2, q0 * 2.0**e0)
    assert Q.quantize_fp8(a, bound=np.inf) == (None, None)
    with pytest.raises(ValueError):
        Q.quantize_fp8(a, bound=0.4)
