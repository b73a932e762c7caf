"""Pins for the paper-faithful variants in the oracle: 2x2 max-pooling of
inputs (section 4.1), exponential sigma decay and self-adaptive sigma
(section 3.2) with the float32 exp."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import leea as L
from oracle import normal32 as N
from oracle import philox

F32 = np.float32


def test_exp32_accuracy_and_special_values():
    x = np.linspace(-30, 30, 600001).astype(F32)
    y = N.exp32(x)
    ref = np.exp(x.astype(np.float64))
    ulp = np.abs(y - ref) / np.spacing(ref.astype(F32)).astype(np.float64)
    assert ulp.max() <= 1.5
    assert N.exp32(F32(0.0)) == F32(1.0)
    xs = np.linspace(-25, 25, 1001).astype(F32)
    prod = N.exp32(xs).astype(np.float64) * N.exp32(-xs).astype(np.float64)
    assert np.all(np.abs(prod - 1.0) < 4 * 2.0**-23)
    with pytest.raises(ValueError):
        N.exp32(F32(81.0))


def test_exp32_small_arguments_and_monotone():
    x = np.sort(np.random.Generator(np.random.PCG64(0)).standard_normal(200000) * 0.05).astype(F32)
    y = N.exp32(x)
    ref = np.exp(x.astype(np.float64))
    assert (np.abs(y - ref) / np.spacing(ref.astype(F32))).max() <= 1.0
    assert np.all(np.diff(y.astype(np.float64)) >= 0)


def test_pool2x2_hand_example_and_brute_force():
    img = np.array([[1, 5, 2, 0],
                    [3, 4, 8, 1],
                    [0, 0, -1, -2],
                    [7, 0, -3, -4]], dtype=F32).reshape(1, 16)
    assert np.array_equal(L.pool2x2(img, 4), np.array([[5, 8, 7, -1]], dtype=F32))
    rng = np.random.Generator(np.random.PCG64(1))
    x = rng.random((5, 28 * 28)).astype(F32)
    out = L.pool2x2(x, 28)
    assert out.shape == (5, 196)
    for n in range(5):
        im = x[n].reshape(28, 28)
        for r in range(14):
            for c in range(14):
                assert out[n, r * 14 + c] == max(im[2 * r, 2 * c], im[2 * r, 2 * c + 1],
                                                 im[2 * r + 1, 2 * c], im[2 * r + 1, 2 * c + 1])
    nan_img = np.zeros((1, 16), dtype=F32)
    nan_img[0, 5] = np.nan          # window (0, 0)
    nan_img[0, 15] = np.nan         # window (1, 1)
    got = L.pool2x2(nan_img, 4)[0]
    assert np.isnan(got[0]) and np.isnan(got[3]) and got[1] == 0 and got[2] == 0


def test_paper_network_on_pooled_inputs_has_92k_params():
    assert L.param_count((196, 256, 128, 64, 10)) == 92234


def test_sigma_decay_closed_form():
    s = 0.01
    assert L.sigma_decay(s, 0, 10) == F32(s)
    assert abs(float(L.sigma_decay(s, 10, 10)) - 0.99 * s) <= float(np.spacing(F32(0.0099)))
    assert abs(float(L.sigma_decay(s, 1000, 10)) - s * 0.99**100) <= 1e-9
    vals = [float(L.sigma_decay(s, g, 3)) for g in range(50)]
    assert all(a > b for a, b in zip(vals, vals[1:]))


def _cfg(**kw):
    d = dict(widths=(4, 3, 2), pop=400, p_elite=0.05, p_cross=0.5, p_mut=0.45, rho=0.5,
             sigma=0.02, sigma_mode="self_adaptive", tau=0.3, seed=3)
    d.update(kw)
    return L.Config(**d)


def test_child_sigmas_rules():
    cfg = _cfg()
    rng = np.random.Generator(np.random.PCG64(2))
    sig = rng.uniform(0.001, 0.1, cfg.pop).astype(F32)
    f = rng.standard_normal(cfg.pop)
    ops, p1, p2, _ = L.plan(L.rank(f), f, cfg, 4)
    new = L.child_sigmas(sig, ops, p1, p2, cfg, 4)
    e = ops == L.ELITE
    c = ops == L.CROSS
    m = ops == L.MUT
    assert np.array_equal(new[e], sig[p1[e]])
    assert np.array_equal(new[c], ((sig[p1[c]] + sig[p2[c]]) * F32(0.5)).astype(F32))
    z = np.log(new[m].astype(np.float64) / sig[p1[m]]) / 0.3
    for j in np.nonzero(m)[0][:5]:
        w = philox.draw(cfg.seed, philox.SIGMA, 4, j, 0)
        zz, _ = N.normal_pair(w[0], w[1])
        assert abs(np.log(new[j] / np.float64(sig[p1[j]])) / 0.3 - float(zz)) < 1e-4


def test_self_adaptive_log_steps_are_normal():
    cfg = _cfg(pop=2000, p_elite=0.0, p_cross=0.0, p_mut=1.0)
    sig = np.full(cfg.pop, 0.05, dtype=F32)
    zs = []
    for g in range(1, 6):
        ops, p1, p2, _ = L.plan(np.arange(cfg.pop), np.zeros(cfg.pop), cfg, g)
        new = L.child_sigmas(sig, ops, p1, p2, cfg, g)
        zs.append(np.log(new.astype(np.float64) / 0.05) / 0.3)
    z = np.concatenate(zs)
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_adaptive_vary_reduces_to_constant_sigma():
    cfg = _cfg(widths=(30, 5, 3), pop=12, p_gene=1.0)
    rng = np.random.Generator(np.random.PCG64(5))
    pop = rng.standard_normal((12, L.param_count(cfg.widths))).astype(F32)
    f = rng.standard_normal(12)
    ops, p1, p2, _ = L.plan(L.rank(f), f, cfg, 2)
    const = L.vary(pop, ops, p1, p2, cfg, 2, sigma=0.02)
    adapt = L.vary_adaptive(pop, np.full(12, 0.02, dtype=F32), ops, p1, p2, cfg, 2)
    assert np.array_equal(const, adapt)
