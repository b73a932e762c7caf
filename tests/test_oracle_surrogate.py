"""Pins for the fitness-surrogate oracle: the MLP against torch's own
layers and autograd, Kendall tau against scipy, the projection by its
algebra (linearity, exact integer dot products on representable genomes),
the candidate generation against the regular variation, and the
screening by brute force."""
import math

import numpy as np
import pytest
import torch
from scipy import stats

from oracle import leea as L
from oracle import philox
from oracle import surrogate as S

F32 = np.float32


def test_projection_signs_are_balanced_and_independent():
    R = S.projection_signs(3000, seed=5)
    assert R.shape == (256, 3000)
    assert set(np.unique(R)) == {-1, 1}
    # fair coins: the total of 768k signs is within 5 sigma of 0
    assert abs(int(R.astype(np.int64).sum())) < 5 * math.sqrt(R.size)
    C = (R.astype(np.float64) @ R.T.astype(np.float64)) / R.shape[1]
    off = C[~np.eye(256, dtype=bool)]
    assert np.max(np.abs(off)) < 6 / math.sqrt(3000)
    assert np.array_equal(R, S.projection_signs(3000, seed=5))
    assert not np.array_equal(R, S.projection_signs(3000, seed=6))


def test_features_algebra():
    rng = np.random.Generator(np.random.PCG64(0))
    g = 700
    R = S.projection_signs(g, seed=1)
    # genomes representable in bfloat16: integer multiples of 2^-6 below 2
    kids = (rng.integers(-100, 100, (5, g)) * 2.0**-6).astype(F32)
    par = kids.copy()
    par[:, 3] += F32(0.5)
    fp = np.array([-1.0, -2.0, -0.5, -3.0, -2.25], dtype=F32)
    X = S.features(kids, par, fp, fp * 2, R)
    s = float(S.scale(g))
    exact = (np.rint(kids.astype(np.float64) * 64).astype(np.int64) @ R.T.astype(np.int64))
    assert np.array_equal(X[:, :256], exact * (s / 64))
    assert np.allclose(X[:, 258], 0.5 * s, rtol=0, atol=1e-15)
    assert np.array_equal(X[:, 256], fp.astype(np.float64))
    assert np.array_equal(X[:, 257], (fp * 2).astype(np.float64))
    X2 = S.features(kids * F32(4), kids * F32(4), fp, fp, R)
    assert np.array_equal(X2[:, :256], 4 * X[:, :256]) and np.all(X2[:, 258] == 0)


def test_init_mlp_bounds_and_statistics():
    p = S.init_mlp(seed=3)
    a1 = math.sqrt(6.0 / (S.INPUTS + S.HIDDEN))
    assert p["W1"].shape == (S.HIDDEN, S.INPUTS) and p["w2"].shape == (S.HIDDEN,)
    assert np.max(np.abs(p["W1"])) <= a1 and np.all(p["b1"] == 0) and p["b2"] == 0
    v = float(np.var(p["W1"].astype(np.float64)))
    assert abs(v - a1 * a1 / 3) < 0.05 * a1 * a1 / 3


def _torch_mlp(p):
    net = torch.nn.Sequential(torch.nn.Linear(S.INPUTS, S.HIDDEN), torch.nn.ReLU(),
                              torch.nn.Linear(S.HIDDEN, 1)).double()
    with torch.no_grad():
        net[0].weight.copy_(torch.from_numpy(np.asarray(p["W1"], dtype=np.float64)))
        net[0].bias.copy_(torch.from_numpy(np.asarray(p["b1"], dtype=np.float64)))
        net[2].weight.copy_(torch.from_numpy(np.asarray(p["w2"], dtype=np.float64))[None, :])
        net[2].bias.fill_(float(p["b2"]))
    return net


def test_mlp_forward_and_step_match_torch():
    rng = np.random.Generator(np.random.PCG64(1))
    p = S.init_mlp(seed=4)
    p["b1"] = rng.standard_normal(S.HIDDEN).astype(F32) * F32(0.1)
    p["b2"] = F32(-0.3)
    X = rng.standard_normal((50, S.INPUTS))
    y = rng.standard_normal(50)
    y[7] = np.nan
    pred, _ = S.mlp_forward(p, X)
    net = _torch_mlp(p)
    ref = net(torch.from_numpy(X)).detach().numpy()[:, 0]
    assert np.allclose(pred, ref, rtol=1e-12, atol=1e-12)
    new = S.mlp_gradient_step(p, X, y, lr=0.05)
    ok = np.isfinite(y)
    loss = torch.mean((net(torch.from_numpy(X[ok]))[:, 0] - torch.from_numpy(y[ok])) ** 2)
    loss.backward()
    with torch.no_grad():
        for prm in net.parameters():
            prm -= 0.05 * prm.grad
    assert np.allclose(new["W1"], net[0].weight.detach().numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(new["b1"], net[0].bias.detach().numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(new["w2"], net[2].weight.detach().numpy()[0], rtol=1e-12, atol=1e-12)
    assert abs(new["b2"] - float(net[2].bias.detach()[0])) < 1e-12


def test_kendall_tau_against_scipy_and_brute_force():
    rng = np.random.Generator(np.random.PCG64(2))
    a = rng.standard_normal(200)
    b = a + rng.standard_normal(200)
    assert abs(S.kendall_tau_a(a, b) - stats.kendalltau(a, b).statistic) < 1e-12
    a = rng.integers(0, 5, 40).astype(float)
    b = rng.integers(0, 5, 40).astype(float)
    s = 0
    for i in range(40):
        for j in range(i + 1, 40):
            s += np.sign(a[i] - a[j]) * np.sign(b[i] - b[j])
    assert abs(S.kendall_tau_a(a, b) - s / (40 * 39 / 2)) < 1e-15
    assert S.kendall_tau_a([1, 2, 3], [1, 2, 3]) == 1.0
    assert S.kendall_tau_a([1, 2, 3], [3, 2, 1]) == -1.0


def _cfg(**kw):
    d = dict(widths=(20, 6, 3), pop=24, p_elite=0.05, p_cross=0.5, p_mut=0.45, rho=0.5,
             sigma=0.02, p_gene=0.5, seed=9)
    d.update(kw)
    return L.Config(**d)


def test_candidate_plan_structure_and_slots():
    cfg = _cfg()
    rng = np.random.Generator(np.random.PCG64(3))
    f = rng.standard_normal(cfg.pop).astype(F32)
    order = L.rank(f)
    n_e, n_c, n_m, n_rho = L.counts(cfg.pop, cfg.p_elite, cfg.p_cross, cfg.p_mut, cfg.rho)
    ops, p1, p2, fi = S.candidate_plan(order, f, cfg, 3, k=4)
    assert len(ops) == 4 * (cfg.pop - n_e)
    assert np.all(ops[:4 * n_c] == L.CROSS) and np.all(ops[4 * n_c:] == L.MUT)
    top = set(order[:n_rho].tolist())
    assert set(p1.tolist()) <= top and set(p2.tolist()) <= top
    # candidate c is the regular plan's rule at slot P + c
    big = L.Config(**{**cfg.__dict__, "pop": cfg.pop})
    for c in (0, 5, 4 * n_c, len(ops) - 1):
        r = L._parent_rank(big, n_rho, 3, cfg.pop + c, 0)
        assert p1[c] == order[r]
    cr = ops == L.CROSS
    assert np.array_equal(fi[cr], (f[p1[cr]] + f[p2[cr]]) * F32(0.5))
    assert np.array_equal(fi[~cr], f[p1[~cr]])
    ops1, p11, _, _ = S.candidate_plan(order, f, _cfg(rho=1.0 / cfg.pop), 3, k=2)
    assert np.all(p11 == order[0])


def test_candidates_are_regular_children_at_shifted_slots():
    cfg = _cfg()
    rng = np.random.Generator(np.random.PCG64(4))
    g = L.param_count(cfg.widths)
    pop = rng.standard_normal((cfg.pop, g)).astype(F32)
    f = rng.standard_normal(cfg.pop).astype(F32)
    ops, p1, p2, _ = S.candidate_plan(L.rank(f), f, cfg, 2, k=3)
    kids = S.candidates(pop, ops, p1, p2, cfg, 2)
    P = cfg.pop
    # a regular plan whose slots P .. P + M - 1 hold the candidates
    M = len(ops)
    big_ops = np.concatenate([np.zeros(P, np.int32), ops])
    big_p1 = np.concatenate([np.zeros(P, np.int64), p1])
    big_p2 = np.concatenate([np.zeros(P, np.int64), p2])
    ref = L.vary(pop, big_ops, big_p1, big_p2, cfg, 2, slots=range(P, P + M))
    assert np.array_equal(kids.view(np.uint32), ref.view(np.uint32))
    for c in range(M):   # provenance: every gene from a parent, or mutated
        if ops[c] == L.CROSS and cfg.crossover == "uniform":
            assert np.all((kids[c] == pop[p1[c]]) | (kids[c] == pop[p2[c]]))


def test_screen_brute_force_and_fallback():
    rng = np.random.Generator(np.random.PCG64(5))
    pred = rng.standard_normal(40).astype(F32)
    pred[[3, 9]] = pred[5]                 # ties resolved by candidate index
    pred[11] = np.nan
    keep = S.screen(pred, 10, True, 4, 6, 4)
    ref = sorted(range(40), key=lambda c: (np.isnan(pred[c]), -np.nan_to_num(pred[c]), c))[:10]
    assert keep.tolist() == ref
    fb = S.screen(pred, 10, False, 4, 6, 4)
    assert fb.tolist() == list(range(6)) + [24, 25, 26, 27]


def test_standardize_closed_forms():
    rng = np.random.Generator(np.random.PCG64(9))
    X = rng.standard_normal((500, 7)) * np.array([1e-4, 1, 3, 0, 1e3, 2, 5]) + 10.0
    Z = S.standardize(X)
    ok = np.array([True, True, True, False, True, True, True])
    assert np.allclose(Z[:, ok].mean(axis=0), 0.0, atol=1e-9)
    assert np.allclose(Z[:, ok].std(axis=0), 1.0, rtol=1e-9)
    assert np.array_equal(Z[:, 3], np.zeros(500))               # a constant column
    # invariant under a positive affine map of a column, negated under a negative one
    X2 = X.copy()
    X2[:, 1] = 7.5 * X[:, 1] - 3.0
    X2[:, 2] = -0.25 * X[:, 2] + 1.0
    Z2 = S.standardize(X2)
    assert np.allclose(Z2[:, 1], Z[:, 1], atol=1e-12)
    assert np.allclose(Z2[:, 2], -Z[:, 2], atol=1e-12)
    # a two-valued column: +-1 exactly
    X3 = np.array([[0.0], [2.0], [0.0], [2.0]])
    assert np.array_equal(S.standardize(X3)[:, 0], np.array([-1.0, 1.0, -1.0, 1.0]))


def test_mlp_inputs_weight_the_projection_block_as_one_feature():
    rng = np.random.Generator(np.random.PCG64(10))
    X = rng.standard_normal((300, S.INPUTS)) * rng.uniform(0.1, 10.0, S.INPUTS) + 3.0
    X[:, 5] = 2.0                                               # one constant projection
    Z = S.mlp_inputs(X)
    Zs = S.standardize(X)
    # the scalar features are the standardised ones, unchanged
    assert np.array_equal(Z[:, S.FEATURES:], Zs[:, S.FEATURES:])
    # the projections are the standardised ones times 2^-4 exactly
    assert np.array_equal(Z[:, :S.FEATURES] * 16.0, Zs[:, :S.FEATURES])
    assert np.array_equal(Z[:, 5], np.zeros(300))
    # block weight: mean over candidates of the squared block norm = (varying columns) / 256
    blk = (Z[:, :S.FEATURES] ** 2).sum(axis=1).mean()
    assert abs(blk - (S.FEATURES - 1) / S.FEATURES) < 1e-12
    assert np.allclose((Z[:, S.FEATURES:] ** 2).mean(axis=0), 1.0, rtol=1e-12)


def test_standardize_targets():
    y = np.array([-2.0, -1.0, np.nan, 0.0, np.inf, 3.0])
    t = S.standardize_targets(y)
    f = np.isfinite(y)
    assert np.allclose(t[f].mean(), 0.0, atol=1e-12) and np.isclose(t[f].std(), 1.0)
    assert np.isnan(t[2]) and np.isinf(t[4])
    assert np.array_equal(S.standardize_targets(np.full(5, -2.3)), np.zeros(5))
    # ranks are kept: Kendall tau of targets and their standardisation is 1
    v = np.random.Generator(np.random.PCG64(1)).standard_normal(200)
    assert S.kendall_tau_a(v, S.standardize_targets(v)) == 1.0
