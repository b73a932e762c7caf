"""Pins for the oracle's EA steps: counts, layout, init, forward, fitness
(Eq. 1), inheritance, rank, selection plan, crossover, mutation, batch draw,
and the generation loop."""
import json
import math
import os

import numpy as np
import pytest
import torch
from scipy import special, stats

from oracle import leea as L
from oracle import philox
from oracle.normal32 import normals4

F32 = np.float32


def cfg_small(**kw):
    d = dict(widths=(784, 32, 10), pop=16, p_elite=0.05, p_cross=0.5, p_mut=0.45,
             rho=0.25, crossover="uniform", sigma=0.01, p_gene=0.1, alpha=1.0, seed=2)
    d.update(kw)
    return L.Config(**d)


# ---------------------------------------------------------------- counts ---

def test_counts_paper_settings():
    assert L.counts(16, 0.05, 0.50, 0.45, 0.25) == (1, 8, 7, 4)
    assert L.counts(1000, 0.05, 0.50, 0.45, 0.50) == (50, 500, 450, 500)
    assert L.counts(2000, 0.05, 0.75, 0.20, 0.50) == (100, 1500, 400, 1000)


def test_counts_conserved_brute_force():
    for pop in range(1, 4097, 7):
        for fr in ((0.05, 0.50, 0.45), (0.05, 0.75, 0.20), (0.1, 0.3, 0.6), (0.0, 0.0, 1.0)):
            for rho in (0.01, 0.1, 0.25, 0.5, 1.0):
                e, c, m, r = L.counts(pop, *fr, rho)
                assert e + c + m == pop and min(e, c, m) >= 0 and 1 <= r <= pop
                assert abs(e - fr[0] * pop) <= 0.5 and abs(c - fr[1] * pop) <= 0.5


def test_counts_reject_bad_fractions():
    with pytest.raises(ValueError):
        L.counts(10, 0.5, 0.5, 0.5, 0.5)
    with pytest.raises(ValueError):
        L.counts(0, 0.05, 0.5, 0.45, 0.5)


def test_mutation_threshold():
    assert L.mutation_threshold(1.0) == 1 << 32
    assert L.mutation_threshold(0.0) == 0
    assert L.mutation_threshold(0.5) == 1 << 31
    # 0.1 as a binary double is 0.1000000000000000055...; times 2^32 = 429496729.6
    assert L.mutation_threshold(0.1) == 429496729


# ---------------------------------------------------------------- layout ---

def test_param_counts():
    assert L.param_count((784, 32, 10)) == 25450
    assert L.param_count((784, 112, 32, 10)) == 91866
    assert L.param_count((196, 256, 128, 64, 10)) == 92234   # the paper's "92k"


def test_layer_slices_tile_the_genome():
    w = (5, 4, 3, 2)
    sl = L.layer_slices(w)
    pos = 0
    for (a, b), (c, d) in sl:
        assert a == pos and c == b
        pos = d
    assert pos == L.param_count(w)


# ------------------------------------------------------------------ init ---

def test_init_bounds_and_biases():
    cfg = cfg_small(pop=4)
    pop = L.init_population(cfg)
    assert pop.dtype == F32 and pop.shape == (4, 25450)
    (w1, b1), (w2, b2) = L.layer_slices(cfg.widths)
    a1 = math.sqrt(6 / (784 + 32))
    a2 = math.sqrt(6 / (32 + 10))
    assert np.all(pop[:, b1[0]:b1[1]] == 0) and np.all(pop[:, b2[0]:b2[1]] == 0)
    W1 = pop[:, w1[0]:w1[1]].astype(np.float64)
    assert np.all(np.abs(W1) <= a1 * (1 + 1e-7))
    assert np.all(np.abs(pop[:, w2[0]:w2[1]]) <= a2 * (1 + 1e-7))
    n = W1.size
    assert abs(W1.mean()) < 5 * a1 / math.sqrt(3 * n)
    assert abs(W1.var() / (a1 * a1 / 3) - 1) < 0.02


def test_init_first_gene_from_known_answer():
    # seed 0, slot 0, gene 0 uses word 0 of Philox(counter 0, key 0), the
    # first published known-answer vector: 0x6627e8d5
    cfg = cfg_small(pop=1, seed=0)
    pop = L.init_population(cfg)
    u = (0x6627e8d5 >> 8) / 2**24
    a1 = F32(math.sqrt(6 / (784 + 32)))
    assert pop[0, 0] == F32(F32(2 * u - 1) * a1)


def test_init_slots_differ_and_are_reproducible():
    cfg = cfg_small(pop=3)
    a = L.init_population(cfg)
    b = L.init_population(cfg)
    assert np.array_equal(a, b)
    assert not np.array_equal(a[0], a[1])


# --------------------------------------------------------------- forward ---

def test_forward_hand_computed(golden_dir):
    with open(os.path.join(golden_dir, "tiny_forward.json")) as fh:
        cases = json.load(fh)["cases"]
    for case in cases:
        g = np.array(case["genome"], dtype=F32)
        assert g.size == L.param_count(case["widths"])
        z = L.forward(g, tuple(case["widths"]), np.array(case["x"], dtype=F32))
        assert np.array_equal(z, np.array(case["logits"]))


def test_single_layer_is_a_gemm():
    rng = np.random.Generator(np.random.PCG64(0))
    w = (37, 11)
    g = rng.standard_normal(L.param_count(w)).astype(F32)
    x = rng.standard_normal((9, 37)).astype(F32)
    W = torch.from_numpy(g[:37 * 11].reshape(11, 37)).double()
    ref = torch.nn.functional.linear(torch.from_numpy(x).double(), W,
                                     torch.from_numpy(g[37 * 11:]).double()).numpy()
    np.testing.assert_allclose(L.forward(g, w, x), ref, rtol=1e-13, atol=1e-13)


def test_two_layer_matches_torch_mlp():
    rng = np.random.Generator(np.random.PCG64(1))
    w = (13, 7, 5)
    g = rng.standard_normal(L.param_count(w)).astype(F32)
    x = rng.standard_normal((6, 13)).astype(F32)
    (a, b), (c, d) = L.layer_slices(w)
    t = torch.from_numpy(g).double()
    h = torch.relu(torch.from_numpy(x).double() @ t[a[0]:a[1]].reshape(7, 13).T + t[b[0]:b[1]])
    z = h @ t[c[0]:c[1]].reshape(5, 7).T + t[d[0]:d[1]]
    np.testing.assert_allclose(L.forward(g, w, x), z.numpy(), rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------- fitness ---

def test_fitness_uniform_output_is_minus_log_d():
    z = np.zeros((8, 10))
    y = np.array([0, 3, 0, 9, 1, 0, 2, 5])
    f, acc = L.fitness_from_logits(z, y)
    assert abs(f + math.log(10)) < 1e-15
    assert acc == 3 / 8          # argmax ties go to class 0
    assert abs(L.fitness_rhs_scale(f, 10) + math.log(10) / 10) < 1e-15


def test_fitness_two_class_closed_form():
    for gap in (-5.0, -0.3, 0.0, 0.7, 12.0, 60.0):
        f, acc = L.fitness_from_logits(np.array([[gap, 0.0]]), np.array([0]))
        assert abs(f + math.log1p(math.exp(-gap))) < 1e-14
        assert acc == (1.0 if gap >= 0 else 0.0)


def test_fitness_matches_torch_cross_entropy_and_scipy():
    rng = np.random.Generator(np.random.PCG64(3))
    z = rng.standard_normal((64, 10)) * 3
    y = rng.integers(0, 10, 64)
    f, acc = L.fitness_from_logits(z, y)
    ce = torch.nn.functional.cross_entropy(torch.from_numpy(z), torch.from_numpy(y)).item()
    assert abs(f + ce) < 1e-13
    ll = z[np.arange(64), y] - special.logsumexp(z, axis=1)
    assert abs(f - ll.mean()) < 1e-13
    assert acc == np.mean(np.argmax(z, axis=1) == y)


def test_fitness_stable_for_huge_logits():
    f, acc = L.fitness_from_logits(np.array([[1e4, -1e4, 0.0]]), np.array([1]))
    assert f == -2e4 and acc == 0.0


# ----------------------------------------------------------- inheritance ---

def test_inheritance_special_cases():
    fr = np.array([-1.0, -2.0, -0.5])
    fi = np.array([-3.0, -1.0, -0.25])
    assert np.array_equal(L.inherit(fr, fi, 1.0), fr)
    assert np.array_equal(L.inherit(fr, fi, 0.0), fi)
    assert np.array_equal(L.inherit(fr, fi, 0.3, has_inh=False), fr)
    np.testing.assert_allclose(L.inherit(fr, fi, 0.25), 0.75 * fi + 0.25 * fr, rtol=1e-15)
    f32 = L.inherit_f32(fr.astype(F32), fi.astype(F32), 0.0)
    assert np.array_equal(f32, fi.astype(F32))
    assert np.array_equal(L.inherit_f32(fr, fi, 1.0), fr.astype(F32))
    np.testing.assert_allclose(L.inherit_f32(fr, fi, 0.5), 0.5 * (fr + fi), rtol=1e-7)


# ------------------------------------------------------------------ rank ---

def test_rank_brute_force_four_individuals():
    vals = [1.0, 0.5, 0.0, -0.0, float("nan")]

    def spec(f):
        # NaN last; larger fitness first; -0 == +0; ties by slot
        return sorted(range(4), key=lambda i: (math.isnan(f[i]),
                                               0.0 if math.isnan(f[i]) else -f[i], i))
    import itertools
    for f in itertools.product(vals, repeat=4):
        for dt in (np.float64, F32):
            assert list(L.rank(np.array(f, dtype=dt))) == spec(f)


def test_rank_infinities():
    f = np.array([-np.inf, np.nan, np.inf, 0.0, -1.0])
    assert list(L.rank(f)) == [2, 3, 4, 0, 1]


# ------------------------------------------------------------- selection ---

def _plans(cfg, gens, f=None):
    P = cfg.pop
    f = np.linspace(0, -1, P) if f is None else f
    order = L.rank(f)
    out = []
    for g in gens:
        out.append(L.plan(order, f, cfg, g))
    return order, out


def test_plan_structure_and_elites():
    cfg = cfg_small(pop=40, rho=0.5)
    f = np.random.Generator(np.random.PCG64(0)).standard_normal(40)
    order = L.rank(f)
    ops, p1, p2, fi = L.plan(order, f, cfg, 1)
    e, c, m, r = L.counts(40, 0.05, 0.5, 0.45, 0.5)
    assert list(ops) == [L.ELITE] * e + [L.CROSS] * c + [L.MUT] * m
    assert list(p1[:e]) == list(order[:e])
    top = set(order[:r].tolist())
    assert set(p1[e:].tolist()) <= top and set(p2[e:e + c].tolist()) <= top
    assert np.all(p1[e + c:] == p2[e + c:])
    np.testing.assert_allclose(fi[e:e + c], 0.5 * (f[p1[e:e + c]] + f[p2[e:e + c]]))
    assert np.array_equal(fi[:e], f[p1[:e]]) and np.array_equal(fi[e + c:], f[p1[e + c:]])


def test_truncation_ranks_uniform():
    cfg = cfg_small(pop=100, rho=0.3, p_elite=0.0, p_cross=1.0, p_mut=0.0)
    order = np.arange(100)
    f = -np.arange(100.0)
    counts = np.zeros(30)
    for g in range(1, 301):
        ops, p1, p2, _ = L.plan(order, f, cfg, g)
        counts += np.bincount(p1, minlength=100)[:30] + np.bincount(p2, minlength=100)[:30]
    assert counts.sum() == 300 * 200
    assert stats.chisquare(counts).pvalue > 1e-4


def test_truncation_n_rho_one_and_two():
    cfg = cfg_small(pop=50, rho=0.02, p_elite=0.0, p_cross=0.5, p_mut=0.5)   # n_rho = 1
    order = np.random.Generator(np.random.PCG64(1)).permutation(50)
    ops, p1, p2, _ = L.plan(order, np.zeros(50), cfg, 3)
    assert np.all(p1 == order[0]) and np.all(p2 == order[0])
    cfg = cfg_small(pop=50, rho=0.04, p_elite=0.0, p_cross=1.0, p_mut=0.0)   # n_rho = 2
    ops, p1, p2, _ = L.plan(order, np.zeros(50), cfg, 3)
    for j in range(50):
        w = philox.draw(cfg.seed, philox.SEL, 3, j, 0)
        assert p1[j] == order[int(w[0]) >> 31] and p2[j] == order[int(w[1]) >> 31]


def test_tournament_two_rank_distribution():
    P = 20
    cfg = cfg_small(pop=P, selection="tournament", tournament_k=2,
                    p_elite=0.0, p_cross=1.0, p_mut=0.0)
    order = np.arange(P)
    counts = np.zeros(P)
    for g in range(1, 1001):
        ops, p1, p2, _ = L.plan(order, -np.arange(P, dtype=float), cfg, g)
        counts += np.bincount(p1, minlength=P) + np.bincount(p2, minlength=P)
    r = np.arange(P)
    expect = (2 * (P - r) - 1) / P**2 * counts.sum()
    assert stats.chisquare(counts, expect).pvalue > 1e-4


def test_plan_float32_inherited_fitness():
    cfg = cfg_small(pop=16)
    f = np.random.Generator(np.random.PCG64(2)).standard_normal(16).astype(F32)
    ops, p1, p2, fi = L.plan(L.rank(f), f, cfg, 1)
    assert fi.dtype == F32
    for j in np.nonzero(ops == L.CROSS)[0]:
        assert fi[j] == (f[p1[j]] + f[p2[j]]) * F32(0.5)


# ------------------------------------------------------------- crossover ---

def _mask_with_words(monkeypatch, words_of_block, c, gen=5, slot=0):
    """oracle.leea.uniform_mask with its generator replaced: block B's four
    words are words_of_block(B).  The mask function is exercised as written;
    only the random source is substituted."""
    def fake_draw(seed, purpose, g, s, block, run=0):
        assert purpose == philox.XO and g == gen and s == slot
        block = np.atleast_1d(np.asarray(block, dtype=np.int64))
        return np.stack([words_of_block(int(b)) for b in block]).astype(np.uint32)
    monkeypatch.setattr(L.philox, "draw", fake_draw)
    return L.uniform_mask(123, gen, slot, c)


def _bit_words(k):
    w = [0, 0, 0, 0]
    w[k >> 5] = 1 << (k & 31)
    return w


def test_uniform_mask_uses_every_generator_bit_once(monkeypatch):
    """Section 3.2: every gene of a uniform crossover is its own fair coin.
    With a counter-based generator that holds iff no two genes read the
    same bit of the same block.  The gene -> (block, bit) map is recovered
    from the function itself: 128 calls light one bit position in every
    block (each gene must light up in exactly one of them), 9 calls light
    whole blocks by the bits of block + 1 (the gene's block).  The map must
    be injective and use all 128 bits of every block of a full group."""
    c = 2 * 8192 + 1000 + 3          # two full groups and a ragged third
    n_blocks = 3 * 64
    hits = np.zeros(c, dtype=np.int64)
    bit_of = np.full(c, -1, dtype=np.int64)
    for k in range(128):
        m = _mask_with_words(monkeypatch, lambda b, k=k: _bit_words(k), c)
        hits += m
        bit_of[m] = k
    assert np.all(hits == 1), "a gene reads no bit or more than one"
    block_of = np.zeros(c, dtype=np.int64)
    full = [0xFFFFFFFF] * 4
    for r in range(9):
        m = _mask_with_words(monkeypatch,
                             lambda b, r=r: full if ((b + 1) >> r) & 1 else [0, 0, 0, 0], c)
        block_of |= m.astype(np.int64) << r
    block_of -= 1
    assert np.all((block_of >= 0) & (block_of < n_blocks))
    key = block_of * 128 + bit_of
    assert np.unique(key).size == c, "two genes share a generator bit"
    full_groups = key[:2 * 8192]
    assert np.array_equal(np.sort(full_groups), np.arange(2 * 64 * 128)), \
        "the blocks of a full 8192-gene group are not used bit for bit"
    # the real generator through the recovered map (Philox itself is pinned
    # by its published known-answer vectors)
    monkeypatch.undo()
    seed, gen, slot, run = 0x1234ABCD5678, 9, 17, 3
    mask = L.uniform_mask(seed, gen, slot, c, run)
    genes = np.array([0, 1, 2, 3, 4, 255, 256, 257, 1023, 4099, 8191, 8192, 12345, c - 1])
    w = philox.philox4x32_10(block_of[genes], slot, gen, (run << 8) | philox.XO,
                             seed & 0xFFFFFFFF, seed >> 32)
    word = np.stack(w, axis=-1)[np.arange(genes.size), bit_of[genes] >> 5]
    expect = (word >> (bit_of[genes] & 31).astype(np.uint32)) & 1
    assert np.array_equal(mask[genes], expect.astype(bool))


def test_uniform_mask_known_answer():
    """A few genes worked out by hand from raw Philox words under the gene
    layout the device uses (gene i = 8192 G + 256 t + 4 q + e reads bit
    4 (t mod 8) + e of word t div 8 of block 64 G + q)."""
    seed, gen, slot = 42, 3, 5
    mask = L.uniform_mask(seed, gen, slot, 12000)
    cases = {  # gene: (block, word, bit)
        0: (0, 0, 0), 3: (0, 0, 3), 4: (1, 0, 0), 252: (63, 0, 0), 256: (0, 0, 4),
        2047: (63, 0, 31), 2048: (0, 1, 0), 8191: (63, 3, 31), 8192: (64, 0, 0),
        8192 + 256 * 9 + 4 * 2 + 1: (66, 1, 5)}
    for i, (blk, wd, bit) in cases.items():
        w = philox.philox4x32_10(blk, slot, gen, philox.XO, seed, 0)[wd]
        assert bool((int(w) >> bit) & 1) == bool(mask[i]), i


def test_uniform_mask_neighbouring_coins_independent():
    """Fair, pairwise independent coins: neighbouring genes (distance 1, 2,
    3, 4, 256) agree half the time (binomial z-test), and the 16 patterns of
    four consecutive genes are uniform (chi-square)."""
    c = 3 * 8192 * 4
    masks = np.concatenate([L.uniform_mask(7, 11, s, c) for s in range(4)])
    n = masks.size
    assert abs(masks.sum() - n / 2) < 5 * math.sqrt(n / 4)
    for d in (1, 2, 3, 4, 256):
        agree = np.count_nonzero(masks[:-d] == masks[d:])
        m = n - d
        assert abs(agree - m / 2) < 5 * math.sqrt(m / 4), d
    q = masks[: n - n % 4].reshape(-1, 4).astype(np.int64)
    pat = q[:, 0] + 2 * q[:, 1] + 4 * q[:, 2] + 8 * q[:, 3]
    cnt = np.bincount(pat, minlength=16)
    assert stats.chisquare(cnt).pvalue > 1e-4


def test_uniform_crossover_provenance_and_mask():
    c = 20000
    rng = np.random.Generator(np.random.PCG64(4))
    pop = rng.standard_normal((3, c)).astype(F32)
    pop[0] = np.arange(1, c + 1, dtype=F32)          # sentinels
    pop[1] = -np.arange(1, c + 1, dtype=F32)
    cfg = cfg_small(pop=3, widths=(c - 1, 1), crossover="uniform")
    ops = np.array([L.CROSS, L.CROSS, L.ELITE])
    out = L.vary(pop, ops, np.array([0, 2, 2]), np.array([1, 2, 2]), cfg, 5)
    mask = L.uniform_mask(cfg.seed, 5, 0, c)
    assert np.array_equal(out[0] < 0, mask)           # read the mask back
    assert np.array_equal(out[0], np.where(mask, pop[1], pop[0]))
    assert np.array_equal(out[1], pop[2]) and np.array_equal(out[2], pop[2])
    k = mask.sum()
    assert abs(k - c / 2) < 5 * math.sqrt(c / 4)


def test_arithmetic_crossover_exact():
    rng = np.random.Generator(np.random.PCG64(6))
    pop = rng.standard_normal((2, 500)).astype(F32)
    cfg = cfg_small(pop=2, widths=(499, 1), crossover="arithmetic")
    out = L.vary(pop, np.array([L.CROSS, L.CROSS]), np.array([0, 1]), np.array([1, 1]), cfg, 1)
    exact = (pop[0].astype(np.float64) + pop[1]) / 2
    assert np.all(np.abs(out[0] - exact) <= 0.5 * np.spacing(np.abs(out[0])) + 1e-45)
    assert np.array_equal(out[1], pop[1])


# -------------------------------------------------------------- mutation ---

def test_mutation_identities():
    pop = np.random.Generator(np.random.PCG64(7)).standard_normal((1, 3000)).astype(F32)
    for kw in (dict(sigma=0.0), dict(p_gene=0.0)):
        cfg = cfg_small(pop=1, widths=(2999, 1), **kw)
        out = L.vary(pop, np.array([L.MUT]), np.array([0]), np.array([0]), cfg, 2)
        assert np.array_equal(out, pop)


def test_mutation_mask_share_and_unmutated_genes():
    c = 100000
    pop = np.ones((1, c), dtype=F32)
    cfg = cfg_small(pop=1, widths=(c - 1, 1), sigma=0.5, p_gene=0.1)
    out = L.vary(pop, np.array([L.MUT]), np.array([0]), np.array([0]), cfg, 9)
    changed = out[0] != pop[0]
    k = changed.sum()
    assert abs(k - 0.1 * c) < 5 * math.sqrt(c * 0.09)
    mutated, z = L.mutation_parts(cfg.seed, 9, 0, c, L.mutation_threshold(0.1))
    assert np.all(~changed | mutated)
    assert np.array_equal(out[0][~mutated], pop[0][~mutated])


def test_mutation_noise_is_sigma_normal():
    c = 200000
    pop = np.zeros((1, c), dtype=F32)
    sigma = 2.0 ** -10                                  # exact scaling
    cfg = cfg_small(pop=1, widths=(c - 1, 1), sigma=sigma, p_gene=1.0)
    out = L.vary(pop, np.array([L.MUT]), np.array([0]), np.array([0]), cfg, 4)
    z = out[0].astype(np.float64) / sigma
    assert abs(z.mean()) < 5 / math.sqrt(c) and abs(z.var() - 1) < 5 * math.sqrt(2 / c)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    blocks = np.arange(c // 4)
    ref = normals4(philox.draw(cfg.seed, philox.MUTNORM, 4, 0, blocks)).reshape(-1)
    assert np.array_equal(out[0], (F32(sigma) * ref).astype(F32))


def test_crossover_children_are_not_mutated():
    pop = np.random.Generator(np.random.PCG64(8)).standard_normal((1, 4000)).astype(F32)
    cfg = cfg_small(pop=1, widths=(3999, 1), sigma=1.0, p_gene=1.0)
    out = L.vary(pop, np.array([L.CROSS]), np.array([0]), np.array([0]), cfg, 1)
    assert np.array_equal(out, pop)


# ----------------------------------------------------------------- batch ---

def test_batch_indices_range_and_uniformity():
    idx = L.batch_indices(3, 7, 100000, 45000)
    assert idx.min() >= 0 and idx.max() < 45000
    h = np.bincount(idx // 450, minlength=100)
    assert stats.chisquare(h).pvalue > 1e-4
    assert np.all(L.batch_indices(3, 7, 64, 1) == 0)
    assert not np.array_equal(L.batch_indices(3, 7, 64, 1000), L.batch_indices(3, 8, 64, 1000))


# ------------------------------------------------------------------ loop ---

def test_generation_loop_invariants_and_progress():
    from paper_1806_09819_amd import datagen
    x, y = datagen.teacher_data(4000)
    cfg = cfg_small(pop=16, p_gene=0.1, sigma=0.01)
    pop, f_adj, hist = L.run(cfg, x, y, generations=4, batch=32)
    assert len(hist) == 5
    for rec in hist[1:]:
        assert np.bincount(rec["ops"], minlength=3).tolist() == [1, 8, 7]
    # elites of the last generation are bitwise the best of the previous one
    prev = L.init_population(cfg)
    for rec in hist[1:]:
        nxt = L.vary(prev, rec["ops"], rec["p1"], rec["p2"], cfg, rec["gen"])
        assert np.array_equal(nxt[0], prev[rec["order"][0]])
        prev = nxt
    assert np.array_equal(prev, pop)
