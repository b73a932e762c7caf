"""GPU parity of the fused evaluation (forward pass + Eq. 1 fitness +
accuracy) against the float64 oracle, over tile-spanning and ragged shapes,
both layer-1 schemes, the paper-scale population at every measured batch
size, and the degenerate cases."""
import numpy as np
import pytest
import torch

from gpu_helpers import (F32, batch, check_fitness, genomes_np, make_run, oracle_eval, say,
                         to_dev, to_np)
from oracle import leea as O
from paper_1806_09819_amd import presets
from paper_1806_09819_amd.leea import LeeaError

pytestmark = pytest.mark.gpu

BASE = dict(presets.SMALL)

CASES = [
    # name, widths, pop, b, oracle sample (None = all)
    ("small_cfg", (784, 32, 10), 16, 32, None),
    ("paper_b1", (784, 112, 32, 10), 1000, 1, 24),
    ("paper_b8", (784, 112, 32, 10), 1000, 8, 24),
    ("paper_b16", (784, 112, 32, 10), 40, 16, None),
    ("paper_b17", (784, 112, 32, 10), 40, 17, None),
    ("paper_b64", (784, 112, 32, 10), 1000, 64, 24),
    ("paper_b512", (784, 112, 32, 10), 1000, 512, 16),
    ("paper_net", (196, 256, 128, 64, 10), 12, 20, None),
    ("paper_net_b8", (196, 256, 128, 64, 10), 12, 8, None),
    ("single_layer", (64, 10), 8, 5, None),
    ("ragged_n1_k", (36, 20, 3), 5, 16, None),
    ("ragged_b", (48, 17, 5), 3, 65, None),
    ("two_classes", (8, 4, 2), 3, 3, None),
    ("deep", (32, 24, 20, 16, 12, 10, 8, 6, 4), 5, 40, None),
    ("wide_input_small_b", (2048, 64, 10), 4, 8, None),
    ("n1_256_small_b", (100, 256, 10), 4, 11, None),
    ("b_max_tile_edge", (52, 16, 7), 2, 128, None),
    # row-streaming layer 1 (b <= 4, n0 <= 1024), and its fall-back past 1024
    ("paper_b2", (784, 112, 32, 10), 40, 2, None),
    ("paper_b4", (784, 112, 32, 10), 1000, 4, 24),
    ("stream_ragged", (100, 20, 12, 3), 5, 3, None),
    ("stream_single_layer", (64, 10), 8, 4, None),
    ("stream_wide_input", (1024, 40, 6), 4, 2, None),
    ("wide_input_b2", (2048, 40, 6), 3, 2, None),
    # 1 KiB-row layer 1 (b <= 8, n0 <= 1024, n0 a multiple of 4): ragged row
    # groups, a partial last 256-column unit, four full units, past the
    # limit (falls back), a row the row-streaming kernel refuses (n0 = 4)
    ("rows_ragged_n1", (100, 19, 7, 3), 9, 7, None),
    ("rows_partial_unit", (260, 40, 10), 6, 6, None),
    ("rows_four_units", (1024, 33, 10), 5, 5, None),
    ("rows_past_limit", (1028, 24, 10), 4, 8, None),
    ("rows_tiny_k", (4, 6, 3), 3, 2, None),
    ("rows_paper_b5", (784, 112, 32, 10), 1000, 5, 24),
    # float32 large-batch kernel with global -> LDS staging: chunk counts
    # below, at and past a multiple of its stage count, one column tile,
    # ragged last row tiles
    ("lfw_ragged", (48, 32, 10), 7, 130, None),
    ("lfw_nt1", (64, 16, 4), 5, 100, None),
    ("lfw_wide", (1040, 64, 10), 4, 77, None),
]


def _sample(pop, k):
    if k is None or k >= pop:
        return np.arange(pop)
    rng = np.random.Generator(np.random.PCG64(pop))
    return np.unique(np.concatenate([[0, pop - 1], rng.choice(pop, k - 2, replace=False)]))


@pytest.mark.parametrize("name,widths,pop,b,k", CASES, ids=[c[0] for c in CASES])
def test_evaluate_matches_oracle(name, widths, pop, b, k):
    say("evaluate:", name, widths, "pop", pop, "b", b)
    run, ocfg = make_run(BASE, widths=widths, pop=pop, max_batch=max(b, 1), seed=5)
    x, y = batch(widths[0], b, widths[-1], 11 + b)
    f_adj, f_raw, acc = run.evaluate(to_dev(x), to_dev(y))
    torch.cuda.synchronize()
    sl = _sample(pop, k)
    g = genomes_np(run)
    f_ref, acc_ref, amb = oracle_eval(g[sl], tuple(widths), x, y)
    rel = check_fitness(to_np(f_raw)[sl], to_np(acc)[sl], f_ref, acc_ref, amb, b, name)
    assert np.array_equal(to_np(f_adj), to_np(f_raw))          # no inheritance yet
    say("  max rel fitness error %.2e" % rel)


def test_trained_like_genomes_and_nan_and_bad_labels():
    say("evaluate: scaled genomes, NaN genome, out-of-range label")
    widths = (784, 112, 32, 10)
    run, _ = make_run(BASE, widths=widths, pop=6, max_batch=40, seed=9)
    g = genomes_np(run)
    rng = np.random.Generator(np.random.PCG64(4))
    g = (g * rng.uniform(0.5, 6.0, size=(6, 1))).astype(F32)   # sharper softmax
    g[3, 1000] = np.nan
    full = np.zeros((6, run.stride), dtype=F32)
    full[:, :run.genes] = g
    run.set_state(to_dev(full))
    x, y = batch(784, 40, 10, 3)
    _, f_raw, acc = run.evaluate(to_dev(x), to_dev(y))
    f_ref, acc_ref, amb = oracle_eval(g, widths, x, y)
    assert np.isnan(f_ref[3])
    check_fitness(to_np(f_raw), to_np(acc), f_ref, acc_ref, amb, 40, "scaled")
    y_bad = y.copy()
    y_bad[7] = 10
    _, f_raw2, _ = run.evaluate(to_dev(x), to_dev(y_bad))
    assert np.all(np.isnan(to_np(f_raw2)))


def test_zero_genomes_give_minus_log_d():
    say("evaluate: zero genomes")
    run, _ = make_run(BASE, widths=(784, 112, 32, 10), pop=4, max_batch=100, seed=1)
    run.set_state(torch.zeros((4, run.stride), dtype=torch.float32, device="cuda"))
    x, y = batch(784, 100, 10, 5)
    _, f_raw, acc = run.evaluate(to_dev(x), to_dev(y))
    assert np.allclose(to_np(f_raw), -np.log(10.0), rtol=1e-6)
    assert np.all(to_np(acc) == np.float32(np.count_nonzero(y == 0) / 100))


def test_score_equals_evaluate_and_keeps_state():
    say("score")
    run, _ = make_run(BASE, widths=(784, 32, 10), pop=16, max_batch=700, seed=3)
    x, y = batch(784, 700, 10, 8)
    xs, ys = to_dev(x), to_dev(y)
    f_adj, f_raw, acc = run.evaluate(xs[:32], ys[:32])
    s_raw, s_acc = run.score(xs, ys)
    _, f_full, a_full = run.evaluate(xs, ys)
    assert torch.equal(s_raw, f_full) and torch.equal(s_acc, a_full)


def test_evaluate_is_deterministic():
    say("evaluate twice")
    run, _ = make_run(BASE, widths=(784, 112, 32, 10), pop=64, max_batch=300, seed=2)
    x, y = batch(784, 300, 10, 9)
    a = run.evaluate(to_dev(x), to_dev(y))[1].clone()
    b = run.evaluate(to_dev(x), to_dev(y))[1]
    assert torch.equal(a, b)


def test_unaligned_batch_is_rejected():
    # the kernels read the batch in 16-byte pieces; a batch at a 4-byte
    # offset is refused with LEEA_EINVAL and leaves the state untouched
    say("evaluate: batch at a 4-byte offset")
    run, _ = make_run(BASE, widths=(784, 112, 32, 10), pop=24, max_batch=200, seed=4)
    x, y = batch(784, 200, 10, 12)
    xs, ys = to_dev(x), to_dev(y)
    big = torch.empty(200 * 784 + 1, dtype=torch.float32, device="cuda")
    xu = big[1:].view(200, 784)
    xu.copy_(xs)
    assert xu.data_ptr() % 16 == 4
    before = run.score(xs, ys)[0].clone()
    for b in (3, 17, 200):
        with pytest.raises(LeeaError) as e:
            run.score(xu[:b], ys[:b])
        assert e.value.status == 1 and "aligned" in str(e.value), b
        with pytest.raises(LeeaError):
            run.evaluate(xu[:b], ys[:b])
    assert torch.equal(run.score(xs, ys)[0].view(torch.int32), before.view(torch.int32))
