"""The fused small-batch path of leea_step (variation + evaluation in one
kernel) against the separate crossover_mutate + evaluate calls (bitwise) and
against the oracle (teacher-forced)."""
import numpy as np
import pytest
import torch

from gpu_helpers import F32, genomes_np, make_run, say, teacher_forced, to_dev, to_np
from paper_1806_09819_amd import datagen
from paper_1806_09819_amd import presets

pytestmark = pytest.mark.gpu

PAPER = dict(presets.PAPER)

CASES = [
    ("paper_b8_uniform", dict(PAPER, pop=64, batch=8)),
    ("paper_b1_arith", dict(PAPER, pop=40, batch=1, crossover="arithmetic")),
    ("paper_b16_pgene", dict(PAPER, pop=33, batch=16, p_gene=0.1, sigma=0.01)),
    ("paper_b5_selfadapt", dict(PAPER, pop=48, batch=5, sigma_mode="self_adaptive", tau=0.2,
                                sigma=0.01)),
    ("paper_b8_decay_tournament", dict(PAPER, pop=32, batch=8, sigma_mode="decay",
                                       sigma_decay_k=3.0, selection="tournament")),
    ("ragged_widths", dict(PAPER, widths=(100, 20, 12, 3), pop=24, batch=7, alpha=0.5)),
    ("small_net", dict(presets.SMALL, batch=12)),
]


@pytest.mark.parametrize("name,params", CASES, ids=[c[0] for c in CASES])
def test_fused_step_bitwise_equals_separate(name, params):
    say("fused vs separate:", name)
    n0 = params["widths"][0]
    x = datagen.uniform_inputs((3000, n0), 1)
    y = datagen.labels(3000, params["widths"][-1], 2)
    xd, yd = to_dev(x), to_dev(y)
    b = params["batch"]
    runs = []
    for fused in (True, False):
        run, _ = make_run(params, max_batch=b)
        run.set_fused_step(fused)
        xb, yb = run.draw_batch(0, xd, yd, b)
        run.evaluate(xb, yb)
        outs = []
        for g in range(1, 5):
            xb, yb = run.draw_batch(g, xd, yd, b)
            outs.append([to_np(t) for t in run.step(xb, yb)])
        runs.append((run, outs))
    (ra, oa), (rb, ob) = runs
    for ga, gb in zip(oa, ob):
        for ta, tb in zip(ga, gb):
            assert np.array_equal(ta.view(np.uint32), tb.view(np.uint32))
    assert np.array_equal(genomes_np(ra).view(np.uint32), genomes_np(rb).view(np.uint32))
    if params.get("sigma_mode") == "self_adaptive":
        assert torch.equal(ra.sigmas(), rb.sigmas())


def test_fused_teacher_forced_against_oracle():
    # b = 12: batches of at most 8 take the separate calls (1 KiB-row evaluation)
    x, y = datagen.prototype_data(3000, seed=0)
    params = dict(PAPER, pop=40, batch=12, generations=3)
    teacher_forced(params, 3, x, y, label="fused", use_step=True)
