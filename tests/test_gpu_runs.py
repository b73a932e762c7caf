"""Many runs driven together (grouped launches replayed from a captured HIP
graph) against the same runs driven one by one through the single-run
calls, which the other GPU tests pin to the oracle: genomes and fitness
must be bitwise equal in every generation, graph or eager.  One run is also
checked against the oracle directly, and the autotuner's choices against
the default shapes."""
import numpy as np
import pytest
import torch

from gpu_helpers import F32, fit_tol, make_run, say, to_dev, to_np
from oracle import leea as O
from paper_1806_09819_amd import datagen
from paper_1806_09819_amd import leea as B
from paper_1806_09819_amd import presets

pytestmark = pytest.mark.gpu

BASE = dict(presets.PAPER)


def run_params():
    """Uneven runs: widths 784-h-10 with h in {16, 64, 112, 256}, batches
    {8, 64, 256} plus ragged ones, both crossovers and selections, float32
    and bfloat16 first layers."""
    spec = [
        (7, 16, 8, "uniform", "truncation", "bf16"),
        (33, 64, 64, "arithmetic", "tournament", "bf16"),
        (20, 112, 256, "uniform", "truncation", "bf16"),
        (9, 256, 8, "arithmetic", "truncation", "bf16"),
        (40, 112, 8, "uniform", "tournament", "f32"),
        (12, 64, 100, "uniform", "truncation", "f32"),
        (5, 16, 17, "arithmetic", "truncation", "bf16"),
        (26, 256, 64, "uniform", "truncation", "bf16"),
        (15, 64, 3, "arithmetic", "tournament", "f32"),
    ]
    out = []
    for r, (pop, h, b, xo, sel, dt) in enumerate(spec):
        out.append(dict(BASE, widths=(784, h, 10), pop=pop, batch=b, max_batch=b, crossover=xo,
                        selection=sel, eval_dtype=dt, sigma=0.01, p_gene=0.3, seed=100 + r, run=r,
                        alpha=0.5 if r % 3 == 0 else 1.0))
    return out


def _data():
    x, y = datagen.prototype_data(3000, seed=0)
    return x, y, to_dev(x), to_dev(y)


def _single_generation(run, g, xd, yd, b):
    xb, yb = run.draw_batch(g, xd, yd, b)
    if g > 0:
        run.select()
        run.crossover_mutate()
    return run.evaluate(xb, yb)


@pytest.mark.parametrize("graph", [True, False], ids=["graph", "eager"])
def test_runs_match_single_runs(graph):
    x, y, xd, yd = _data()
    params = run_params()
    runs = B.Runs([B.make_config(**p) for p in params])
    runs.set_graph(graph)
    singles = [make_run(p, max_batch=p["batch"])[0] for p in params]
    for g in range(0, 5):
        say("runs generation", g, "graph" if graph else "eager")
        runs.generation(xd, yd)
        runs.sync()
        # eager work of the program between replays
        _ = torch.ones(1024, device="cuda").sum().item()
        for r, (p, s) in enumerate(zip(params, singles)):
            f_adj, f_raw, acc = _single_generation(s, g, xd, yd, p["batch"])
            gen_r, fa_r, fr_r, ac_r = runs.population(r)
            gen_s, _ = s.population()
            c = s.genes
            assert torch.equal(gen_r[:, :c].view(torch.int32), gen_s[:, :c].view(torch.int32)), (g, r)
            for a, b_, name in ((fa_r, f_adj, "f_adj"), (fr_r, f_raw, "f_raw"), (ac_r, acc, "acc")):
                assert torch.equal(a.view(torch.int32), b_.view(torch.int32)), (g, r, name)
    assert runs.generation_count == 4
    runs.close()


def test_runs_one_run_against_oracle():
    """A float32 run inside a group, teacher-forced against the oracle."""
    x, y, xd, yd = _data()
    params = run_params()
    params[4] = dict(params[4], pop=10)
    runs = B.Runs([B.make_config(**p) for p in params])
    p = params[4]
    ocfg = O.Config(**{k: v for k, v in p.items() if k in O.Config.__dataclass_fields__})
    pop_o = O.init_population(ocfg)
    widths, b = p["widths"], p["batch"]
    f_prev = None
    for g in range(0, 4):
        runs.generation(xd, yd)
        runs.sync()
        gen_r, fa_r, fr_r, _ = runs.population(4)
        if g > 0:
            ops, p1, p2, _ = O.plan(O.rank(f_prev), f_prev, ocfg, g)
            pop_o = O.vary(pop_o, ops, p1, p2, ocfg, g)
        c = pop_o.shape[1]
        assert np.array_equal(to_np(gen_r)[:, :c].view(np.uint32), pop_o.view(np.uint32)), g
        idx = O.batch_indices(ocfg.seed, g, b, x.shape[0], ocfg.run)
        f_o, _ = O.evaluate(pop_o, widths, x[idx], y[idx])
        f = to_np(fr_r).astype(np.float64)
        assert np.all(np.abs(f - f_o) <= fit_tol(f_o)), g
        f_prev = to_np(fa_r).copy()
    runs.close()


def test_runs_autotune_choices():
    x, y, xd, yd = _data()
    params = run_params()
    runs = B.Runs([B.make_config(**p) for p in params])
    default = [runs.shape(r) for r in range(runs.n)]
    kind, mw, us = runs.autotune(xd, yd)
    say("autotune", list(zip(default, kind.tolist(), mw.tolist(), np.round(us, 1).tolist())))
    for r, p in enumerate(params):
        assert (kind[r], mw[r]) == runs.shape(r)
        assert us[r] > 0
        if p["batch"] > 16:
            assert kind[r] != 0                       # the small-batch kernel needs b <= 16
        if p["batch"] > 8:
            assert kind[r] != 4                       # the 1 KiB-row kernel needs b <= 8
        assert kind[r] in ((0, 1, 3, 4) if p["eval_dtype"] == "f32" else (0, 2, 4))
    # the tuned group still evaluates what the single runs evaluate
    runs.generation(xd, yd)
    runs.sync()
    for r, p in enumerate(params):
        s = make_run(p, max_batch=p["batch"])[0]
        _, f_raw, _ = _single_generation(s, 0, xd, yd, p["batch"])
        _, _, fr_r, _ = runs.population(r)
        a, b_ = to_np(fr_r).astype(np.float64), to_np(f_raw).astype(np.float64)
        assert np.all(np.abs(a - b_) <= 1e-6 * np.abs(b_) + 1e-7), r
    runs.close()


def test_runs_set_shape_rejects_missing_shapes():
    params = run_params()
    runs = B.Runs([B.make_config(**p) for p in params])
    with pytest.raises(B.LeeaError):
        runs.set_shape(1, 0, 1)           # b = 64 has no small-batch shape
    with pytest.raises(B.LeeaError):
        runs.set_shape(4, 2, 1)           # float32 run has no bfloat16 kernel
    with pytest.raises(B.LeeaError):
        runs.set_shape(5, 4, 1)           # b = 100 has no 1 KiB-row shape
    with pytest.raises(B.LeeaError):
        runs.set_shape(1, 4, 1)           # bfloat16 b = 64 has no 1 KiB-row shape
    assert runs.shape(0) == (4, 1)        # bfloat16 b = 8: the 1 KiB-row kernel by default
    runs.set_shape(2, 2, 1)               # b = 256: one row tile per wave exists
    assert runs.shape(2) == (2, 1)
    assert runs.shape(4) == (4, 1)        # float32 b = 8: the 1 KiB-row kernel by default
    runs.set_shape(4, 0, 1)               # ... and the small-batch kernel on request
    assert runs.shape(4) == (0, 1)
    runs.close()
