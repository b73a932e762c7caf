"""Paper-scale chain of generations (Algorithm 1, section 3.1): the device
runs select -> crossover_mutate -> evaluate three times in a row at
P = 1000 on the 784-112-32-10 network, with fitness inheritance
(alpha = 0.5, the f_adj weighting of section 3.1) and tournament-2
selection, at a large batch (512) and a small one (8).  Each generation is
checked teacher-forced against the oracle: the plan and the inherited
fitness of every slot bit for bit, children bit for bit on sampled slots of
every operator, raw fitness of sampled networks within the fitness
tolerance, and the adjusted fitness of every slot bit for bit against the
float32 weighting of the device's raw and inherited values."""
import numpy as np
import pytest

from gpu_helpers import F32, check_fitness, genomes_np, make_run, oracle_eval, say, to_dev, to_np
from oracle import leea as O
from paper_1806_09819_amd import datagen
from paper_1806_09819_amd import presets

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("b", [512, 8])
def test_paper_scale_chain_inheritance_tournament(b):
    params = dict(presets.PAPER, batch=b, alpha=0.5, selection="tournament", tournament_k=2,
                  sigma=0.01, seed=21)
    run, ocfg = make_run(params, max_batch=b)
    widths = tuple(params["widths"])
    x, y = datagen.prototype_data(4000, seed=0)
    xd, yd = to_dev(x), to_dev(y)
    n_e, n_c, n_m, _ = O.counts(ocfg.pop, ocfg.p_elite, ocfg.p_cross, ocfg.p_mut, ocfg.rho)
    rng = np.random.Generator(np.random.PCG64(b))
    xb, yb = run.draw_batch(0, xd, yd, b)
    f_adj, f_raw, acc = run.evaluate(xb, yb)
    for g in (1, 2, 3):
        say("chain b=%d generation %d" % (b, g))
        f_prev = to_np(f_adj).copy()
        pop_prev = genomes_np(run)
        xb, yb = run.draw_batch(g, xd, yd, b)
        plan, f_inh, order = run.select()
        run.crossover_mutate()
        f_adj, f_raw, acc = run.evaluate(xb, yb)
        # rank, plan and inherited fitness of every slot
        o_order = O.rank(f_prev)
        assert np.array_equal(to_np(order), o_order), g
        ops, p1, p2, fi = O.plan(o_order, f_prev, ocfg, g)
        pl = to_np(plan)
        assert np.array_equal(pl[:, 0], ops) and np.array_equal(pl[:, 1], p1), g
        assert np.array_equal(pl[:, 2], p2), g
        assert np.array_equal(to_np(f_inh).view(np.uint32), fi.view(np.uint32)), g
        # children on sampled slots of every operator
        sample = np.unique(np.concatenate([
            [0, n_e - 1, n_e, n_e + n_c - 1, n_e + n_c, ocfg.pop - 1],
            rng.choice(ocfg.pop, 12, replace=False)]))
        kids = O.vary(pop_prev, ops, p1, p2, ocfg, g, slots=sample)
        new = genomes_np(run)
        assert np.array_equal(new[sample].view(np.uint32), kids.view(np.uint32)), g
        # raw fitness of sampled networks on this generation's batch
        idx = O.batch_indices(ocfg.seed, g, b, x.shape[0], ocfg.run)
        assert np.array_equal(to_np(xb), x[idx]) and np.array_equal(to_np(yb), y[idx])
        fo, acc_o, amb = oracle_eval(new[sample], widths, x[idx], y[idx])
        err = check_fitness(to_np(f_raw)[sample], to_np(acc)[sample], fo, acc_o, amb, b,
                            "chain b=%d gen%d" % (b, g))
        say("  worst relative fitness error", err)
        # adjusted fitness of every slot: fl(fl((1 - alpha) f_inh) + fl(alpha f_raw))
        fa_o = O.inherit_f32(to_np(f_raw), to_np(f_inh), ocfg.alpha)
        assert np.array_equal(to_np(f_adj).view(np.uint32), fa_o.view(np.uint32)), g
    run.close()
