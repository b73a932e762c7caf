"""Shared helpers of the GPU parity tests (inputs, oracle comparisons)."""
import sys

import numpy as np
import torch

from oracle import leea as O
from paper_1806_09819_amd import datagen
from paper_1806_09819_amd import leea as B

F32 = np.float32
DEV = "cuda"
FIT_RTOL = 1e-5      # fitness tolerance relative to the float64 oracle
FIT_ATOL = 1e-6      # absolute floor, only for fitness values below FIT_ABS_BELOW
FIT_ABS_BELOW = 0.1  # |f| below which float32 log-softmax loses log(1 + t) terms outright


def fit_tol(f_ref, rtol=FIT_RTOL):
    """Allowed |f_gpu - f_ref|: rtol |f_ref|, plus FIT_ATOL where |f_ref| <
    FIT_ABS_BELOW (a network that fits its batch almost perfectly: its
    per-sample log-likelihoods are -log(1 + t) with t below float32's
    resolution, which the float32 softmax rounds to 0; relative error cannot
    bound that)."""
    a = np.abs(np.asarray(f_ref, dtype=np.float64))
    return rtol * a + np.where(a < FIT_ABS_BELOW, FIT_ATOL, 0.0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to(DEV)


def to_np(t, dtype=None):
    a = t.detach().cpu().numpy()
    if dtype is not None:
        a = a.view(dtype)
    return a


def oracle_cfg(params, **kw):
    d = dict(params)
    d.update(kw)
    keep = {f for f in O.Config.__dataclass_fields__}
    return O.Config(**{k: v for k, v in d.items() if k in keep})


def make_run(params, **kw):
    d = dict(params)
    d.update(kw)
    return B.Leea(B.make_config(**d)), oracle_cfg(d)


def genomes_np(run):
    g, _ = run.population()
    return to_np(g)[:, :run.genes].copy()


def batch(n0, b, d, seed):
    x = datagen.uniform_inputs((b, n0), seed)
    y = datagen.labels(b, d, seed + 1)
    return x, y


def oracle_eval(rows, widths, x, y):
    """float64 fitness, accuracy and, per network, the number of samples
    whose top-two logits are too close for float32 to decide the argmax."""
    f = np.empty(len(rows))
    acc = np.empty(len(rows))
    amb = np.empty(len(rows), dtype=np.int64)
    for i, g in enumerate(rows):
        z = O.forward(g, widths, x)
        f[i], acc[i] = O.fitness_from_logits(z, y)
        s = np.sort(z, axis=1)
        gap = s[:, -1] - s[:, -2]
        amb[i] = np.count_nonzero(gap < 1e-4 * (1.0 + np.abs(s[:, -1])))
    return f, acc, amb


def check_fitness(f_gpu, acc_gpu, f_ref, acc_ref, amb, b, label=""):
    f_gpu = np.asarray(f_gpu, dtype=np.float64)
    nan_ref = np.isnan(f_ref)
    assert np.array_equal(np.isnan(f_gpu), nan_ref), label
    ok = ~nan_ref
    err = np.abs(f_gpu[ok] - f_ref[ok])
    tol = fit_tol(f_ref[ok])
    assert np.all(err <= tol), (label, float(np.max(err / np.maximum(np.abs(f_ref[ok]), 1e-30))))
    dc = np.abs(np.rint(np.asarray(acc_gpu, dtype=np.float64) * b) - np.rint(acc_ref * b))
    assert np.all(dc[ok] <= amb[ok]), (label, dc.max())
    return float(np.max(err / np.maximum(np.abs(f_ref[ok]), 1e-30))) if ok.any() else 0.0


def teacher_forced(params, gens, x, y, check_every=1, label="", use_step=False):
    """Run `gens` generations on the device and, teacher-forced with the
    device's float32 adjusted fitness, in the oracle; assert plans, sigma
    genes and genomes bit-exact and fitness within tolerance each generation.
    use_step: the second half of each generation is one
    crossover_mutate_evaluate call with the fused small-batch path allowed.
    x is the raw training set (pooled on the way when params['pool'] == 2)."""
    from oracle import leea as O
    b = params["batch"]
    run, ocfg = make_run(params, max_batch=b)
    if use_step:
        run.set_fused_step(True)
    widths = tuple(params["widths"])
    mode = params.get("sigma_mode", "constant")
    side = int(round(np.sqrt(x.shape[1]))) if params.get("pool", 0) else 0
    xd, yd = to_dev(x), to_dev(y)

    def obatch(g):
        idx = O.batch_indices(ocfg.seed, g, b, x.shape[0], ocfg.run)
        xb = x[idx]
        return (O.pool2x2(xb, side) if side else xb), y[idx]

    pop_o = O.init_population(ocfg)
    assert np.array_equal(genomes_np(run), pop_o)
    sig_o = np.full(run.pop, F32(params["sigma"]), dtype=F32)
    xb, yb = run.draw_batch(0, xd, yd, b)
    xo, yo = obatch(0)
    assert np.array_equal(to_np(xb), xo)
    f_adj, f_raw, acc = run.evaluate(xb, yb)
    f_o, acc_o, amb = oracle_eval(pop_o, widths, xo, yo)
    check_fitness(to_np(f_raw), to_np(acc), f_o, acc_o, amb, b, label + " gen0")
    for g in range(1, gens + 1):
        say(label, "generation", g)
        f_prev = to_np(f_adj).copy()
        xb, yb = run.draw_batch(g, xd, yd, b)
        plan, f_inh, order = run.select()
        if use_step:
            f_adj, f_raw, acc = run.crossover_mutate_evaluate(xb, yb)
        else:
            run.crossover_mutate()
            f_adj, f_raw, acc = run.evaluate(xb, yb)
        ops, p1, p2, fi = O.plan(O.rank(f_prev), f_prev, ocfg, g)
        pl = to_np(plan)
        assert np.array_equal(pl[:, 1], p1) and np.array_equal(pl[:, 2], p2), g
        if mode == "self_adaptive":
            sig_o = O.child_sigmas(sig_o, ops, p1, p2, ocfg, g)
            assert np.array_equal(to_np(run.sigmas()).view(np.uint32), sig_o.view(np.uint32)), g
            pop_o = O.vary_adaptive(pop_o, sig_o, ops, p1, p2, ocfg, g)
        else:
            sigma = O.sigma_decay(ocfg.sigma, g, ocfg.sigma_decay_k) if mode == "decay" else None
            pop_o = O.vary(pop_o, ops, p1, p2, ocfg, g, sigma=sigma)
        assert np.array_equal(genomes_np(run).view(np.uint32), pop_o.view(np.uint32)), g
        if g % check_every == 0 or g == gens:
            xo, yo = obatch(g)
            f_o, acc_o, amb = oracle_eval(pop_o, widths, xo, yo)
            check_fitness(to_np(f_raw), to_np(acc), f_o, acc_o, amb, b, "%s gen%d" % (label, g))
    return run
