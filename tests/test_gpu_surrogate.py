"""GPU parity of the fitness surrogate against the oracle, teacher-forced
with the device's float32 fitness and MLP parameters each generation:
candidate plans, candidate genomes, screening and the new population
bit-exact; features, predictions, the training step and Kendall tau
within tolerances derived from float32 accumulation.  A longer run at the
surrogate's configuration (784-32-10, P = 1000, b = 64) reports its
screening error and accuracy next to plain LEEA."""
import numpy as np
import pytest
import torch

from gpu_helpers import (F32, check_fitness, fit_tol, genomes_np, make_run,
                         oracle_eval, say, to_dev, to_np)
from oracle import leea as O
from oracle import surrogate as S
from oracle.precision import round_bf16
from paper_1806_09819_amd import datagen
from paper_1806_09819_amd import presets

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def check_inputs(Xd, Zd, label):
    """The device's MLP inputs against the oracle's (standardisation, then
    the projection block times 2^-4) of the device's own features, within
    the float32 error of the fixed-order sums (depth M / 256 + 8) and of
    x - mean, scaled like the inputs."""
    M = Xd.shape[0]
    Zo = S.mlp_inputs(Xd)
    mu = Xd.mean(axis=0)
    sd = np.sqrt(((Xd - mu) ** 2).mean(axis=0))
    depth = M / 256.0 + 16.0
    ok = sd > 0
    wgt = np.ones(Xd.shape[1])
    wgt[:S.FEATURES] = 1.0 / 16.0
    scale = np.abs(Xd).mean(axis=0) + np.abs(Xd - mu)
    tol = np.where(ok, 4 * depth * U * (wgt * scale / np.where(ok, sd, 1.0) + np.abs(Zo)),
                   0.0) + 1e-6
    assert np.all(np.abs(Zd - Zo) <= tol), (label, float(np.max(np.abs(Zd - Zo) - tol)))


def _teacher_forced(params, gens, k, steps, lr, warmup, tau_min, seed=0):
    b = params["batch"]
    run, ocfg = make_run(params, max_batch=b)
    run.attach_surrogate(oversample=k, steps=steps, lr=lr, warmup=warmup, tau_min=tau_min)
    widths = tuple(params["widths"])
    g_genes = O.param_count(widths)
    x, y = datagen.prototype_data(2000, seed=seed) if widths[0] == 784 else (
        datagen.uniform_inputs((2000, widths[0]), seed), datagen.labels(2000, widths[-1], seed + 1))
    xd, yd = to_dev(x), to_dev(y)
    R = S.projection_signs(g_genes, ocfg.seed, ocfg.run)
    n_e, n_c, n_m, _ = O.counts(ocfg.pop, ocfg.p_elite, ocfg.p_cross, ocfg.p_mut, ocfg.rho)
    pop_o = O.init_population(ocfg)
    xb, yb = run.draw_batch(0, xd, yd, b)
    f_adj, _, _ = run.evaluate(xb, yb)
    used = []
    for g in range(1, gens + 1):
        say("surrogate generation", g)
        f_prev = to_np(f_adj).copy()
        views0 = run.surrogate_views()
        prm0 = to_np(views0["params"]).copy()
        xb, yb = run.draw_batch(g, xd, yd, b)
        f_adj, f_raw, acc, stats = run.surrogate_step(xb, yb)
        v = run.surrogate_views()
        st = to_np(stats)
        used.append(int(st[0]))
        # candidate plan and genomes: bit-exact
        order = O.rank(f_prev)
        ops, p1, p2, _ = S.candidate_plan(order, f_prev, ocfg, g, k)
        plan = to_np(v["plan"])
        assert np.array_equal(plan[:, 0], ops) and np.array_equal(plan[:, 1], p1), g
        assert np.array_equal(plan[:, 2], p2), g
        kids = S.candidates(pop_o, ops, p1, p2, ocfg, g)
        assert np.array_equal(to_np(v["candidates"])[:, :g_genes].view(np.uint32),
                              kids.view(np.uint32)), g
        # features within the float32 accumulation bound
        X = S.features(kids, pop_o[p1], f_prev[p1], f_prev[p2], R)
        Xd = to_np(v["features"])[:, :S.INPUTS].astype(np.float64)
        mag = (np.abs(round_bf16(kids).astype(np.float64)).sum(axis=1)
               * float(S.scale(g_genes)))[:, None]
        nchunks = (g_genes + 31) // 32
        bound = (nchunks + 40) * U * mag + 2 * U * np.abs(X[:, :256]) + 1e-30
        assert np.all(np.abs(Xd[:, :256] - X[:, :256]) <= bound), g
        assert np.array_equal(Xd[:, 256:258], X[:, 256:258]), g
        assert np.allclose(Xd[:, 258], X[:, 258], rtol=1e-5, atol=1e-9), g
        # standardised inputs, then predictions from the device's inputs and
        # parameters
        Zd = to_np(v["inputs"])[:, :S.INPUTS].astype(np.float64)
        check_inputs(Xd, Zd, g)
        prm = {"W1": prm0[:64 * 259].reshape(64, 259), "b1": prm0[64 * 259:64 * 260],
               "w2": prm0[64 * 260:64 * 261], "b2": prm0[64 * 261]}
        pred_o, _ = S.mlp_forward(prm, Zd)
        pred = to_np(v["pred"]).astype(np.float64)
        scl = np.abs(Zd) @ np.abs(prm["W1"].astype(np.float64)).T
        pbound = 600 * U * (np.maximum(scl, 1e-30) @ np.abs(prm["w2"].astype(np.float64))) + 1e-6
        assert np.all(np.abs(pred - pred_o) <= pbound), g
        # screening (device float32 predictions) and the new population
        keep = S.screen(to_np(v["pred"]), ocfg.pop - n_e, bool(st[0]), k, n_c, n_m)
        assert np.array_equal(to_np(v["chosen"]), keep), g
        new_o = np.concatenate([pop_o[order[:n_e]], kids[keep]])
        assert np.array_equal(genomes_np(run).view(np.uint32), new_o.view(np.uint32)), g
        idx = O.batch_indices(ocfg.seed, g, b, x.shape[0], ocfg.run)
        fo, _ = O.evaluate(new_o, widths, x[idx], y[idx])
        fr = to_np(f_raw).astype(np.float64)
        assert np.all(np.abs(fr - fo) <= fit_tol(fo)), g
        # judge and training
        yk = to_np(f_raw)[n_e:].astype(np.float64)
        cp = to_np(v["chosen_pred"]).astype(np.float64)
        assert abs(S.kendall_tau_a(cp, yk) - float(st[1])) < 1e-6, g
        p_o = prm
        for _ in range(steps):
            p_o = S.mlp_gradient_step(p_o, Zd[keep], S.standardize_targets(yk), lr)
        prm1 = to_np(v["params"]).astype(np.float64)
        ref = np.concatenate([p_o["W1"].ravel(), p_o["b1"], p_o["w2"], [p_o["b2"]]])
        assert np.allclose(prm1, ref, rtol=2e-4, atol=2e-6), (g, np.max(np.abs(prm1 - ref)))
        pop_o = new_o
    return used


def test_surrogate_teacher_forced_small():
    params = dict(presets.PAPER, widths=(96, 24, 5), pop=30, batch=16, sigma=0.05, p_gene=0.5,
                  seed=4)
    used = _teacher_forced(params, gens=5, k=3, steps=3, lr=0.05, warmup=1, tau_min=-1.0)
    assert used[0] == 0 and all(u == 1 for u in used[1:])      # off for warm-up, then on


def test_surrogate_teacher_forced_arithmetic_tournament():
    params = dict(presets.PAPER, widths=(100, 20, 12, 3), pop=23, batch=33, sigma=0.02,
                  crossover="arithmetic", selection="tournament", alpha=0.5, seed=5)
    used = _teacher_forced(params, gens=3, k=2, steps=2, lr=0.02, warmup=0, tau_min=0.0)
    assert len(used) == 3


def test_surrogate_teacher_forced_configured_size():
    """The surrogate's own configuration: 784-32-10, P = 1000, b = 64, k = 4,
    so M = 4 * 950 = 3800 candidates of 25,450 genes, a 4096-key screen and
    the projection split the launch takes at that size.  Two generations,
    teacher-forced with the device's population, fitness and MLP parameters
    (generation 1 keeps plain LEEA's mix, generation 2 screens): candidate
    plan, screen (chosen set and order) and the gathered population
    bit-exact in full; candidate genomes bit-exact on sampled candidates;
    features on those, predictions on all 3800 within float32 bounds;
    fitness of sampled networks within the fitness tolerance; Kendall tau
    and the training step as in the small tests."""
    params = dict(presets.SMALL, pop=1000, batch=64)
    k, steps, lr, warmup, tau_min = 4, 2, 0.01, 1, -1.0
    b = params["batch"]
    run, ocfg = make_run(params, max_batch=b)
    run.attach_surrogate(oversample=k, steps=steps, lr=lr, warmup=warmup, tau_min=tau_min)
    widths = tuple(params["widths"])
    g_genes = O.param_count(widths)
    x, y = datagen.teacher_data(4000)
    xd, yd = to_dev(x), to_dev(y)
    R = S.projection_signs(g_genes, ocfg.seed, ocfg.run)
    n_e, n_c, n_m, _ = O.counts(ocfg.pop, ocfg.p_elite, ocfg.p_cross, ocfg.p_mut, ocfg.rho)
    N, M, kc = ocfg.pop - n_e, k * (ocfg.pop - n_e), k * n_c
    assert (M, kc) == (3800, 2000)
    thr = O.mutation_threshold(ocfg.p_gene)
    rng = np.random.Generator(np.random.PCG64(11))
    xb, yb = run.draw_batch(0, xd, yd, b)
    f_adj, _, _ = run.evaluate(xb, yb)
    for g in (1, 2):
        say("configured-size surrogate generation", g)
        f_prev = to_np(f_adj).copy()
        pop_prev = genomes_np(run)
        prm0 = to_np(run.surrogate_views()["params"]).copy()
        xb, yb = run.draw_batch(g, xd, yd, b)
        f_adj, f_raw, acc, stats = run.surrogate_step(xb, yb)
        v = run.surrogate_views()
        st = to_np(stats)
        assert int(st[0]) == (0 if g == 1 else 1), (g, st)
        order = O.rank(f_prev)
        ops, p1, p2, _ = S.candidate_plan(order, f_prev, ocfg, g, k)
        plan = to_np(v["plan"])
        assert np.array_equal(plan[:, 0], ops) and np.array_equal(plan[:, 1], p1), g
        assert np.array_equal(plan[:, 2], p2), g
        cand = to_np(v["candidates"])[:, :g_genes]
        sample = np.unique(np.concatenate([
            [0, 1, kc - 1, kc, kc + 1, M - 2, M - 1],
            rng.choice(M, 25, replace=False)]))
        kids = np.stack([O._child(pop_prev, ops, p1, p2, ocfg, g, F32(ocfg.sigma), thr, int(c),
                                  g_genes, slot=ocfg.pop + int(c)) for c in sample])
        assert np.array_equal(cand[sample].view(np.uint32), kids.view(np.uint32)), g
        X = S.features(kids, pop_prev[p1[sample]], f_prev[p1[sample]], f_prev[p2[sample]], R)
        Xd_all = to_np(v["features"])[:, :S.INPUTS].astype(np.float64)
        Xd = Xd_all[sample]
        mag = (np.abs(round_bf16(kids).astype(np.float64)).sum(axis=1)
               * float(S.scale(g_genes)))[:, None]
        nchunks = (g_genes + 31) // 32
        bound = (nchunks + 40) * U * mag + 2 * U * np.abs(X[:, :256]) + 1e-30
        assert np.all(np.abs(Xd[:, :256] - X[:, :256]) <= bound), g
        assert np.array_equal(Xd[:, 256:258], X[:, 256:258]), g
        assert np.allclose(Xd[:, 258], X[:, 258], rtol=1e-5, atol=1e-9), g
        Zd_all = to_np(v["inputs"])[:, :S.INPUTS].astype(np.float64)
        check_inputs(Xd_all, Zd_all, g)
        prm = {"W1": prm0[:64 * 259].reshape(64, 259), "b1": prm0[64 * 259:64 * 260],
               "w2": prm0[64 * 260:64 * 261], "b2": prm0[64 * 261]}
        pred_o, _ = S.mlp_forward(prm, Zd_all)
        pred = to_np(v["pred"]).astype(np.float64)
        scl = np.abs(Zd_all) @ np.abs(prm["W1"].astype(np.float64)).T
        pbound = 600 * U * (np.maximum(scl, 1e-30) @ np.abs(prm["w2"].astype(np.float64))) + 1e-6
        assert np.all(np.abs(pred - pred_o) <= pbound), g
        keep = S.screen(to_np(v["pred"]), N, bool(st[0]), k, n_c, n_m)
        chosen = to_np(v["chosen"])
        assert np.array_equal(chosen, keep), g
        if g == 2:
            assert not np.array_equal(keep, S.screen(None, N, False, k, n_c, n_m))
        new = genomes_np(run)
        assert np.array_equal(new[:n_e].view(np.uint32), pop_prev[order[:n_e]].view(np.uint32)), g
        assert np.array_equal(new[n_e:].view(np.uint32), cand[chosen].view(np.uint32)), g
        for i, c in enumerate(sample):
            hit = np.nonzero(chosen == c)[0]
            if hit.size:
                assert np.array_equal(new[n_e + hit[0]].view(np.uint32), kids[i].view(np.uint32))
        idx = O.batch_indices(ocfg.seed, g, b, x.shape[0], ocfg.run)
        rows = np.unique(np.concatenate([[0, n_e - 1, n_e, ocfg.pop - 1],
                                         rng.choice(ocfg.pop, 28, replace=False)]))
        fo, acc_o, amb = oracle_eval(new[rows], widths, x[idx], y[idx])
        check_fitness(to_np(f_raw)[rows], to_np(acc)[rows], fo, acc_o, amb, b,
                      "configured surrogate gen%d" % g)
        yk = to_np(f_raw)[n_e:].astype(np.float64)
        cp = to_np(v["chosen_pred"]).astype(np.float64)
        assert abs(S.kendall_tau_a(cp, yk) - float(st[1])) < 1e-6, g
        p_o = prm
        for _ in range(steps):
            p_o = S.mlp_gradient_step(p_o, Zd_all[keep], S.standardize_targets(yk), lr)
        prm1 = to_np(v["params"]).astype(np.float64)
        ref = np.concatenate([p_o["W1"].ravel(), p_o["b1"], p_o["w2"], [p_o["b2"]]])
        assert np.allclose(prm1, ref, rtol=2e-4, atol=2e-6), (g, np.max(np.abs(prm1 - ref)))
    run.close()


def test_surrogate_report_small_config_at_scale():
    """784-32-10, P = 1000, b = 64, k = 4: surrogate screening error over
    20 generations and the best network's validation accuracy against
    plain LEEA from the same seed, once with the tau gate (tau_min = 0.1)
    and once with screening forced on after the warm-up (tau_min = -1).
    Every generation's flag must follow the documented rule: screened
    exactly when the MLP had trained for `warmup` generations and the
    previous generation's tau reached tau_min."""
    data = datagen.splits("teacher", sizes=(20000, 2000, 0))
    xt, yt = to_dev(data["x_train"]), to_dev(data["y_train"])
    xv, yv = to_dev(data["x_val"]), to_dev(data["y_val"])
    params = dict(presets.SMALL, pop=1000, batch=64, sigma=0.01, p_gene=0.1)
    gens, warmup = 20, 2
    out = {}
    for mode, tau_min in (("plain", None), ("gated", 0.1), ("forced", -1.0)):
        run, _ = make_run(params, max_batch=max(64, xv.shape[0]))
        if tau_min is not None:
            run.attach_surrogate(oversample=4, steps=8, lr=0.01, warmup=warmup, tau_min=tau_min)
        xb, yb = run.draw_batch(0, xt, yt, 64)
        run.evaluate(xb, yb)
        stats = []
        for g in range(1, gens + 1):
            xb, yb = run.draw_batch(g, xt, yt, 64)
            if tau_min is not None:
                _, _, _, st = run.surrogate_step(xb, yb)
                stats.append(to_np(st).astype(np.float64).copy())
            else:
                run.step(xb, yb)
        f_raw, acc = run.score(xv, yv)
        _, f_adj = run.population()
        best = int(torch.argmax(f_adj).item())
        rec = dict(val_acc_best=float(to_np(acc)[best]), val_acc_max=float(to_np(acc).max()))
        if stats:
            st = np.array(stats)
            used, tau, rmse, trained = st[:, 0], st[:, 1], st[:, 2], st[:, 3]
            assert np.array_equal(trained, np.arange(1, gens + 1)), (mode, trained)
            rule = np.zeros(gens)
            rule[1:] = (trained[:-1] >= warmup) & (tau[:-1] >= tau_min)
            assert np.array_equal(used, rule), (mode, used, tau)
            assert np.all(np.isfinite(tau)) and np.all(np.abs(tau) <= 1.0), (mode, tau)
            assert np.all(np.isfinite(rmse)) and np.all(rmse >= 0.0), (mode, rmse)
            rec.update(tau_mean=float(tau.mean()), tau_last5=float(tau[-5:].mean()),
                       rmse_last5=float(rmse[-5:].mean()), screened_generations=int(used.sum()))
        out[mode] = rec
        run.close()
    say("surrogate report", out)
    assert out["forced"]["screened_generations"] == gens - warmup
