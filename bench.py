#!/usr/bin/env python3
"""Throughput of one LEEA generation on one MI355X.

A step is one whole generation of the paper's Algorithm 1 on the device:
draw the minibatch, rank + plan, crossover/mutation into the other
population buffer, and the fused forward + fitness evaluation of all P
networks on that batch.  Workload: the paper-scale configuration (MLP
784-112-32-10, 91,866 parameters; population 1000; batch 512; section-4
default hyperparameters), synthetic prototype data resident in HBM.

Prints ONE JSON line: value = network-sample evaluations per second
(P * b * generations / s), plus the roofline of the dominant kernel
(measured with HIP events on the launch stream over the timed region) and
the CPU oracle timed on a bounded sample of the same workload.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

METRIC = "network-sample evals/s (pop×batch fwd+fitness), gens/s vs plain FP32, same acc"
HBM_PEAK = 8.0e12          # bytes/s, MI355X HBM3E
MFMA_F32_PEAK = 157.3e12   # FLOP/s, MI355X dense FP32 matrix
MFMA_PEAK = {"f32": MFMA_F32_PEAK, "bf16": 2.5e15, "fp8": 5.0e15}   # dense, per operand type


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(batch, eval_dtype="f32"):
    from paper_1806_09819_amd import presets
    p = dict(presets.PAPER)
    p["batch"] = batch
    p["eval_dtype"] = eval_dtype
    return p


OPERAND_BYTES = {"f32": 4, "bf16": 2, "fp8": 1}

# surrogate settings of the comparison run (leea_surrogate_config fields)
SURROGATE = dict(oversample=4, steps=8, lr=0.01, warmup=2, tau_min=0.1)


def algorithmic(params, genes, b):
    """Per-launch algorithmic FLOPs and HBM bytes of the evaluation kernel:
    2 * sum n_{l-1} n_l FLOPs per network-sample; every weight read once
    plus the shared batch, the first layer's weights and the batch at the
    first layer's operand size (its bfloat16 / FP8 copy), the other genes in
    float32."""
    w = params["widths"]
    per_sample = 2 * sum(w[i] * w[i + 1] for i in range(len(w) - 1))
    P = params["pop"]
    flops = float(per_sample) * P * b
    ob = OPERAND_BYTES[params.get("eval_dtype", "f32")]
    w1 = w[0] * w[1]
    nbytes = P * (ob * w1 + 4.0 * (genes - w1)) + b * (ob * w[0] + 4.0) + 8.0 * P
    return flops, nbytes


def layer1_flops(params, b):
    """FLOPs of the first layer alone (the product on the bfloat16 / FP8 matrix cores)."""
    w = params["widths"]
    return 2.0 * w[0] * w[1] * params["pop"] * b


def vary_bytes(params, genes):
    """Algorithmic bytes of one variation launch: every child written once;
    elites and mutants read one parent, crossover children two; with a
    bfloat16 or FP8 weights also each child's W_1 written once more at
    that operand size (the copy the evaluation reads)."""
    from paper_1806_09819_amd import leea as B
    n_e, n_c, n_m, _ = B.counts(params["pop"], params["p_elite"], params["p_cross"],
                                params["p_mut"], params["rho"])
    nbytes = 4.0 * genes * (2 * n_e + 3 * n_c + 2 * n_m)
    w = params["widths"]
    dt = params.get("eval_dtype", "f32")
    if dt in ("bf16", "fp8"):       # the child's W_1 copy, at its operand size
        nbytes += OPERAND_BYTES[dt] * w[0] * w[1] * params["pop"]
    return nbytes


TRAFFIC_SOURCES = ("paper_1806_09819_amd/csrc/evaluate.hip",
                   "paper_1806_09819_amd/csrc/evaluate_lpw.hip",
                   "paper_1806_09819_amd/csrc/eval_common.hpp",
                   "paper_1806_09819_amd/csrc/lp_common.hpp",
                   "paper_1806_09819_amd/csrc/reg_tail.hpp",
                   "paper_1806_09819_amd/csrc/device.hpp")


def sources_sha256(paths):
    """sha256 over the concatenated bytes of the given repository files."""
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        h.update(open(os.path.join(HERE, p), "rb").read())
    return h.hexdigest()


def measured_traffic(workload_tag):
    """HBM bytes per launch of the evaluate kernel from the committed
    rocprofv3 counter summary, or None when the kernel sources have changed
    since the counters were taken (or no record exists)."""
    path = os.path.join(HERE, "profiles", "pmc_traffic_evaluate.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if not line.startswith("{"):
            continue
        rec = json.loads(line)
        if rec.get("workload") != workload_tag:
            continue
        if rec.get("sources_sha256") != sources_sha256(rec.get("sources", ())):
            return None
        return float(rec["hbm_bytes_per_launch"])
    return None


def run_gpu(params, steps, warmup, x_train, y_train, timed_events=True, fused=False):
    """Time `steps` generations.  Variation and evaluation are timed as
    separate calls; with fused=True (b <= 16 only) the second half of the step
    is the single fused variation + evaluation call instead."""
    import torch
    from paper_1806_09819_amd import leea as B

    run = B.Leea(B.make_config(**dict(params, max_batch=params["batch"])))
    lib = B.library()
    ctx = run._ctx
    b = params["batch"]
    fused = fused and b <= 16
    xb = torch.empty((b, params["widths"][0]), dtype=torch.float32, device="cuda")
    yb = torch.empty((b,), dtype=torch.int32, device="cuda")
    P = B._ptr

    def call(st):
        if st != 0:
            raise B.LeeaError(st, lib.leea_last_error(ctx).decode())

    run.set_fused_step(fused)
    run.draw_batch(0, x_train, y_train, b, xb, yb)
    run.evaluate(xb, yb)
    gen = [0]
    names = ["batch", "select", "vary+evaluate"] if fused else ["batch", "select", "vary",
                                                                 "evaluate"]

    def one_step(ev=None):
        g = gen[0] + 1
        if ev is not None:
            ev[0].record()
        call(lib.leea_draw_batch(ctx, g, P(x_train), P(y_train), x_train.shape[0], b, P(xb),
                                 P(yb)))
        if ev is not None:
            ev[1].record()
        call(lib.leea_select(ctx, None, None, None))
        if ev is not None:
            ev[2].record()
        if fused:
            call(lib.leea_crossover_mutate_evaluate(ctx, P(xb), P(yb), b, None, None, None))
        else:
            call(lib.leea_crossover_mutate(ctx))
            if ev is not None:
                ev[3].record()
            call(lib.leea_evaluate(ctx, P(xb), P(yb), b, None, None, None))
        if ev is not None:
            ev[len(names)].record()
        gen[0] = g

    for _ in range(warmup):
        one_step()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
              for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        one_step(events[k] if timed_events else None)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases = np.zeros(len(names))
    if timed_events:
        for ev in events:
            for i in range(len(names)):
                phases[i] += ev[i].elapsed_time(ev[i + 1])
        phases /= steps
    _, f_adj = run.population()
    best = float(torch.max(torch.nan_to_num(f_adj, nan=-np.inf)).item())
    out = dict(seconds=t1 - t0, phases_ms=dict(zip(names, phases.tolist())), genes=run.genes,
               stride=run.stride, best_f_adj=best, fused=fused)
    run.close()
    return out


def fused_bytes(params, stride, b):
    """Algorithmic bytes of one fused variation + evaluation launch: every
    child written once, one parent read per elite and mutant, two per
    crossover child, and the shared batch."""
    from paper_1806_09819_amd import leea as B
    n_e, n_c, n_m, _ = B.counts(params["pop"], params["p_elite"], params["p_cross"],
                                params["p_mut"], params["rho"])
    return 4.0 * stride * (2 * n_e + 3 * n_c + 2 * n_m) + 4.0 * b * (params["widths"][0] + 1)


def roofline_of(params, r, b):
    """Roofline object of the dominant kernel of a measured run."""
    if r["fused"]:
        nbytes = fused_bytes(params, r["stride"], b)
        sec = r["phases_ms"]["vary+evaluate"] * 1e-3
        achieved = nbytes / sec / 1e9
        return dict(bound="hbm", achieved=achieved, peak=HBM_PEAK / 1e9, unit="GB/s",
                    frac=achieved / (HBM_PEAK / 1e9), traffic=None,
                    kernel="fused variation + evaluation (crossover_mutate_evaluate call)",
                    per_launch=dict(bytes=nbytes, avg_ms=r["phases_ms"]["vary+evaluate"]))
    flops, nbytes = algorithmic(params, r["genes"], b)
    sec = r["phases_ms"]["evaluate"] * 1e-3
    dt = params.get("eval_dtype", "f32")
    # reduced precision: layer 1 at its operand type's peak, the tail layers
    # at the FP32 peak; the effective peak is the total over that ideal time
    l1 = layer1_flops(params, b) if dt != "f32" else flops
    ideal = l1 / MFMA_PEAK[dt] + (flops - l1) / MFMA_F32_PEAK
    peak = flops / ideal
    if flops / nbytes > peak / HBM_PEAK:
        achieved = flops / sec / 1e12
        roof = dict(bound="mfma", achieved=achieved, peak=peak / 1e12,
                    unit="TFLOP/s", frac=achieved / (peak / 1e12))
        if dt != "f32":
            roof["peak_note"] = ("effective peak of the mix: layer 1 at %.1f TFLOP/s (%s), "
                                 "the float32 tail at %.1f" % (MFMA_PEAK[dt] / 1e12, dt,
                                                               MFMA_F32_PEAK / 1e12))
    else:
        achieved = nbytes / sec / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK / 1e9, unit="GB/s",
                    frac=achieved / (HBM_PEAK / 1e9))
    dt_tag = params.get("eval_dtype", "f32")
    roof["traffic"] = measured_traffic("paper_b%d" % b if dt_tag == "f32"
                                       else "paper_%s_b%d" % (dt_tag, b))
    roof["vary_hbm_frac"] = vary_bytes(params, r["stride"]) / (r["phases_ms"]["vary"] * 1e-3) / HBM_PEAK
    roof["kernel"] = "evaluate (fused forward + fitness, one launch per generation)"
    roof["per_launch"] = dict(flops=flops, bytes=nbytes, avg_ms=r["phases_ms"]["evaluate"])
    return roof


def uneven_runs(n=64, seed=0):
    """n uneven run configs: populations log-uniform in [32, 2048], MLP
    784-h-10 with h in {16, 64, 112, 256}, batch in {8, 64, 256}, bfloat16
    weights, the paper's other defaults; run index r, seed r."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for r in range(n):
        pop = int(round(float(np.exp(rng.uniform(np.log(32), np.log(2048))))))
        h = int(rng.choice([16, 64, 112, 256]))
        b = int(rng.choice([8, 64, 256]))
        p = workload(b, "bf16")
        p.update(widths=(784, h, 10), pop=pop, max_batch=b, seed=r, run=r)
        out.append(p)
    return out


def multi_run_bench(x_train, y_train, steps=20, warmup=3, n=64):
    """Generations of n uneven runs: grouped launches replayed from one
    captured graph, the same launches eager, and the runs stepped one by
    one through leea_step; then again after the autotuner."""
    import torch
    from paper_1806_09819_amd import leea as B

    params = uneven_runs(n)
    evals_per_gen = sum(p["pop"] * p["batch"] for p in params)

    def time_runs(runs):
        for _ in range(warmup):
            runs.generation(x_train, y_train)
        runs.sync()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(runs.stream)
        for _ in range(steps):
            runs.generation(x_train, y_train)
        e1.record(runs.stream)
        runs.sync()
        wall = time.perf_counter() - t0
        return wall / steps, e0.elapsed_time(e1) * 1e-3 / steps

    runs = B.Runs([B.make_config(**p) for p in params])
    runs.generation(x_train, y_train)
    out = {}
    for mode in ("graph", "eager"):
        runs.set_graph(mode == "graph")
        wall, dev = time_runs(runs)
        out[mode] = dict(ms_per_gen=wall * 1e3, device_ms_per_gen=dev * 1e3,
                         value=evals_per_gen / wall)
    default = [runs.shape(r) for r in range(n)]
    kind, mw, us = runs.autotune(x_train, y_train)
    runs.set_graph(True)
    wall, dev = time_runs(runs)
    out["graph_tuned"] = dict(ms_per_gen=wall * 1e3, device_ms_per_gen=dev * 1e3,
                              value=evals_per_gen / wall,
                              shapes_changed=int(sum(1 for r in range(n)
                                                     if (kind[r], mw[r]) != default[r])))
    runs.close()
    del runs
    torch.cuda.empty_cache()
    # one by one: n single-run contexts, each a leea_step per generation
    singles = [B.Leea(B.make_config(**p)) for p in params]
    xb = [torch.empty((p["batch"], 784), device="cuda") for p in params]
    yb = [torch.empty((p["batch"],), dtype=torch.int32, device="cuda") for p in params]
    for s_, p, xx, yy in zip(singles, params, xb, yb):
        s_.draw_batch(0, x_train, y_train, p["batch"], xx, yy)
        s_.evaluate(xx, yy)
    lib = B.library()

    def single_gen(g):
        for s_, p, xx, yy in zip(singles, params, xb, yb):
            s_.draw_batch(g, x_train, y_train, p["batch"], xx, yy)
            st = lib.leea_step(s_._ctx, B._ptr(xx), B._ptr(yy), p["batch"], None, None, None)
            if st != 0:
                raise B.LeeaError(st, lib.leea_last_error(s_._ctx).decode())

    for g in range(1, warmup + 1):
        single_gen(g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in range(warmup + 1, warmup + 1 + steps):
        single_gen(g)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    out["one_by_one"] = dict(ms_per_gen=wall * 1e3, value=evals_per_gen / wall)
    for s_ in singles:
        s_.close()
    out["runs"] = n
    out["network_samples_per_gen"] = evals_per_gen
    out["pops"] = [p["pop"] for p in params]
    out["hidden"] = [p["widths"][1] for p in params]
    out["batches"] = [p["batch"] for p in params]
    out["tuned_shapes"] = [[int(k), int(m)] for k, m in zip(kind, mw)]
    return out


def host_info():
    """CPU model and the BLAS threads numpy runs with (threadpoolctl)."""
    import threadpoolctl
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    info = threadpoolctl.threadpool_info()
    blas = max([i.get("num_threads", 1) for i in info] or [1])
    return model, int(blas), len(os.sched_getaffinity(0))


def cpu_baseline(params, b, sample_pop=100, reps=3):
    """The oracle (numpy: float64 forward and fitness, float32 genetic
    operators) on a bounded sample of the same workloads.  Paper scale: a
    population of `sample_pop` networks of the 784-112-32-10 workload with the
    paper's fractions, initialised by the oracle's own Glorot-uniform init;
    `evaluate` timed at b = 1, 8, 64, 512 and whole generations (rank, plan,
    vary, evaluate) at batch b, with the vary step timed on its own.  Small
    workload: all 10 generations of the 784-32-10 population of 16.  Throughput
    is network-sample evaluations per second (networks * batch / time)."""
    from oracle import leea as O
    from paper_1806_09819_amd import datagen, presets

    model, blas, host = host_info()
    out = dict(unit="network-sample evals/s", cores=blas, kind="oracle", cpu_model=model,
               host_cpus=host)
    # paper scale, sampled population
    cfg = O.Config(**{k: v for k, v in dict(params, pop=sample_pop).items()
                      if k in O.Config.__dataclass_fields__})
    widths = tuple(params["widths"])
    t0 = time.perf_counter()
    pop = O.init_population(cfg)
    t_init = time.perf_counter() - t0
    x_all, y_all = datagen.prototype_data(512 * (reps + 1), seed=0, sample_seed=5)
    evals = {}
    for bb in (1, 8, 64, 512):
        ts = []
        for r in range(reps):
            xb, yb = x_all[r * 512:r * 512 + bb], y_all[r * 512:r * 512 + bb]
            t = time.perf_counter()
            O.evaluate(pop, widths, xb, yb)
            ts.append(time.perf_counter() - t)
        evals[bb] = float(np.median(ts))
    f = O.evaluate(pop, widths, x_all[:b], y_all[:b])[0].astype(np.float32)
    t_step, t_vary = [], []
    for g in range(1, reps + 1):
        xb, yb = x_all[g * 512:g * 512 + b], y_all[g * 512:g * 512 + b]
        t = time.perf_counter()
        order = O.rank(f)
        ops, p1, p2, fi = O.plan(order, f, cfg, g)
        tv = time.perf_counter()
        pop = O.vary(pop, ops, p1, p2, cfg, g)
        t_vary.append(time.perf_counter() - tv)
        f_raw, _ = O.evaluate(pop, widths, xb, yb)
        f = O.inherit(f_raw, fi, cfg.alpha).astype(np.float32)
        t_step.append(time.perf_counter() - t)
    step = float(np.median(t_step))
    out["value"] = sample_pop * b / step
    out["paper_scale"] = dict(
        networks=sample_pop, batch_for_step=b, init_s=t_init,
        evaluate_evals_per_s={str(k): sample_pop * k / v for k, v in evals.items()},
        step_s=step, step_gens_per_s_at_pop_1000=1.0 / (step * 1000 / sample_pop),
        vary_s=float(np.median(t_vary)),
        vary_children_per_s=sample_pop / float(np.median(t_vary)))
    # small workload, every generation
    sp = dict(presets.SMALL)
    scfg = O.Config(**{k: v for k, v in sp.items() if k in O.Config.__dataclass_fields__})
    sw = tuple(sp["widths"])
    xs, ys = datagen.teacher_data(4000)
    t = time.perf_counter()
    spop = O.init_population(scfg)
    idx = O.batch_indices(scfg.seed, 0, sp["batch"], xs.shape[0])
    t_eval_small = []
    te = time.perf_counter()
    sf = O.evaluate(spop, sw, xs[idx], ys[idx])[0].astype(np.float32)
    t_eval_small.append(time.perf_counter() - te)
    for g in range(1, sp["generations"] + 1):
        idx = O.batch_indices(scfg.seed, g, sp["batch"], xs.shape[0])
        order = O.rank(sf)
        ops, p1, p2, fi = O.plan(order, sf, scfg, g)
        spop = O.vary(spop, ops, p1, p2, scfg, g)
        te = time.perf_counter()
        f_raw, _ = O.evaluate(spop, sw, xs[idx], ys[idx])
        t_eval_small.append(time.perf_counter() - te)
        sf = O.inherit(f_raw, fi, scfg.alpha).astype(np.float32)
    t_small = time.perf_counter() - t
    out["small_workload"] = dict(
        generations=sp["generations"], seconds=t_small, gens_per_s=sp["generations"] / t_small,
        evaluate_evals_per_s=sp["pop"] * sp["batch"] / float(np.median(t_eval_small)))
    out["sample"] = ("paper-scale workload on a %d-network sample (oracle Glorot init, paper "
                     "fractions): evaluate at b = 1/8/64/512 (median of %d) and %d whole "
                     "generations at batch %d (rank, plan, vary, evaluate; value = networks * "
                     "batch / step time); small workload: all %d generations of its population "
                     "of 16" % (sample_pop, reps, reps, b, sp["generations"]))
    return out


def accuracy_runs(x_train, y_train, x_val, y_val, gens=1000, every=50, batch=512,
                  seeds=(1, 2, 3)):
    """The metric's second half: the paper-scale workload (784-112-32-10,
    P = 1000, batch 512) run for `gens` generations in float32, bfloat16 and
    FP8, each from the same seeds (one run per seed and arithmetic: the
    trajectory of one run depends on every rounding, so single runs differ by
    a few points of accuracy).  Generations are timed alone (validation
    scoring every `every` generations sits outside the timed segments).
    Reported per arithmetic: generations/s, the validation accuracy (5000
    held-out samples) of the rank-0 network after the last generation (mean
    over the seeds and per seed), the mean trajectory, its largest distance
    from the float32 one, and the generations and seconds the seed-mean
    accuracy needs to come within one point of the float32 runs' final
    seed-mean accuracy."""
    import torch
    from paper_1806_09819_amd import leea as B

    out = {}
    nv = x_val.shape[0]
    for dt in ("f32", "bf16", "fp8"):
        per_seed, t_total, trajs = [], 0.0, []
        for seed in seeds:
            params = dict(workload(batch, dt), seed=seed)
            run = B.Leea(B.make_config(**dict(params, max_batch=max(batch, nv))))
            xb = torch.empty((batch, params["widths"][0]), dtype=torch.float32, device="cuda")
            yb = torch.empty((batch,), dtype=torch.int32, device="cuda")
            run.draw_batch(0, x_train, y_train, batch, xb, yb)
            run.evaluate(xb, yb)
            traj, t_gen = [], 0.0
            for g0 in range(1, gens + 1, every):
                torch.cuda.synchronize()
                t = time.perf_counter()
                for g in range(g0, min(g0 + every, gens + 1)):
                    run.draw_batch(g, x_train, y_train, batch, xb, yb)
                    run.step(xb, yb, outputs=False)
                torch.cuda.synchronize()
                t_gen += time.perf_counter() - t
                _, acc = run.score(x_val, y_val)
                _, f_adj = run.population()
                best = int(torch.argmax(torch.nan_to_num(f_adj, nan=-np.inf)).item())
                traj.append((min(g0 + every - 1, gens), t_gen, float(acc[best].item())))
            run.close()
            t_total += t_gen
            per_seed.append(traj[-1][2])
            trajs.append(traj)
        gens_per_s = gens * len(seeds) / t_total
        mean_traj = [(trajs[0][i][0], float(np.mean([tr[i][2] for tr in trajs])))
                     for i in range(len(trajs[0]))]
        out[dt] = dict(gens_per_s=gens_per_s, val_acc_rank0=float(np.mean(per_seed)),
                       val_acc_rank0_per_seed=per_seed,
                       trajectory=[[g, round(a, 4)] for g, a in mean_traj])
    # "same accuracy": within one point of the float32 runs' final seed-mean
    # accuracy (the seed means themselves spread by about that much)
    target = out["f32"]["val_acc_rank0"] - 0.01
    f32_traj = dict((g, a) for g, a in out["f32"]["trajectory"])
    for dt, r in out.items():
        hit = [g for g, a in r["trajectory"] if a >= target]
        r["gens_to_f32_final_acc"] = hit[0] if hit else None
        r["seconds_to_f32_final_acc"] = hit[0] / r["gens_per_s"] if hit else None
        r["max_abs_diff_vs_f32"] = round(max(abs(a - f32_traj[g]) for g, a in r["trajectory"]), 4)
    out["matched_accuracy_target"] = target
    out["workload"] = ("784-112-32-10, P = 1000, batch %d, %d generations, paper defaults, "
                       "prototype data (45k train, 5k validation), seeds %s"
                       % (batch, gens, list(seeds)))
    return out


def surrogate_vs_plain(gens=300, data_kind="teacher", k=4, batch=64, dtype="bf16"):
    """The surrogate's workload (784-32-10 with the small workload's operators,
    P = 1000, 4x over-generated offspring, bfloat16 weights and batch) run with
    plain LEEA and with the pre-screening surrogate from the same seed:
    generations/s, the rank-0 network's validation accuracy, and the
    surrogate's screening (generations screened, Kendall tau of its
    predictions against the evaluated fitness: mean, and share of
    generations at or above tau_min)."""
    import torch
    from paper_1806_09819_amd import datagen, presets
    from paper_1806_09819_amd import leea as B

    data = datagen.splits(data_kind, sizes=(45000, 5000, 0))
    xt, yt = torch.from_numpy(data["x_train"]).cuda(), torch.from_numpy(data["y_train"]).cuda()
    xv, yv = torch.from_numpy(data["x_val"]).cuda(), torch.from_numpy(data["y_val"]).cuda()
    params = dict(presets.SMALL, pop=1000, batch=batch, eval_dtype=dtype)
    res = {}
    for mode in ("plain", "surrogate"):
        run = B.Leea(B.make_config(**dict(params, max_batch=xv.shape[0])))
        if mode == "surrogate":
            run.attach_surrogate(**SURROGATE)
        xb = torch.empty((batch, 784), dtype=torch.float32, device="cuda")
        yb = torch.empty((batch,), dtype=torch.int32, device="cuda")
        run.draw_batch(0, xt, yt, batch, xb, yb)
        run.evaluate(xb, yb)
        stats = []
        torch.cuda.synchronize()
        t = time.perf_counter()
        for g in range(1, gens + 1):
            run.draw_batch(g, xt, yt, batch, xb, yb)
            if mode == "surrogate":
                stats.append(run.surrogate_step(xb, yb)[3])
            else:
                run.step(xb, yb, outputs=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        _, acc = run.score(xv, yv)
        _, f_adj = run.population()
        best = int(torch.argmax(torch.nan_to_num(f_adj, nan=-np.inf)).item())
        r = dict(gens_per_s=gens / dt, us_per_gen=dt / gens * 1e6,
                 val_acc_rank0=float(acc[best].item()), val_acc_best=float(acc.max().item()))
        if stats:
            st = torch.stack(stats).cpu().numpy()
            r.update(screened_generations=int(st[:, 0].sum()),
                     tau_mean=float(st[:, 1].mean()),
                     tau_share_at_min=float((st[:, 1] >= SURROGATE["tau_min"]).mean()),
                     rmse_mean=float(st[:, 2].mean()))
        res[mode] = r
        run.close()
    res["workload"] = ("784-32-10, P = 1000, batch %d, %s weights, sigma 0.01, p_gene 0.1, "
                       "truncation top 25 %%, %s data, %d generations; surrogate: %d x offspring, "
                       "%s" % (batch, dtype, data_kind, gens, k, SURROGATE))
    return res


def small_workload(steps=2000, warmup=50):
    """The small workload (784-32-10, P = 16, batch 32, its operators), which
    is launch-latency bound: microseconds per generation through leea_step
    (draw + step, eager launches) and through a one-run group replayed from a
    captured HIP graph (leea_runs)."""
    import torch
    from paper_1806_09819_amd import datagen, presets
    from paper_1806_09819_amd import leea as B

    p = dict(presets.SMALL)
    b = p["batch"]
    x, y = datagen.teacher_data(45000)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    run = B.Leea(B.make_config(**dict(p, max_batch=b)))
    lib = B.library()
    xb = torch.empty((b, 784), dtype=torch.float32, device="cuda")
    yb = torch.empty((b,), dtype=torch.int32, device="cuda")
    run.draw_batch(0, xt, yt, b, xb, yb)
    run.evaluate(xb, yb)
    P = B._ptr

    def gen(g):
        st = lib.leea_draw_batch(run._ctx, g, P(xt), P(yt), xt.shape[0], b, P(xb), P(yb))
        st = st or lib.leea_step(run._ctx, P(xb), P(yb), b, None, None, None)
        if st:
            raise B.LeeaError(st, lib.leea_last_error(run._ctx).decode())

    for g in range(1, warmup + 1):
        gen(g)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for g in range(warmup + 1, warmup + 1 + steps):
        gen(g)
    torch.cuda.synchronize()
    eager = (time.perf_counter() - t) / steps
    run.close()
    runs = B.Runs([B.make_config(**dict(p, max_batch=b))])
    runs.generation(xt, yt)
    for _ in range(warmup):
        runs.generation(xt, yt)
    runs.sync()
    t = time.perf_counter()
    for _ in range(steps):
        runs.generation(xt, yt)
    runs.sync()
    graph = (time.perf_counter() - t) / steps
    runs.close()
    return dict(workload="784-32-10, P = 16, batch 32, sigma 0.01, p_gene 0.1, truncation "
                         "top 25 %, teacher data",
                eager_us_per_gen=eager * 1e6, eager_gens_per_s=1.0 / eager,
                graph_us_per_gen=graph * 1e6, graph_gens_per_s=1.0 / graph,
                evals_per_s_graph=p["pop"] * b / graph)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--sweep-steps", type=int, default=50)
    ap.add_argument("--no-multi-run", action="store_true",
                    help="skip the 64 uneven runs measurement")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the f32 / bf16 / fp8 accuracy runs and the surrogate comparison")
    ap.add_argument("--accuracy-gens", type=int, default=1000)
    ap.add_argument("--no-small", action="store_true", help="skip the small workload")
    ap.add_argument("--eval-dtype", default="f32", choices=("f32", "bf16", "fp8"),
                    help="arithmetic of the weights and the batch (bf16 / fp8: reduced-precision "
                         "variants; activations and sums stay float32)")
    ap.add_argument("--fused", action="store_true",
                    help="time the fused variation + evaluation call at batch <= 16")
    ap.add_argument("--surrogate-only", type=int, default=0, metavar="GENS",
                    help="only time GENS surrogate generations at the surrogate's workload "
                         "(prototypes, batch 64, FP32; for kernel traces) and exit")
    ap.add_argument("--copy-calibrate", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes 5 times (scales the "
                         "FETCH_SIZE / WRITE_SIZE counters to bytes) and exit")
    args = ap.parse_args()
    if args.copy_calibrate:
        import torch
        n = args.copy_calibrate // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 4, "copies": 5}), flush=True)
        return
    if args.surrogate_only:
        r = surrogate_vs_plain(gens=args.surrogate_only, data_kind="prototypes", batch=64,
                               dtype="f32")
        print(json.dumps(r), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the LEEA hot path here runs on a single MI355X "
              "(multi-GPU sharding by individual is a design note, not a build target); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1806_09819_amd import datagen

    torch.cuda.init()
    data = datagen.splits("prototypes", sizes=(45000, 5000, 0))
    x_train = torch.from_numpy(data["x_train"]).cuda()
    y_train = torch.from_numpy(data["y_train"]).cuda()
    x_val = torch.from_numpy(data["x_val"]).cuda()
    y_val = torch.from_numpy(data["y_val"]).cuda()

    params = workload(args.batch, args.eval_dtype)
    log("bench: timed run, batch", args.batch)
    r = run_gpu(params, args.steps, args.warmup, x_train, y_train, fused=args.fused)
    P, b, K = params["pop"], args.batch, args.steps
    value = P * b * K / r["seconds"]
    roof = roofline_of(params, r, b)
    phases = {k: round(v, 4) for k, v in r["phases_ms"].items()}
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "network-sample evals/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": r["seconds"] / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.eval_dtype,
        "data": "synthetic",
        "config": {
            "workload": "paper-scale LEEA generation: MLP 784-112-32-10 (91,866 params), "
                        "population 1000, batch %d, uniform crossover, p_E/p_C/p_M "
                        "0.05/0.50/0.45, sigma 0.001, rho 0.5, alpha 1; synthetic 10-prototype "
                        "Gaussian inputs (45k train set in HBM)" % b,
            "widths": list(params["widths"]), "pop": P, "batch": b,
            "first_layer": args.eval_dtype,
            "gens_per_s": K / r["seconds"],
        },
        "phases_ms": phases,
        "roofline": roof,
    }
    if not args.no_sweep:
        sweep = []
        for bb in (1, 8, 64, 512):
            if bb == b:
                continue
            log("bench: sweep batch", bb)
            pb = workload(bb, args.eval_dtype)
            rs = run_gpu(pb, args.sweep_steps, 3, x_train, y_train, fused=args.fused)
            rf = roofline_of(pb, rs, bb)
            sweep.append(dict(batch=bb, value=P * bb * args.sweep_steps / rs["seconds"],
                              ms_per_step=rs["seconds"] / args.sweep_steps * 1e3,
                              phases_ms={k: round(v, 4) for k, v in rs["phases_ms"].items()},
                              dominant=rf["kernel"], bound=rf["bound"],
                              frac=round(rf["frac"], 4)))
        line["batch_sweep"] = sweep
    if not args.no_multi_run:
        log("bench: 64 uneven runs")
        line["multi_run"] = multi_run_bench(x_train, y_train)
    if not args.no_small:
        log("bench: small workload")
        line["small_workload"] = small_workload()
    if not args.no_accuracy:
        log("bench: accuracy runs (f32 / bf16 / fp8)")
        line["accuracy"] = accuracy_runs(x_train, y_train, x_val, y_val, gens=args.accuracy_gens)
        log("bench: surrogate vs plain")
        line["surrogate"] = {
            "teacher_b64": surrogate_vs_plain(data_kind="teacher", batch=64),
            "prototypes_b64": surrogate_vs_plain(data_kind="prototypes", batch=64),
            "prototypes_b512": surrogate_vs_plain(data_kind="prototypes", batch=512),
        }
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(params, b)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
