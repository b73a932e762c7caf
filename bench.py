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
    """FLOPs of the first layer alone (the reduced-precision product)."""
    w = params["widths"]
    return 2.0 * w[0] * w[1] * params["pop"] * b


def vary_bytes(params, genes):
    """Algorithmic bytes of one variation launch: every child written once;
    elites and mutants read one parent, crossover children two; with a
    bfloat16 first layer at batches above 16, also each child's W_1 written
    once more in bfloat16 (the copy the evaluation reads)."""
    from paper_1806_09819_amd import leea as B
    n_e, n_c, n_m, _ = B.counts(params["pop"], params["p_elite"], params["p_cross"],
                                params["p_mut"], params["rho"])
    nbytes = 4.0 * genes * (2 * n_e + 3 * n_c + 2 * n_m)
    if params.get("eval_dtype", "f32") == "bf16" and params.get("batch", 0) > 16:
        w = params["widths"]
        nbytes += 2.0 * w[0] * w[1] * params["pop"]
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
    roof["traffic"] = (measured_traffic("paper_b%d" % b)
                       if params.get("eval_dtype", "f32") == "f32" else None)
    roof["vary_hbm_frac"] = vary_bytes(params, r["stride"]) / (r["phases_ms"]["vary"] * 1e-3) / HBM_PEAK
    roof["kernel"] = "evaluate (fused forward + fitness, one launch per generation)"
    roof["per_launch"] = dict(flops=flops, bytes=nbytes, avg_ms=r["phases_ms"]["evaluate"])
    return roof


def uneven_runs(n=64, seed=0):
    """n uneven run configs: populations log-uniform in [32, 2048], MLP
    784-h-10 with h in {16, 64, 112, 256}, batch in {8, 64, 256}, bfloat16
    first layer, the paper's other defaults; run index r, seed r."""
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


def cpu_baseline(params, b, min_seconds=12.0, max_gens=8):
    """The oracle (numpy: float64 forward and fitness, float32 genetic
    operators) running whole generations of the same workload -- rank, plan,
    vary and evaluate every slot -- until at least min_seconds have passed
    (at most max_gens generations)."""
    from oracle import leea as O
    from paper_1806_09819_amd import datagen
    import threadpoolctl

    cfg = O.Config(**{k: v for k, v in params.items() if k in O.Config.__dataclass_fields__})
    widths = tuple(params["widths"])
    c = O.param_count(widths)
    rng = np.random.Generator(np.random.PCG64(0))
    pop = (rng.standard_normal((cfg.pop, c), dtype=np.float32) * np.float32(0.05))
    f = rng.standard_normal(cfg.pop).astype(np.float32)
    info = threadpoolctl.threadpool_info()
    blas_threads = max([i.get("num_threads", 1) for i in info] or [1])
    gens = 0
    t0 = time.perf_counter()
    while gens < max_gens:
        g = gens + 1
        x, y = datagen.prototype_data(b, seed=0, sample_seed=5 + g)
        order = O.rank(f)
        ops, p1, p2, fi = O.plan(order, f, cfg, g)
        pop = O.vary(pop, ops, p1, p2, cfg, g)
        f_raw, _ = O.evaluate(pop, widths, x, y)
        f = O.inherit(f_raw, fi, cfg.alpha).astype(np.float32)
        gens += 1
        if time.perf_counter() - t0 >= min_seconds:
            break
    t1 = time.perf_counter()
    return dict(value=gens * cfg.pop * b / (t1 - t0), unit="network-sample evals/s",
                cores=int(blas_threads), kind="oracle",
                sample="%d whole generation(s) of the same workload (pop %d, batch %d, "
                       "91,866-parameter nets): rank, plan, vary and evaluate every slot, "
                       "%.1f s on the host; value = generations*pop*batch/s"
                       % (gens, cfg.pop, b, t1 - t0),
                host_cpus=len(os.sched_getaffinity(0)))


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
    ap.add_argument("--eval-dtype", default="f32", choices=("f32", "bf16", "fp8"),
                    help="arithmetic of the first layer (bf16 / fp8: reduced-precision variants)")
    ap.add_argument("--fused", action="store_true",
                    help="time the fused variation + evaluation call at batch <= 16")
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
    if args.gpus != 1:
        print("bench.py measures one GPU only: the LEEA hot path here runs on a single MI355X "
              "(multi-GPU sharding by individual is a design note, not a build target); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1806_09819_amd import datagen

    torch.cuda.init()
    data = datagen.splits("prototypes", sizes=(45000, 0, 0))
    x_train = torch.from_numpy(data["x_train"]).cuda()
    y_train = torch.from_numpy(data["y_train"]).cuda()

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
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(params, b)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
