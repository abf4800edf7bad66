"""Benchmark: GAME training generations on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: 200,000 patterns x 20 features (mixture of three Gaussians clipped
to [-1, 1]), Legendre expansion of degree 8 (161 genes), population 2,048,
regression target; synthetic, seeded.  One step is one generation of the
training loop: fitness of the whole population over all patterns, ranking
and stop test, and the genetic step (elitism, tournament, crossover,
mutation).  Inputs are resident in GPU memory before timing starts.

Prints one JSON line with whole-job throughput (chromosome x pattern
evaluations per second), the fitness kernel's position on the MFMA roofline
(timed with HIP events on the library's stream), and the CPU oracle timed on
a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "chromosome×pattern evals/s (% MFMA peak); time-to-target MSE, plain vs chosen"
FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0


def profiled_traffic(summary):
    """HBM bytes per launch recorded in a committed rocprofv3 summary
    (FETCH_SIZE and WRITE_SIZE scaled by the copy calibration), or None when
    the summary is missing or the kernel's sources changed since it was
    taken."""
    try:
        text = open(os.path.join(ROOT, "profiles", summary)).read()
    except OSError:
        return None
    fields = dict(re.findall(r"^(traffic_bytes_per_launch|kernel_sources|kernel_sources_sha256): "
                             r"(.+)$", text, re.M))
    if len(fields) != 3:
        return None
    h = hashlib.sha256()
    try:
        for f in fields["kernel_sources"].split():
            h.update(open(os.path.join(ROOT, f), "rb").read())
    except OSError:
        return None
    if h.hexdigest()[:16] != fields["kernel_sources_sha256"].strip():
        return None
    return float(fields["traffic_bytes_per_launch"])


def log(msg):
    """Progress on stderr; stdout carries only the result line."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(prob, P, seconds=10.0):
    """The oracle on the host: float64 fitness (expansion then a BLAS
    product) of a 128-chromosome batch over every pattern, repeated for about
    `seconds`, plus one oracle genetic step of the whole population; scaled
    to one generation."""
    from oracle import ga as oga
    from oracle import game as og
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    rng = np.random.default_rng(1)
    batch = 128
    W = rng.uniform(-1, 1, (batch, prob.n_genes)).astype(np.float32)
    n_batches = 0
    t0 = time.perf_counter()
    while True:
        og.fitness(prob.X, prob.t, W, prob.basis, prob.degree)
        n_batches += 1
        if time.perf_counter() - t0 >= seconds:
            break
    t_fit = (time.perf_counter() - t0) / n_batches
    pop = rng.uniform(-1, 1, (P, prob.n_genes)).astype(np.float32)
    fit = rng.uniform(0, 1, P).astype(np.float32)
    t1 = time.perf_counter()
    oga.ga_next(pop, fit, 1, oga.GAConfig(population=P))
    t_ga = time.perf_counter() - t1
    t_gen = t_fit * (P / batch) + t_ga
    return {"value": P * prob.n_patterns / t_gen, "unit": "evals/s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"{n_batches} float64 fitness batches of {batch} chromosomes x "
                      f"{prob.n_patterns} patterns ({t_fit:.2f} s each) + one genetic step of "
                      f"{P} x {prob.n_genes} genes ({t_ga:.2f} s); scaled to one generation "
                      f"of {P} chromosomes"}


def cpu_serial(prob, seconds=5.0):
    """The oracle's plain serial C fitness (one thread, one term at a time:
    the counterpart of the paper's serial version) on chromosomes of the
    workload over every pattern, for about `seconds`; evals/s."""
    from oracle import serial
    rng = np.random.default_rng(2)
    W = rng.uniform(-1, 1, (1, prob.n_genes)).astype(np.float32)
    n = 0
    t0 = time.perf_counter()
    while True:
        serial.fitness(prob.X, prob.t, W, prob.basis, prob.degree)
        n += 1
        if time.perf_counter() - t0 >= seconds:
            break
    el = time.perf_counter() - t0
    return {"value": n * prob.n_patterns / el, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} chromosomes x {prob.n_patterns} patterns, serial C float64 "
                      f"({el / n:.2f} s each)"}


def time_median(fn, stream, reps=25, warmup=3):
    """Median duration (s) of `reps` calls of fn(), each bracketed by its own
    pair of HIP events on `stream` (the stream the library queues on), after
    `warmup` untimed calls.  After an idle moment the GPU clock needs about
    20 ms of sustained load to come back up (a fitness launch then runs up
    to 20 % slower), so the fitness timings warm up for longer than that."""
    import torch
    for _ in range(warmup):
        fn()
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
             for _ in range(reps)]
    for e0, e1 in pairs:
        e0.record(stream)
        fn()
        e1.record(stream)
    pairs[-1][1].synchronize()
    return float(np.median([e0.elapsed_time(e1) for e0, e1 in pairs])) / 1e3


def time_fitness(gg, game, genes, n, reps, stream):
    """Median duration (s) of one fitness launch (plus its few-microsecond
    finish kernel) on the library's stream, HIP events around each launch,
    after 30 untimed launches."""
    import torch
    f32 = torch.empty(n, dtype=torch.float32, device=genes.device)
    return time_median(lambda: gg.game_fitness(game.h, genes, n, f32), stream, reps=max(20, reps),
                       warmup=30)


def time_steps(game, steps, warmup):
    import torch
    for _ in range(warmup):
        game.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        game.step()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def precision_problem():
    """The precision problem with its training and validation sets resident
    on the GPU."""
    import torch
    from paper_1304_0597_amd import datagen
    prob = datagen.precision()
    dev = torch.device("cuda:0")
    prob.X_dev, prob.t_dev = torch.from_numpy(prob.X).to(dev), torch.from_numpy(prob.t).to(dev)
    prob.Xv_dev = torch.from_numpy(prob.X_val).to(dev)
    prob.tv_dev = torch.from_numpy(prob.t_val).to(dev)
    return prob


def form_bf16(gg, prob, steps, warmup):
    """Precision form: 1,000,000 patterns x 32 features, Chebyshev degree 8
    (257 genes), population 4,096, BF16 operands with FP32 accumulation; the
    error of the BF16 fitness against the float64 re-score of a sample."""
    import torch
    P = prob.population
    dev = torch.device("cuda:0")
    cfg = gg.config(basis=prob.basis, degree=prob.degree, population=P, precision=gg.GAME_BF16,
                    seed=0, max_generations=1 << 30, target=-1.0)
    game = gg.Game(cfg, prob.X_dev, prob.t_dev)
    game.init_population()
    stream = torch.cuda.current_stream()
    elapsed = time_steps(game, steps, warmup)
    pop, _ = game.population()
    t_kernel = time_fitness(gg, game, pop, P, max(10, steps), stream)
    flops = 2.0 * (prob.n_genes - 1) * P * prob.n_patterns
    f16 = game.fitness(pop, with64=True)[1]
    idx = torch.arange(0, P, P // 64, device=dev)
    r64 = game.rescore64(pop[idx].contiguous())
    rel = ((f16[idx] - r64).abs() / r64).cpu().numpy()
    game.close()
    achieved = flops / t_kernel / 1e12
    return {"workload": "precision: 1,000,000 patterns x 32 features, Chebyshev degree 8 "
                        "(257 genes), population 4,096, BF16 operands, FP32 accumulation",
            "value": P * prob.n_patterns * steps / elapsed, "unit": "evals/s",
            "ms_per_step": elapsed * 1e3 / steps, "dtype": "bf16",
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": BF16_MFMA_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": achieved / BF16_MFMA_PEAK_TFLOPS,
                         "traffic": profiled_traffic("fitness_bf16_precision.md"), "kernel_ms": t_kernel * 1e3,
                         "kernel_timing": f"median of {max(20, max(10, steps))} launches",
                         "flops_per_launch": flops},
            "error_vs_float64": {"max_rel": float(rel.max()), "median_rel": float(np.median(rel)),
                                 "sample": f"{idx.numel()} chromosomes of the population, "
                                           "float64 re-score on the GPU"}}


SURROGATE_CFG = dict(hidden=256, fp32_operands=0, archive=16384, minibatch=1024, train_steps=48,
                     lr=2e-3, oversample=8, audit=256, rho_min=0.8, min_archive=4096, seed=0)


def _run_to_target(gg, prob, precision, cap, val_target=None, train_target=None,
                   surrogate=None, seed=0, chunk=5, split_at=None, trace_every=None):
    """One GA run on the precision problem from generation 0.

    With val_target None the run takes exactly `cap` generations (the plain
    float32 reference; with split_at it stops there once and resumes, so the
    best training error at that generation is recorded on the way).  Else it
    advances `chunk` generations at a time and after each chunk re-scores its
    best chromosome (best by training error) in float64 on the validation
    set, stopping once that is <= val_target or after `cap` generations.
    Wall time covers initialisation, graph capture, the generations, the
    surrogate's training and the validation checks.  The first time the
    best training error is <= train_target is recorded too.  With
    trace_every, every that many generations the best's float64 validation
    error is recorded (and a progress line logged)."""
    import torch
    dev = torch.device("cuda:0")
    P = prob.population
    cfg = gg.config(basis=prob.basis, degree=prob.degree, population=P, precision=precision,
                    seed=seed, max_generations=cap, target=0.0)
    game = gg.Game(cfg, prob.X_dev, prob.t_dev)
    sur = None
    if surrogate is not None:
        surrogate = dict(surrogate, seed=seed)
        sur = gg.Surrogate(gg.surrogate_config(**surrogate), prob.n_genes,
                           surrogate["oversample"] * (P - cfg.elitism))
        gg.game_attach_surrogate(game.h, sur.h)

    def val_of(best):
        b = torch.from_numpy(best).to(dev).view(1, -1)
        return float(game.rescore64(b, prob.Xv_dev, prob.tv_dev)[0])

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    game.init_population()
    reached_val = reached_train = None
    split = None
    trace = []

    def traced(gens, best):
        if trace_every and gens % trace_every == 0:
            trace.append({"generation": gens, "seconds": time.perf_counter() - t0,
                          "validation_mse_fp64": val_of(best)})
            log(f"  generation {gens}: validation {trace[-1]['validation_mse_fp64']:.5f}")

    if val_target is None:
        if split_at is not None:
            g1, best1, err1 = game.run(max_generations=split_at)
            split = {"generations": g1, "seconds": time.perf_counter() - t0,
                     "train_mse_fp64": float(game.rescore64(
                         torch.from_numpy(best1).to(dev).view(1, -1))[0])}
        step = trace_every or cap
        gen = 0
        while gen < cap:
            gen = min(gen + step, cap)
            gens, best, err = game.run(max_generations=gen)
            traced(gens, best)
    else:
        gen = 0
        while True:
            gen = min(gen + chunk, cap)
            gens, best, err = game.run(max_generations=gen)
            if train_target is not None and reached_train is None and err <= train_target:
                reached_train = {"generations": gens, "seconds": time.perf_counter() - t0}
            if val_of(best) <= val_target:
                reached_val = {"generations": gens, "seconds": time.perf_counter() - t0}
                break
            traced(gens, best)
            if gens >= cap:
                break
    elapsed = time.perf_counter() - t0
    best_dev = torch.from_numpy(best).to(dev).view(1, -1)
    train64 = float(game.rescore64(best_dev)[0])
    val64 = val_of(best)
    # exact evaluations: the population each generation (generation 0
    # included), plus the audited children when a surrogate screens
    per_gen = P + (surrogate["audit"] if surrogate is not None else 0)
    res = {"generations": gens, "seconds": elapsed, "train_mse_fp64": train64,
           "validation_mse_fp64": val64, "exact_evaluations": (int(gens) + 1) * per_gen,
           "ms_per_generation": elapsed * 1e3 / max(gens, 1)}
    if val_target is not None:
        res["reached"] = reached_val is not None
        res["reached_train_target"] = reached_train
    if split is not None:
        res["at_split"] = split
    if trace:
        res["validation_trace"] = trace
    if sur is not None:
        st = sur.stats()
        res["surrogate"] = {"last_rho": st["rho"], "screened_generations": st["screened_total"],
                            "screened_fraction": st["screened_total"] / max(gens, 1),
                            "adam_steps": st["adam_steps"]}
        sur.close()
    game.close()
    return res


def _rho_trace(gg, prob, generations, surrogate):
    """The audit's rank correlation and the screening count every 5
    generations of the surrogate run (same seed, stepped one generation at a
    time)."""
    P = prob.population
    cfg = gg.config(basis=prob.basis, degree=prob.degree, population=P,
                    precision=gg.GAME_BF16, seed=0, max_generations=1 << 30, target=-1.0)
    game = gg.Game(cfg, prob.X_dev, prob.t_dev)
    sur = gg.Surrogate(gg.surrogate_config(**surrogate), prob.n_genes,
                       surrogate["oversample"] * (P - cfg.elitism))
    gg.game_attach_surrogate(game.h, sur.h)
    game.init_population()
    trace = []
    for gen in range(generations):
        game.step()
        if gen % 5 == 4:
            st = sur.stats()
            trace.append({"generation": gen + 1, "rho": round(st["rho"], 3),
                          "screened_total": st["screened_total"]})
    sur.close()
    game.close()
    return trace


def form_time_to_target(gg, prob, reference_generations=1000, secondary_generations=300, cap=3,
                        seeds=(0, 1, 2, 3, 4), surrogate_cfg=None):
    """Time to a validation-error target on the precision problem, per GA
    seed.  Plain float32 GAME runs `reference_generations` generations; the
    float64 validation error of its best chromosome is the target T*.  Plain
    BF16 and the surrogate-screened BF16 form (network 257-256-256-1, 8x
    oversampled offspring, exact fallback below rank correlation 0.8) run
    with the same seed until the float64 validation error of their best
    chromosome is <= T* (checked every 5 generations), at most `cap` times as
    many generations.  Medians over the seeds are reported.  Secondary line:
    the earlier target, the plain float32 best training error after
    `secondary_generations` generations, reached by the other two forms on
    their way.  For the first seed the surrogate run's audit correlation is
    traced, and an untrained, always-trusted network is run as the
    ablation."""
    sur_cfg = dict(surrogate_cfg or SURROGATE_CFG)
    per_seed = []
    first = None
    for seed in seeds:
        log(f"time to target: seed {seed}, plain FP32 reference")
        plain = _run_to_target(gg, prob, gg.GAME_FP32, reference_generations, seed=seed,
                               split_at=secondary_generations)
        T = plain["validation_mse_fp64"]
        T2 = plain["at_split"]["train_mse_fp64"]
        log(f"time to target: seed {seed}, T* = {T:.5f}; plain BF16, surrogate + BF16")
        cap_g = cap * reference_generations
        bf16 = _run_to_target(gg, prob, gg.GAME_BF16, cap_g, val_target=T, train_target=T2,
                              seed=seed)
        chosen = _run_to_target(gg, prob, gg.GAME_BF16, cap_g, val_target=T, train_target=T2,
                                surrogate=sur_cfg, seed=seed)
        per_seed.append({"seed": seed, "target_validation_mse": T,
                         "secondary_target_train_mse": T2,
                         "plain_fp32": plain, "plain_bf16": bf16, "surrogate_bf16": chosen})
        if first is None:
            first = per_seed[-1]
            log("time to target: rho trace and untrained-network ablation")
            chosen["rho_trace"] = _rho_trace(gg, prob, chosen["generations"], sur_cfg)
            # Ablation: the same screening with a network that is never
            # trained and always trusted (offspring picked by random-weight
            # predictions).
            untrained_cfg = dict(sur_cfg, train_steps=0, rho_min=-1.0, min_archive=0)
            first["untrained_surrogate_bf16"] = _run_to_target(
                gg, prob, gg.GAME_BF16, cap_g, val_target=T, train_target=T2,
                surrogate=untrained_cfg, seed=seed)

    def med(vals):
        vals = [v for v in vals if v is not None]
        return float(np.median(vals)) if vals else None

    def primary(r, run):
        return r[run]["seconds"] if run == "plain_fp32" else (
            r[run]["seconds"] if r[run]["reached"] else None)

    median = {"plain_fp32": {"seconds": med([r["plain_fp32"]["seconds"] for r in per_seed]),
                             "generations": med([r["plain_fp32"]["generations"] for r in per_seed]),
                             "validation_mse_fp64": med([r["plain_fp32"]["validation_mse_fp64"]
                                                         for r in per_seed])}}
    for run in ("plain_bf16", "surrogate_bf16"):
        rs = [r[run] for r in per_seed]
        median[run] = {"seconds": med([x["seconds"] if x["reached"] else None for x in rs]),
                       "generations": med([x["generations"] if x["reached"] else None for x in rs]),
                       "validation_mse_fp64": med([x["validation_mse_fp64"] for x in rs]),
                       "reached": sum(bool(x["reached"]) for x in rs)}
    speed = [r["plain_fp32"]["seconds"] / r["surrogate_bf16"]["seconds"] for r in per_seed
             if r["surrogate_bf16"]["reached"]]
    vs_bf16 = [r["plain_bf16"]["seconds"] / r["surrogate_bf16"]["seconds"] for r in per_seed
               if r["surrogate_bf16"]["reached"] and r["plain_bf16"]["reached"]]
    # secondary: the 300-generation training target
    sec = {}
    for run in ("plain_bf16", "surrogate_bf16"):
        hit = [r[run]["reached_train_target"] for r in per_seed]
        sec[run] = {"seconds": med([h["seconds"] if h else None for h in hit]),
                    "generations": med([h["generations"] if h else None for h in hit]),
                    "reached": sum(h is not None for h in hit)}
    sec["plain_fp32"] = {"seconds": med([r["plain_fp32"]["at_split"]["seconds"] for r in per_seed]),
                         "generations": secondary_generations, "reached": len(per_seed)}
    s_speed = [r["plain_fp32"]["at_split"]["seconds"] / r["surrogate_bf16"]["reached_train_target"]["seconds"]
               for r in per_seed if r["surrogate_bf16"]["reached_train_target"]]
    sec["speedup_chosen_vs_plain_fp32_median"] = med(s_speed)
    out = {"workload": "precision problem (1,000,000 x 32, Chebyshev degree 8, population "
                       "4,096, validation 250,000 patterns), GA seeds "
                       f"{list(seeds)}; target T* = float64 validation error of plain FP32's "
                       f"best after {reference_generations} generations, per seed; the other "
                       "forms stop once their best's float64 validation error is <= T* "
                       f"(checked every 5 generations, at most {cap_g} generations)",
           "median": median,
           "speedup_chosen_vs_plain_fp32_median": med(speed),
           "speedup_chosen_vs_plain_bf16_median": med(vs_bf16),
           "chosen_beats_plain_fp32": bool(speed) and med(speed) > 1.0,
           "secondary_300_generation_training_target": sec,
           "seeds": [{"seed": r["seed"], "target_validation_mse": r["target_validation_mse"],
                      **{run: {k: r[run].get(k) for k in ("generations", "seconds", "reached",
                                                          "validation_mse_fp64")}
                         for run in ("plain_fp32", "plain_bf16", "surrogate_bf16")},
                      "surrogate": r["surrogate_bf16"].get("surrogate")}
                     for r in per_seed],
           "surrogate_config": sur_cfg}
    # the first seed in full: runs, surrogate statistics, rho trace, ablation
    out.update({"first_seed": {k: first[k] for k in (
        "target_validation_mse", "secondary_target_train_mse", "plain_fp32", "plain_bf16",
        "surrogate_bf16", "untrained_surrogate_bf16")}})
    return out


def form_long_horizon(gg, prob, generations=5000, seed=0, cap=3, surrogate_cfg=None):
    """The time-to-target comparison at a later target, one seed: plain
    float32 GAME runs `generations` generations (its best's float64
    validation error every 1,000 generations is recorded) and the final one
    is T*; plain BF16 and surrogate + BF16 then run until their best's
    float64 validation error is <= T*, at most `cap` times as many
    generations.  Shows whether the surrogate's lead holds further down the
    descent than the 1,000-generation target."""
    sur_cfg = dict(surrogate_cfg or SURROGATE_CFG)
    log(f"long horizon: plain FP32, {generations} generations (seed {seed})")
    plain = _run_to_target(gg, prob, gg.GAME_FP32, generations, seed=seed, trace_every=1000)
    T = plain["validation_mse_fp64"]
    cap_g = cap * generations
    log(f"long horizon: T* = {T:.5f}; plain BF16")
    bf16 = _run_to_target(gg, prob, gg.GAME_BF16, cap_g, val_target=T, seed=seed,
                          trace_every=1000)
    log("long horizon: surrogate + BF16")
    chosen = _run_to_target(gg, prob, gg.GAME_BF16, cap_g, val_target=T, surrogate=sur_cfg,
                            seed=seed, trace_every=1000)
    return {"workload": "precision problem (1,000,000 x 32, Chebyshev degree 8, population "
                        f"4,096, validation 250,000 patterns), GA seed {seed}; target T* = "
                        f"float64 validation error of plain FP32's best after {generations} "
                        "generations; the other forms stop once their best's float64 "
                        f"validation error is <= T* (checked every 5 generations, at most "
                        f"{cap_g} generations)",
            "target_validation_mse": T,
            # the error of the best constant predictor on the validation set
            "validation_target_variance": float(np.var(prob.t_val.astype(np.float64))),
            "plain_fp32": plain, "plain_bf16": bf16, "surrogate_bf16": chosen,
            "speedup_chosen_vs_plain_fp32": (plain["seconds"] / chosen["seconds"]
                                             if chosen["reached"] else None),
            "surrogate_config": sur_cfg}


# Whole-training wall time (TOT, seconds) of the paper's GPU version for
# 4,000 generations of the shared-gene polytrigo model, by degree and data
# size (Table 3; GeForce GT540M, host transfers included).  Context only:
# another machine, and its time includes host-device transfers.
PAPER_TABLE3_TOT = {1: (15.00, 240.00, 1870.50, 7680.00), 2: (16.00, 256.00, 1993.55, 8192.00),
                    4: (19.00, 304.00, 2372.11, 9728.00), 8: (24.00, 384.00, 3006.12, 12288.00)}


def form_paper_shaped(gg, generations=4000):
    """The paper's scaling table on this GPU: the shared-gene polytrigo
    model (2d+1 genes, Eq. 9) of degree 1, 2, 4 and 8 on the 2,100 x 11
    binary set replicated to 0.15, 16, 128 and 512 MB of the paper's data
    size, 23 chromosomes, tournament 4, crossover 0.9, mutation 0.2,
    elitism 2, TMSE R = 0.49, 4,000 generations.

    Each row is split into Table 3's columns (Eqs. 11-13): HtoD is the upload
    of the replicated patterns and targets from host memory; DP the device
    time of the run (HIP events around the cos/sin sums, initialisation and
    the graph-captured training loop on the stream); HP the host time of the
    run not covered by device time (wall clock minus DP); DtoH the copy of
    the final population and its errors back to the host; DtoD is zero (the
    loop copies nothing on the device: populations alternate between two
    buffers).  P = DP + HP, T = HtoD + DtoH + DtoD, TOT = P + T."""
    import torch
    from paper_1304_0597_amd import datagen
    base = datagen.paper_shaped()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    def make_cfg(gens):
        return gg.config(basis=gg.GAME_POWER, degree=1, population=23, tournament_k=4,
                         elitism=2, p_crossover=0.9, p_mutation=0.2, sigma_mutation=0.1,
                         error_fn=gg.GAME_TMSE, tmse_R=0.49, seed=0, max_generations=gens,
                         target=0.0)

    # Untimed warm-up: the process's first host-to-device copy, kernel loads
    # and graph capture are one-time costs, not a row's.
    Xw = torch.from_numpy(np.ascontiguousarray(base.X)).to(dev)
    tw = torch.from_numpy(np.ascontiguousarray(base.t)).to(dev)
    Zw = torch.empty((base.n_patterns, 2), dtype=torch.float32, device=dev)
    gw = gg.Game(make_cfg(100), Zw, tw)
    gg.game_trig_sums(Xw, 1, Zw, stream)
    gw.init_population()
    gw.run()
    gw.population()[0].cpu()
    gw.close()
    torch.cuda.synchronize()
    rows = {}
    for d, paper in PAPER_TABLE3_TOT.items():
        for size, tot in zip(datagen.PAPER_SIZES_MB, paper):
            n = datagen.paper_rows(size)
            reps = -(-n // base.n_patterns)
            Xh = np.ascontiguousarray(np.tile(base.X, (reps, 1))[:n])
            th = np.ascontiguousarray(np.tile(base.t, reps)[:n])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            X = torch.from_numpy(Xh).to(dev)
            t = torch.from_numpy(th).to(dev)
            torch.cuda.synchronize()
            htod = time.perf_counter() - t0
            Z = torch.empty((n, 2 * d), dtype=torch.float32, device=dev)
            game = gg.Game(make_cfg(generations), Z, t)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            e0.record(stream)
            gg.game_trig_sums(X, d, Z, stream)
            game.init_population()
            gens, _, err = game.run()
            e1.record(stream)
            e1.synchronize()
            wall = time.perf_counter() - t1
            dp = e0.elapsed_time(e1) / 1e3
            hp = max(0.0, wall - dp)
            t2 = time.perf_counter()
            pop, fit = game.population()
            pop_h, fit_h = pop.cpu(), fit.cpu()
            dtoh = time.perf_counter() - t2
            game.close()
            P_ = dp + hp
            T_ = htod + dtoh
            rows[f"d{d}_{size:g}MB"] = {
                "patterns": n, "generations": gens, "best_tmse": err,
                "seconds": P_ + T_,
                "table3": {"DP": dp, "HP": hp, "HtoD": htod, "DtoH": dtoh, "DtoD": 0.0,
                           "P": P_, "T": T_, "TOT": P_ + T_},
                "paper_tot_seconds": tot, "ratio_paper_over_this": tot / (P_ + T_)}
            del X, t, Z, Xh, th, pop_h, fit_h
    return {"workload": "shared-gene polytrigo (Eq. 9), 2,100 x 11 binary set replicated to "
                        "0.15/16/128/512 MB of the paper's size, population 23, 4,000 "
                        "generations, TMSE R = 0.49; the patterns start in host memory",
            "columns": "Table 3: DP device processing (HIP events), HP host processing not "
                       "covered by device time, HtoD pattern upload, DtoH population and "
                       "errors back, DtoD none; P = DP + HP, T = HtoD + DtoH + DtoD, "
                       "TOT = P + T (seconds)",
            "runs": rows,
            "paper_hardware": "GeForce GT540M (Table 3 TOT, host transfers included)"}


def form_trig(gg, prob, reps=25):
    """The trigonometric expansion (Eq. 8) on the scale workload's patterns:
    degree 4 gives 2 x 20 x 4 + 1 = 161 genes, the same product shape as the
    Legendre degree-8 headline (M = 200,000, N = 2,048, K = 160), so the two
    fractions of peak differ only by what the expansion costs: the trig
    recurrence is seeded with cos x and sin x of each (pattern, feature) in
    every chromosome tile."""
    import torch
    dev = torch.device("cuda:0")
    P = prob.population
    X = torch.from_numpy(prob.X).to(dev)
    t = torch.from_numpy(prob.t).to(dev)
    cfg = gg.config(basis=gg.GAME_TRIG, degree=4, population=P, seed=0,
                    max_generations=1 << 30, target=-1.0)
    game = gg.Game(cfg, X, t)
    game.init_population()
    pop, _ = game.population()
    t_kernel = time_fitness(gg, game, pop, P, reps, torch.cuda.current_stream())
    game.close()
    K = gg.game_num_genes(cfg, prob.n_features)
    flops = 2.0 * (K - 1) * P * prob.n_patterns
    achieved = flops / t_kernel / 1e12
    return {"workload": "trig: 200,000 patterns x 20 features, trigonometric degree 4 "
                        "(161 genes), population 2,048, FP32",
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP32_MFMA_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": achieved / FP32_MFMA_PEAK_TFLOPS,
                         "traffic": profiled_traffic("fitness_f32_trig.md"),
                         "kernel_ms": t_kernel * 1e3, "kernel_timing": f"median of {reps} launches",
                         "flops_per_launch": flops}}


def form_degree_sweep(gg, degrees=(1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 16), reps=25):
    """The fused fitness kernels across degrees on the precision problem's
    shape (1,000,000 patterns x 32 features, Chebyshev, population 4,096,
    K - 1 = 32 d expansion terms): FP32 and BF16 kernel time (median of
    `reps` HIP-event-timed launches after 30 untimed ones) and fraction of
    each precision's MFMA peak.  Shows the tile choices the plans make: FP32
    128-chromosome tiles while the genes fit one LDS chunk (d <= 8 here),
    64-chromosome tiles through two gene buffers above; BF16 eight waves
    per workgroup where a lane half's group holds at most 4 sub-features,
    four waves otherwise."""
    import torch
    from paper_1304_0597_amd import datagen
    dev = torch.device("cuda:0")
    NP, N, P = 1_000_000, 32, 4096
    rng = np.random.default_rng(11)
    X = torch.from_numpy(rng.uniform(-1, 1, (NP, N)).astype(np.float32)).to(dev)
    t = torch.from_numpy(rng.normal(0, 1, NP).astype(np.float32)).to(dev)
    rows = []
    for d in degrees:
        row = {"degree": d}
        for name, precision, peak in (("fp32", gg.GAME_FP32, FP32_MFMA_PEAK_TFLOPS),
                                      ("bf16", gg.GAME_BF16, BF16_MFMA_PEAK_TFLOPS)):
            cfg = gg.config(basis=datagen.CHEBYSHEV, degree=d, population=P, precision=precision,
                            seed=d, max_generations=1 << 30, target=-1.0)
            game = gg.Game(cfg, X, t)
            game.init_population()
            pop, _ = game.population()
            t_kernel = time_fitness(gg, game, pop, P, reps, torch.cuda.current_stream())
            game.close()
            K = gg.game_num_genes(cfg, N)
            tf = 2.0 * (K - 1) * P * NP / t_kernel / 1e12
            row["genes"] = K
            row[name] = {"kernel_ms": round(t_kernel * 1e3, 4), "tflops": round(tf, 1),
                         "frac": round(tf / peak, 4)}
        rows.append(row)
        log(f"degree sweep: d = {d}: FP32 {row['fp32']['frac']:.3f}, BF16 {row['bf16']['frac']:.3f}")
    return {"workload": "1,000,000 patterns x 32 features (uniform), Chebyshev degree d, "
                        "population 4,096; fused fitness kernel per precision",
            "kernel_timing": f"median of {reps} launches after 30 untimed ones",
            "rows": rows}


def form_batched(gg, steps, warmup, decomposition=None, autotune=False):
    """Batched form: the 256 runs of the batched workload (sizes drawn from
    seed 3) advanced together, FP32.  The work decomposition is the committed
    table of the bucketed autotuner (paper_1304_0597_amd/batch_tuning.json);
    autotune=True runs the uniform autotuner here instead, and
    decomposition = (tiles per item, grid) sets a uniform one (so that a
    profile traces that decomposition alone).  The evaluation launch is
    timed with HIP events."""
    import torch
    from paper_1304_0597_amd import batch_tuning
    problems, cfgs, shapes = batch_tuning.batched_workload()
    evals = sum(float(sh.population * sh.n_patterns) for sh in shapes)
    flops = sum(2.0 * sh.n_features * sh.degree * sh.population * sh.n_patterns for sh in shapes)
    batch = gg.Batch(problems, cfgs)
    batch.init()
    table = batch_tuning.load()
    if decomposition is not None:
        batch.tune(*decomposition)
        dec = {"source": "given", "tiles_per_item": decomposition[0], "grid": decomposition[1]}
    elif autotune or table is None or table.get("workload") != batch_tuning.WORKLOAD:
        tune = batch.autotune(reps=3)
        dec = {"source": "uniform autotuner", "tiles_per_item": tune["tiles_per_item"],
               "grid": tune["grid"], "best_mean_ms": tune["ms"], "times_ms": tune["times_ms"]}
    else:
        batch.tune_runs(batch_tuning.tiles_for(table, batch.n_genes), table["grid"])
        dec = {"source": "batch_tuning.json (bucketed autotuner)", **table}
    for _ in range(warmup):
        batch.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    n_items, _, grid = batch.items()
    # the evaluation launch of that decomposition alone, median of 25
    t_kernel = time_median(batch.evaluate, torch.cuda.current_stream(), reps=25, warmup=5)
    batch.close()
    achieved = flops / t_kernel / 1e12
    return {"workload": "batched: 256 independent runs, patterns 1e3-2e5 log-uniform, features "
                        "4-64, degree 2-10, population 32-1024, Chebyshev/power, FP32 "
                        "(sizes drawn from seed 3)",
            "value": evals * steps / elapsed, "unit": "evals/s",
            "ms_per_step": elapsed * 1e3 / steps, "dtype": "f32",
            "evals_per_generation": evals,
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP32_MFMA_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": achieved / FP32_MFMA_PEAK_TFLOPS,
                         "traffic": profiled_traffic("fitness_batch_256runs.md"),
                         "kernel_ms": t_kernel * 1e3, "kernel_timing": "median of 25 launches",
                         "flops_per_launch": flops},
            "decomposition": dict(dec, items=n_items)}


def calibrate_gemm(reps=20, fp32=False):
    """The vendor library's GEMM (torch.matmul -> hipBLASLt) on two large
    shapes and on the fitness contraction's own shape: median TFLOP/s over
    HIP-event-timed launches.  BF16 operands with FP32 accumulation on
    131,072 x 4,096 x 256 (the precision workload), or, with fp32, float32
    operands (TF32 off) on 200,000 x 2,048 x 160 (the scale workload).  A
    reference for what the matrix cores sustain on this GPU, not a part of
    the method."""
    import torch
    torch.backends.cuda.matmul.allow_tf32 = False
    dtype = torch.float32 if fp32 else torch.bfloat16
    peak = FP32_MFMA_PEAK_TFLOPS if fp32 else BF16_MFMA_PEAK_TFLOPS
    own = (200_000, 2048, 160) if fp32 else (131072, 4096, 256)
    out = {}
    stream = torch.cuda.current_stream()
    for (M, N, K) in ((8192, 8192, 8192), (16384, 16384, 8192), own):
        a = torch.randn(M, K, dtype=dtype, device="cuda:0")
        b = torch.randn(K, N, dtype=dtype, device="cuda:0")
        t = time_median(lambda: torch.matmul(a, b), stream, reps=reps)
        tf = 2.0 * M * N * K / t / 1e12
        out[f"{M}x{N}x{K}"] = {"ms": t * 1e3, "tflops": tf, "frac": tf / peak}
        del a, b
    return {"calibration": f"torch.matmul {'float32' if fp32 else 'bfloat16'} (hipBLASLt)",
            "peak_tflops": peak, "shapes": out}


def scale_step(gg, prob, steps, warmup):
    """The headline line: generations of the scale workload, and its fused
    fitness kernel on the MFMA roofline."""
    import torch
    P = prob.population
    dev = torch.device("cuda:0")
    X = torch.from_numpy(prob.X).to(dev)
    t = torch.from_numpy(prob.t).to(dev)
    cfg = gg.config(basis=prob.basis, degree=prob.degree, population=P, tournament_k=3,
                    elitism=2, p_crossover=0.9, p_mutation=0.05, sigma_mutation=0.1, seed=0,
                    max_generations=1 << 30, target=-1.0)
    game = gg.Game(cfg, X, t)
    game.init_population()
    stream = torch.cuda.current_stream()
    log("scale workload: timing generations")
    elapsed = time_steps(game, steps, warmup)
    st = game.state()
    assert st["stopped"] == 0, "the run stopped inside the timed region"
    # Dominant kernel: the fused fitness launch (plus its tiny finish kernel)
    # on the same stream and launch configuration, median of HIP-event-timed
    # launches.
    pop, _ = game.population()
    t_kernel = time_fitness(gg, game, pop, P, 25, stream)
    game.close()
    flops = 2.0 * (prob.n_genes - 1) * P * prob.n_patterns
    achieved = flops / t_kernel / 1e12
    return elapsed, {"bound": "mfma", "achieved": achieved, "peak": FP32_MFMA_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_MFMA_PEAK_TFLOPS,
                     "traffic": profiled_traffic("fitness_f32_scale.md"),
                     "kernel_ms": t_kernel * 1e3, "kernel_timing": "median of 25 launches",
                     "flops_per_launch": flops}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the BF16, batched and surrogate workloads")
    ap.add_argument("--no-paper", action="store_true",
                    help="skip the paper-shaped scaling table (shared-gene polytrigo runs)")
    ap.add_argument("--no-target", action="store_true",
                    help="skip the time-to-target comparison (plain FP32 vs surrogate + BF16)")
    ap.add_argument("--target-generations", type=int, default=1000,
                    help="generations of the plain FP32 run that sets the time-to-target goal")
    ap.add_argument("--target-seeds", type=int, default=5,
                    help="GA seeds of the time-to-target comparison (0, 1, ...)")
    ap.add_argument("--long-generations", type=int, default=5000,
                    help="--only long_target: generations of the plain FP32 reference run")
    ap.add_argument("--only", choices=["scale", "bf16", "batched", "target", "paper", "trig",
                                       "long_target", "degrees"],
                    help="run one workload alone and print its result (for profiling)")
    ap.add_argument("--batch-decomp", type=str, default=None,
                    help="batched form: a uniform 'tiles,grid' instead of the committed table")
    ap.add_argument("--batch-autotune", action="store_true",
                    help="batched form: run the uniform autotuner instead of the committed table")
    ap.add_argument("--calibrate-gemm", action="store_true",
                    help="only time the vendor BF16 GEMM (torch.matmul, hipBLASLt) on large "
                         "square-ish shapes: the practical matrix-core throughput of this GPU")
    ap.add_argument("--calibrate-gemm-fp32", action="store_true",
                    help="the same with float32 operands (TF32 off), against the FP32 MFMA peak")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain elementwise kernel of known traffic (256 MiB read, "
                         "256 MiB written per launch) to scale hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        x = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(5):
            torch.neg(x, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "torch.neg float32", "bytes_read": x.numel() * 4,
                          "bytes_written": y.numel() * 4, "launches": 5}), flush=True)
        return
    if args.calibrate_gemm or args.calibrate_gemm_fp32:
        print(json.dumps(calibrate_gemm(fp32=args.calibrate_gemm_fp32)), flush=True)
        return
    from paper_1304_0597_amd import datagen
    from paper_1304_0597_amd import game as gg

    gg.lib()
    seeds = tuple(range(args.target_seeds))
    if args.only in ("bf16", "batched", "target", "paper", "trig", "long_target", "degrees"):
        if args.only == "trig":
            log("trig expansion on the scale patterns: building inputs")
            res = form_trig(gg, datagen.scale())
        elif args.only == "bf16":
            log("precision form: building inputs")
            res = form_bf16(gg, precision_problem(), args.steps, args.warmup)
        elif args.only == "batched":
            log("batched form: building inputs, autotuning, timing")
            dec = tuple(int(v) for v in args.batch_decomp.split(",")) if args.batch_decomp else None
            res = form_batched(gg, args.steps, args.warmup, dec, args.batch_autotune)
        elif args.only == "target":
            log("time to target: building inputs")
            res = form_time_to_target(gg, precision_problem(), args.target_generations,
                                      seeds=seeds)
        elif args.only == "degrees":
            log("degree sweep: FP32 and BF16 fitness kernels on 1,000,000 x 32")
            res = form_degree_sweep(gg)
        elif args.only == "long_target":
            log("long-horizon time to target: building inputs")
            res = form_long_horizon(gg, precision_problem(), args.long_generations)
        else:
            res = form_paper_shaped(gg)
        print(json.dumps({"only": args.only, "result": res}), flush=True)
        return

    log("scale workload: building inputs")
    prob = datagen.scale()
    P = prob.population
    elapsed, roofline = scale_step(gg, prob, args.steps, args.warmup)
    out = {
        "metric": METRIC,
        "value": P * prob.n_patterns * args.steps / elapsed,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "scale: 200,000 patterns x 20 features, Legendre degree 8 "
                               "(161 genes), population 2,048, one generation per step",
                   "n_patterns": prob.n_patterns, "n_features": prob.n_features,
                   "degree": prob.degree, "basis": "legendre", "population": P,
                   "genes": prob.n_genes},
        "roofline": roofline,
    }
    if args.only == "scale":
        print(json.dumps(out), flush=True)
        return
    if not args.no_forms:
        log("precision form: building inputs")
        pprob = precision_problem()
        log("precision form: timing")
        forms = {"bf16": form_bf16(gg, pprob, args.steps, args.warmup)}
        log("trig expansion on the scale patterns")
        forms["trig"] = form_trig(gg, prob)
        log("batched form: building inputs, autotuning, timing")
        forms["batched"] = form_batched(gg, max(5, args.steps // 5), max(2, args.warmup // 5))
        out["forms"] = forms
        if not args.no_paper:
            log("paper-shaped scaling table: shared-gene polytrigo, 16 runs")
            out["paper_shaped"] = form_paper_shaped(gg)
        if not args.no_target:
            log("time to target: plain FP32, plain BF16, surrogate + BF16")
            out["time_to_target"] = form_time_to_target(gg, pprob, args.target_generations,
                                                        seeds=seeds)
        del pprob
    if not args.no_cpu:
        log("oracle on the host cores")
        base = cpu_baseline(prob, P)
        log("serial oracle on one host core")
        ser = cpu_serial(prob)
        ser["gpu_over_this"] = out["value"] / ser["value"]
        base["serial"] = ser
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
