"""Benchmark of the rule-set evaluation hot path on one MI355X.

Step = one hard fitness pass (correct counts + confusion) of 4096 rule sets
(1-32 rules x 1-6 conditions, 30% feature-vs-feature) over a resident
2^20 x 64 fp32 dataset with 4 classes.  `value` is nominal rule-condition
evaluations per second (every condition of every rule for every sample, as
the paper's tensor form computes them).  Synthetic data stands in for the
paper's UCI Breast Cancer table (not available here), at scaled-up shape.

Also reported: the roofline of the hard-eval kernel (VALU lane-ops of the
work a 64-lane wave must do, against 256 CU x 64 lanes x 2.4 GHz), the soft
forward/backward rates, the ragged persistent batch and the serving loop
when those paths are present, and the CPU oracle on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

VALU_PEAK = 256 * 64 * 2.4e9          # lane-ops/s (fp32 VALU, non-packed)
HBM_PEAK = 8.0e12                     # bytes/s


# HBM bytes per launch of the hard-eval kernel on the 2^20 x 64, 4096-set
# workload, from two rocprofv3 --pmc runs (FETCH_SIZE 271,703.5 KiB and
# WRITE_SIZE 65,568.0 KiB per dispatch, scaled by what the counters read for a
# plain 256 MiB copy: x1.99978 and x1.000), and the same for the kernel that
# sums its per-tile counts (FETCH_SIZE 32,957.1 KiB, WRITE_SIZE 10,039.3 KiB).
# Valid only for the kernel, launch-configuration and record-layout sources
# it was measured on.
HARD_TRAFFIC = {"bytes": 6.2356e8, "reduce_bytes": 7.7812e7, "sources_sha256": "70e21aa2705ce79f"}
HARD_SOURCES = ("hard.hip", "hard_block.h", "eval_core.h", "capi.cpp", "pack.cpp", "internal.h")


def hard_traffic(key="bytes"):
    import hashlib
    h = hashlib.sha256()
    for f in HARD_SOURCES:
        with open(os.path.join(ROOT, "paper_2406_01821_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return HARD_TRAFFIC[key] if h.hexdigest()[:16] == HARD_TRAFFIC["sources_sha256"] else None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_work(w):
    """Stored wave-level work counts for this workload (written by
    tests/golden/make_algorithmic_work.py, which calls only the oracle), with
    a spot check of a few rule sets recomputed now."""
    import oracle
    path = os.path.join(ROOT, "tests", "golden", "algorithmic_work.json")
    with open(path) as fh:
        rec = json.load(fh)[w.name]
    pop = w.pop.conds_kind_first()
    ptr, idx = oracle.label_grouped_tiles(w.data.y, w.data.n_classes, 64)
    sample = [0, w.pop.n_sets // 2, w.pop.n_sets - 1]
    wt, wf = oracle.workcount(w.data.x, pop.subset(sample), ptr, idx)
    for k, s in enumerate(sample):
        assert rec["work_t"][s] == wt[k] and rec["work_ff"][s] == wf[k], "stale work counts"
    return rec


def time_cpu_oracle_hard(w, budget_s=15.0):
    import oracle
    threads = oracle.max_threads()
    n_sets = 8
    while True:
        sub = w.pop.subset(range(n_sets))
        t0 = time.perf_counter()
        oracle.hard_eval(w.data.x, w.data.y, w.data.n_classes, sub)
        dt = time.perf_counter() - t0
        if dt * 2 > budget_s or n_sets * 2 > w.pop.n_sets:
            break
        n_sets = min(w.pop.n_sets, int(n_sets * max(2.0, budget_s / max(dt, 1e-3) / 2)))
    nominal = int(sub.nominal_conds_per_set().sum()) * w.data.n
    return dict(value=nominal / dt, unit="cond-evals/s", cores=threads, kind="oracle",
                sample=f"first {n_sets} of {w.pop.n_sets} rule sets x all {w.data.n} samples, "
                       f"{dt:.2f} s")


def time_call_level(ctx, ds, w, reps=3):
    """One whole call from host rule sets to host results: validation and
    packing on the host, the copy to the device, the evaluation and the
    copy of the counts back (median of reps; the dataset stays resident)."""
    import torch
    total, pack = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p = ctx.pack_population(w.pop, w.data.n_features, w.data.n_classes)
        t1 = time.perf_counter()
        c, m = ctx.eval_population(ds, p)
        c.cpu(), m.cpu()
        t2 = time.perf_counter()
        ctx.release_population(p)
        total.append((t2 - t0) * 1e3)
        pack.append((t1 - t0) * 1e3)
    med = lambda v: sorted(v)[len(v) // 2]
    return {"ms": med(total), "host_pack_ms": med(pack),
            "what": "pack on the host + copy to the device + evaluation + counts back"}


def cpu_oracle_detail(w, budget_s=2.0):
    """The oracle on one host thread (a slice of rule sets grown to about
    budget_s of CPU work), with the host's CPU model and usable cores."""
    import oracle
    n_sets = 1
    while True:
        sub = w.pop.subset(range(n_sets))
        t0 = time.perf_counter()
        oracle.hard_eval(w.data.x, w.data.y, w.data.n_classes, sub, nthreads=1)
        dt = time.perf_counter() - t0
        if dt * 2 > budget_s or n_sets * 2 > w.pop.n_sets:
            break
        n_sets = min(w.pop.n_sets, int(n_sets * max(2.0, budget_s / max(dt, 1e-3) / 2)))
    nominal = int(sub.nominal_conds_per_set().sum()) * w.data.n
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"single_thread": {"value": nominal / dt, "unit": "cond-evals/s",
                              "sample": f"first {n_sets} of {w.pop.n_sets} rule sets x all "
                                        f"{w.data.n} samples, {dt:.2f} s"},
            "oracle_threads": oracle.max_threads(), "cpu_model": model,
            "usable_cpus": usable}


# Algorithmic VALU work of the soft path, in lane issue slots of a plain fp32
# operation; a transcendental (v_exp_f32 / v_log_f32) counts as many slots as
# the issue-rate probe measures on the device (multiply rate / transcendental
# rate), once per bench run.
_TRANS = {}


def trans_weight(ctx):
    if "w" not in _TRANS:
        mul, trans = ctx.probe_valu_rates()
        _TRANS.update(w=mul / trans, mul_lane_ops_per_s=mul, trans_lane_ops_per_s=trans)
        log(f"VALU probe: multiply {mul / 1e12:.2f} T, transcendental {trans / 1e12:.2f} T "
            f"lane-op/s (weight {mul / trans:.2f})")
    return _TRANS["w"]


def soft_slots(t):
    """Per-condition and per-rule lane slots of the first-firing soft head,
    for a transcendental weight t: forward condition (z, log sigmoid(z),
    accumulate), forward rule (log(1-r), survival, class log-sum-exp),
    backward condition (sigmoid(-z), dL/dz, parameter terms) and backward
    rule (suffix recurrence)."""
    return 6 + 2 * t, 10 + 3 * t, 10 + 3 * t, 3 * t


def timed(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    return float(np.mean([a.elapsed_time(b) for a, b in ev])), wall * 1e3


def loop_us(fn, reps, warmup, stream):
    """Mean wall time of fn over reps back-to-back calls (host submission
    included), and the GPU time between events around the whole loop, in
    microseconds per call."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps * 1e6
    return wall, a.elapsed_time(b) / reps * 1e3


def bench_c1(ctx, steps, warmup, cpu, n_pools=64):
    """The paper's own shape (569 x 30 samples, 2 classes, pools of 100 rule
    sets): microseconds per pool evaluation, one launch per pool against many
    pools in one graph-replayed persistent launch, with the oracle beside
    it."""
    import torch
    import oracle
    from paper_2406_01821_amd import synth
    w = synth.small_hard(0)
    pools = synth.small_hard_pools(n_pools)
    ds = ctx.upload_dataset(w.data)
    dev = [ctx.pack_population(p, 30, 2) for p in pools]
    outs = [ctx.eval_population(ds, p) for p in dev]
    stream = torch.cuda.current_stream()
    reps = max(20, steps * 5)

    def plain():
        for p, o in zip(dev, outs):
            ctx.eval_population(ds, p, out=o)

    plain_wall, plain_gpu = loop_us(plain, reps, warmup, stream)
    one_wall, one_gpu = loop_us(lambda: ctx.eval_population(ds, dev[0], out=outs[0]), reps * 8,
                                warmup, stream)
    items = [(ds, p, *ctx.batch_outputs(ds, p)) for p in dev]
    ws = ctx.batch_workspace(items, (1, 1))
    (q, tg, kib), _ = ctx.autotune(items, ws)
    plan = ctx.batch_plan(items, ws, graph=True)
    batch_wall, batch_gpu = loop_us(plan.run, reps, warmup, stream)
    torch.cuda.synchronize()
    exact = all(torch.equal(it[2], o[0]) and torch.equal(it[3], o[1]) for it, o in zip(items, outs))
    # a whole call from host rule sets to host counts
    call = []
    for i in range(min(n_pools, 32)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p = ctx.pack_population(pools[i], 30, 2)
        c, m = ctx.eval_population(ds, p)
        c.cpu(), m.cpu()
        call.append((time.perf_counter() - t0) * 1e6)
        ctx.release_population(p)
    call_us = float(np.median(call))
    plan.release()
    for p in dev:
        ctx.release_population(p)
    ctx.release_dataset(ds)
    nominal = int(pools[0].nominal_conds_per_set().sum()) * w.data.n
    out = {
        "workload": "569 x 30 fp32 samples, 2 classes; pools of 100 rule sets x 1-8 rules x 1-4 "
                    "conditions, 30% feature-vs-feature (the paper's pool size and table shape)",
        "pools": n_pools,
        "plain_us_per_pool": plain_wall / n_pools, "plain_gpu_us_per_pool": plain_gpu / n_pools,
        "plain_one_pool_repeated_us": one_wall, "plain_one_pool_gpu_us": one_gpu,
        "batched_us_per_pool": batch_wall / n_pools, "batched_gpu_us_per_pool": batch_gpu / n_pools,
        "batched_split": {"sets_per_task": q, "tiles_per_task": tg, "tile_kib": kib},
        "speedup_vs_plain": plain_wall / batch_wall,
        "call_level_us": call_us,
        "call_level_what": "pack on the host + copy + evaluation + counts back, one pool",
        "bit_identical_to_plain": exact,
        "nominal_cond_evals_pool0": nominal,
    }
    log(f"C1: plain {plain_wall / n_pools:.1f} us/pool, batched {batch_wall / n_pools:.2f} us/pool "
        f"({plain_wall / batch_wall:.1f}x), call level {call_us:.0f} us, identical={exact}")
    if cpu:
        for nt, key in ((1, "oracle_one_thread_us_per_pool"), (0, "oracle_all_cores_us_per_pool")):
            oracle.hard_eval(w.data.x, w.data.y, 2, pools[0], nthreads=nt)
            t0 = time.perf_counter()
            k = 0
            while time.perf_counter() - t0 < 1.0:
                oracle.hard_eval(w.data.x, w.data.y, 2, pools[k % n_pools], nthreads=nt)
                k += 1
            out[key] = (time.perf_counter() - t0) / k * 1e6
        out["oracle_threads"] = oracle.max_threads()
    return out


def bench_finetune(ctx, epochs=20):
    """Fine-tuning epochs per second on the soft workload (262,144 x 32, 1024
    rule sets x 16 rules x 4 conditions): full-batch adjoint plus the fused
    Adam update, no loss history."""
    import torch
    from paper_2406_01821_amd import synth
    w = synth.soft_workload(3)
    ds = ctx.upload_dataset(w.data)
    pop = ctx.pack_population(w.pop, w.data.n_features, w.data.n_classes)
    par = [torch.tensor(a, device=ctx.device) for a in (w.pop.coef, w.pop.coef2, w.pop.theta)]
    ws = ctx.finetune_workspace(ds, pop)
    ctx.finetune(ds, pop, *par, epochs=1, ws=ws)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    ctx.finetune(ds, pop, *par, epochs=epochs, ws=ws)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    ctx.release_population(pop)
    ctx.release_dataset(ds)
    log(f"fine-tuning: {epochs} epochs in {ms:.1f} ms")
    return {"workload": "Adam fine-tuning, 262,144 x 32 fp32 samples, 1024 rule sets x 16 rules "
                        "x 4 threshold conditions, full batch, no loss history",
            "epochs": epochs, "ms": ms, "epochs_per_s": epochs / (ms * 1e-3),
            "ms_per_epoch": ms / epochs}


def bench_evolve(ctx, cpu, gens=200, tune_gens=5, epochs=50):
    """Evolution runs on the 569 x 30 table with the paper's pool of 100,
    with and without 50 epochs of fine-tuning per generation: generations per
    second on the GPU, and the same loop (the library's host breeding) with
    the oracle as the evaluator on the host cores, as the paper compares
    whole runs on a CPU and a GPU."""
    import torch
    import oracle
    from oracle import tune as otune
    from paper_2406_01821_amd import synth
    from paper_2406_01821_amd.aerl import evolve_cfg, breed
    w = synth.small_hard(0)
    x, y = w.data.x, w.data.y
    lo, hi = x.min(axis=0), x.max(axis=0)
    ds = ctx.upload_dataset(w.data)
    out = {"workload": "evolution on 569 x 30 fp32 samples, 2 classes, pool of 100 rule sets of "
                       "1-8 rules x 1-4 conditions, tournament 3, elite 2; fine-tuning: 50 Adam "
                       "epochs per generation (lr 0.01), Baldwinian"}
    for key, kw, n in (("plain", {}, gens), ("finetune", dict(tune_epochs=epochs), tune_gens)):
        cfg = evolve_cfg(seed=1, **kw)
        run = ctx.evolve(ds, cfg, lo, hi)
        run.run(1)
        torch.cuda.synchronize()
        s0 = run.state()
        t0 = time.perf_counter()
        run.run(n)
        dt = time.perf_counter() - t0
        s1 = run.state()
        run.release()
        out[key] = {"generations": n, "s": dt, "gen_per_s": n / dt,
                    "best_accuracy": float(s1["fitness"].max()) / w.data.n,
                    "host_eval_s": s1["seconds_eval"] - s0["seconds_eval"],
                    "host_tune_s": s1["seconds_tune"] - s0["seconds_tune"],
                    "host_breed_s": s1["seconds_breed"] - s0["seconds_breed"]}
        log(f"evolution {key}: {n / dt:.1f} generations/s")
        if cpu:
            pop, fit, state = s1["pool"], s1["fitness"], s1["rng_state"]

            def cpu_generation(pop, fit, state):
                pop, state = breed(pop, fit, cfg, 30, 2, lo, hi, state)
                scored = pop
                if key == "finetune":
                    tau = oracle.tau(x)
                    ps, _ = otune.finetune(x, y, tau, 2, pop, epochs, optimizer="adam", lr=0.01)
                    scored = pop.with_params(*ps[-1])
                fit, _ = oracle.hard_eval(x, y, 2, scored, confusion=False)
                return pop, fit, state

            pop, fit, state = cpu_generation(pop, fit, state)  # warm-up (thread pool start)
            m = max(2, n // 4)
            # each generation timed alone and the median taken: at this size the
            # oracle's thread start-up dominates and varies with the host's load
            # (the median favours the CPU loop)
            times = []
            for _ in range(m):
                t0 = time.perf_counter()
                pop, fit, state = cpu_generation(pop, fit, state)
                times.append(time.perf_counter() - t0)
            dt_cpu = float(np.median(times))
            out[key]["cpu_oracle"] = {"s_per_generation": dt_cpu, "mean_s": float(np.mean(times)),
                                      "generations": m, "statistic": "median",
                                      "cores": oracle.max_threads(), "kind": "oracle",
                                      "what": "library host breeding + oracle evaluation"
                                              + (" + fp64 oracle fine-tuning" if key == "finetune"
                                                 else "")}
            out[key]["cpu_over_gpu"] = dt_cpu / (dt / n)
    ctx.release_dataset(ds)
    return out


def bench_softmax(ctx, steps, warmup, beta=2.0):
    """The softmax head on the soft workload: forward and adjoint rates."""
    import torch
    from paper_2406_01821_amd import synth
    w = synth.soft_workload(3)
    ds = ctx.upload_dataset(w.data)
    pop = ctx.pack_population(w.pop, w.data.n_features, w.data.n_classes)
    c1, c2, th = [torch.tensor(a, device=ctx.device) for a in (w.pop.coef, w.pop.coef2, w.pop.theta)]
    wsf = ctx.soft_workspace(ds, pop, False)
    wsb = ctx.soft_workspace(ds, pop, True)
    dl = torch.ones(w.pop.n_sets, device=ctx.device)
    stream = torch.cuda.current_stream()
    trans_weight(ctx)  # the rate probe, run first: it also brings a cold GPU to speed
    warmup = max(warmup, 3)
    fwd_ms, _ = timed(lambda: ctx.softmax_forward(ds, pop, c1, c2, th, beta, ws=wsf), steps, warmup,
                      stream)
    bwd_ms, _ = timed(lambda: ctx.softmax_backward(ds, pop, c1, c2, th, beta, dl, ws=wsb), steps,
                      warmup, stream)
    n = w.data.n
    conds = int(w.pop.nominal_conds_per_set().sum()) * n
    rules = w.pop.n_rules * n
    nc = 2
    t = trans_weight(ctx)
    fc, _, bc, _ = soft_slots(t)
    # per rule: the first-firing rule cost minus its class log-sum-exp, plus
    # one exponential and nc selects for the vote
    rule_fwd = 10 + 3 * t + nc
    fwd_slots = float(fc * conds + rule_fwd * rules)
    bwd_slots = fwd_slots + float(bc * conds + (1 * t + 2 * nc + 4) * rules)
    ctx.release_population(pop)
    ctx.release_dataset(ds)
    log(f"softmax head: forward {fwd_ms:.3f} ms, backward {bwd_ms:.3f} ms")
    rl = lambda slots, ms: {"bound": "alu", "achieved": slots / (ms * 1e-3) / 1e12,
                            "peak": VALU_PEAK / 1e12, "unit": "Tlane-op/s",
                            "frac": slots / (ms * 1e-3) / VALU_PEAK}
    return {"workload": "softmax head (beta 2), 262,144 x 32 fp32 samples, 2 classes, 1024 rule "
                        "sets x 16 rules x 4 threshold conditions",
            "forward": {"ms": fwd_ms, "cond_evals_per_s": conds / (fwd_ms * 1e-3),
                        "roofline": rl(fwd_slots, fwd_ms)},
            "backward": {"ms": bwd_ms, "cond_evals_per_s": conds / (bwd_ms * 1e-3),
                         "roofline": rl(bwd_slots, bwd_ms)}}


def bench_categorical(ctx, steps, warmup):
    """Hard fitness on a table with categorical columns: 2^18 samples x (24
    numeric + 8 categorical) columns, 3 classes, 1024 rule sets with 30%
    categorical conditions (code-set tests)."""
    import torch
    from paper_2406_01821_amd import synth
    w = synth.categorical_workload(5)
    ds = ctx.upload_dataset(w.data)
    pop = ctx.pack_population(w.pop, w.data.n_features, w.data.n_classes)
    out = ctx.eval_population(ds, pop)
    stream = torch.cuda.current_stream()
    ms, wall = timed(lambda: ctx.eval_population(ds, pop, out=out), steps, warmup, stream)
    nominal = int(w.pop.nominal_conds_per_set().sum()) * w.data.n
    ctx.release_population(pop)
    ctx.release_dataset(ds)
    log(f"categorical: {ms:.3f} ms per pass")
    return {"workload": "hard fitness, 2^18 x (24 numeric + 8 categorical) fp32 columns, 3 "
                        "classes, 1024 rule sets x 1-16 rules x 1-4 conditions, 30% categorical "
                        "(code sets over 12 codes), 20% feature-vs-feature",
            "ms": ms, "wall_ms": wall, "nominal_cond_evals": nominal,
            "cond_evals_per_s": nominal / (wall * 1e-3),
            "categorical_conditions": int((w.pop.kind == 2).sum()), "conditions": w.pop.n_conds}


def bench_soft(ctx, steps, warmup, cpu):
    import torch
    import oracle
    from paper_2406_01821_amd import synth
    w = synth.soft_workload(3)
    ds = ctx.upload_dataset(w.data)
    pop = ctx.pack_population(w.pop, w.data.n_features, w.data.n_classes)
    dev = ctx.device
    c1, c2, th = [torch.tensor(a, device=dev) for a in (w.pop.coef, w.pop.coef2, w.pop.theta)]
    wsf = ctx.soft_workspace(ds, pop, False)
    wsb = ctx.soft_workspace(ds, pop, True)
    dl = torch.ones(w.pop.n_sets, device=dev)
    stream = torch.cuda.current_stream()
    trans_weight(ctx)  # the rate probe, run first: it also brings a cold GPU to speed
    warmup = max(warmup, 3)
    fwd_ms, _ = timed(lambda: ctx.soft_forward(ds, pop, c1, c2, th, ws=wsf), steps, warmup, stream)
    bwd_ms, _ = timed(lambda: ctx.soft_backward(ds, pop, c1, c2, th, dl, ws=wsb), steps, warmup,
                      stream)
    n = w.data.n
    conds = int(w.pop.nominal_conds_per_set().sum()) * n
    rules = w.pop.n_rules * n
    fc, fr, bc, br = soft_slots(trans_weight(ctx))
    fwd_slots = float(fc * conds + fr * rules)
    bwd_slots = fwd_slots + float(bc * conds + br * rules)
    out = {
        "workload": "soft, 262,144 x 32 fp32 samples, 2 classes, 1024 rule sets x 16 rules x 4 "
                    "threshold conditions, tau = 0.05 std",
        "transcendental_weight": dict(_TRANS),
        "forward": {"ms": fwd_ms, "cond_evals_per_s": conds / (fwd_ms * 1e-3),
                    "roofline": {"bound": "alu", "achieved": fwd_slots / (fwd_ms * 1e-3) / 1e12,
                                 "peak": VALU_PEAK / 1e12, "unit": "Tlane-op/s",
                                 "frac": fwd_slots / (fwd_ms * 1e-3) / VALU_PEAK}},
        "backward": {"ms": bwd_ms, "cond_evals_per_s": conds / (bwd_ms * 1e-3),
                     "roofline": {"bound": "alu", "achieved": bwd_slots / (bwd_ms * 1e-3) / 1e12,
                                  "peak": VALU_PEAK / 1e12, "unit": "Tlane-op/s",
                                  "frac": bwd_slots / (bwd_ms * 1e-3) / VALU_PEAK}},
    }
    log(f"soft forward {fwd_ms:.3f} ms, backward {bwd_ms:.3f} ms")
    if cpu:
        tau = oracle.tau(w.data.x)
        k = 4
        while True:  # grow the sample to about 10 s of CPU work
            sub = w.pop.subset(range(k))
            t0 = time.perf_counter()
            oracle.soft_forward(w.data.x, w.data.y, tau, 2, sub)
            dt = time.perf_counter() - t0
            if dt * 2 > 10.0 or k * 2 > w.pop.n_sets:
                break
            k = min(w.pop.n_sets, int(k * max(2.0, 10.0 / max(dt, 1e-3) / 2)))
        sub_conds = int(sub.nominal_conds_per_set().sum()) * n
        out["cpu_baseline_forward"] = {"value": sub_conds / dt, "unit": "cond-evals/s",
                                       "cores": oracle.max_threads(), "kind": "oracle",
                                       "sample": f"first {k} of {w.pop.n_sets} rule sets x all "
                                                 f"{n} samples, fp64, {dt:.2f} s"}
    ctx.release_population(pop)
    ctx.release_dataset(ds)
    return out


def bench_ragged(ctx, steps, warmup):
    """64 independent runs (C3 shape) evaluated one launch per population, and
    as one graph-captured persistent launch with the autotuned work split."""
    import torch
    from paper_2406_01821_amd import synth
    t0 = time.time()
    runs = synth.ragged_runs()
    log(f"generated 64 ragged runs in {time.time() - t0:.1f}s")
    devs = [(ctx.upload_dataset(w.data),
             ctx.pack_population(w.pop, w.data.n_features, w.data.n_classes)) for w in runs]
    nominal = sum(int(w.pop.nominal_conds_per_set().sum()) * w.data.n for w in runs)
    outs = [ctx.eval_population(ds, p) for ds, p in devs]
    stream = torch.cuda.current_stream()

    def plain():
        for (ds, p), o in zip(devs, outs):
            ctx.eval_population(ds, p, out=o)

    plain_ms, plain_wall = timed(plain, steps, warmup, stream)

    def plain_host():  # what a per-run evolution loop does: fitness back to the host each time
        for (ds, p), o in zip(devs, outs):
            ctx.eval_population(ds, p, out=o)
            o[0].cpu()

    _, plain_host_wall = timed(plain_host, steps, warmup, stream)
    items = []
    for ds, p in devs:
        c, m = ctx.batch_outputs(ds, p)
        items.append((ds, p, c, m))
    ws = ctx.batch_workspace(items, (1, 1))
    (q, tg, kib), tune_ms = ctx.autotune(items, ws)
    plan = ctx.batch_plan(items, ws, graph=True)
    batch_ms, batch_wall = timed(plan.run, steps, warmup, stream)

    def batch_host():
        plan.run()
        for _, _, c, _ in items:
            c.cpu()

    _, batch_host_wall = timed(batch_host, steps, warmup, stream)
    torch.cuda.synchronize()
    exact = all(torch.equal(c, o[0]) and torch.equal(m, o[1])
                for (_, _, c, m), o in zip(items, outs))
    log(f"ragged: plain {plain_wall:.3f} ms, batched {batch_wall:.3f} ms; with results on the "
        f"host {plain_host_wall:.3f} vs {batch_host_wall:.3f} ms "
        f"(tuned split {q} sets x {tg} tiles, {kib} KiB tiles), identical={exact}")
    plan.release()
    for ds, p in devs:
        ctx.release_population(p)
        ctx.release_dataset(ds)
    return {
        "workload": "64 independent runs: 1k-200k samples (log-uniform) x 16-128 fp32 features, "
                    "2-4 classes, 16-1024 rule sets of 1-64 rules x 1-8 conditions",
        "nominal_cond_evals": nominal,
        "plain": {"ms": plain_wall, "gpu_ms": plain_ms,
                  "cond_evals_per_s": nominal / (plain_wall * 1e-3)},
        "batched": {"ms": batch_wall, "gpu_ms": batch_ms,
                    "cond_evals_per_s": nominal / (batch_wall * 1e-3),
                    "sets_per_task": q, "tiles_per_task": tg, "tile_kib": kib,
                    "graph": True},
        "speedup_vs_plain": plain_wall / batch_wall,
        "with_results_on_host": {"plain_ms": plain_host_wall, "batched_ms": batch_host_wall,
                                 "speedup": plain_host_wall / batch_host_wall},
        "bit_identical_to_plain": exact,
    }


def bench_serve(ctx, small, ds_small, big, ds_big, n_requests=2000, rate_hz=2000.0):
    """Serving loop on the two resident datasets (569 x 30 and 2^20 x 64):
    Poisson arrivals at rate_hz, half fitness requests (8-2048 rule sets, 10%
    on the big dataset), half predictions (one rule set x 1-4096 rows).  The
    same request stream is also run launching each request alone (pack,
    evaluate, copy back, synchronize), open loop at the same arrival times and
    back to back for saturation throughput."""
    import torch
    from paper_2406_01821_amd import synth
    t0 = time.time()
    reqs = synth.serving_mix(small, big, n_requests, rate_hz=rate_hz, seed=4)
    log(f"generated {n_requests} serving requests in {time.time() - t0:.1f}s")
    datas, dss = (small, big), (ds_small, ds_big)
    nominal = 0.0
    for r in reqs:
        conds = r.pop.nominal_conds_per_set()
        nominal += (float(conds.sum()) * datas[r.dataset].n if r.kind == "fitness"
                    else float(conds[0]) * len(r.rows))

    def submit(r):
        if r.kind == "fitness":
            return ctx.serve_submit_fitness(dss[r.dataset], r.pop)
        return ctx.serve_submit_predict(r.pop, r.rows, big.n_features, big.n_classes, 0)

    def pace(t_start, t_arrival):
        while True:
            dt = t_arrival - (time.perf_counter() - t_start)
            if dt <= 0:
                return
            if dt > 2e-4:
                time.sleep(dt - 1e-4)

    ctx.serve_start(1 << 30)
    for t in [submit(r) for r in reqs[:64]]:  # warm-up
        t.wait()
    ctx.serve_stats(reset=True)
    t_start = time.perf_counter()
    tickets = []
    for r in reqs:
        pace(t_start, r.t_arrival)
        tickets.append(submit(r))
    served_out = [t.wait() for t in tickets]
    open_stats = ctx.serve_stats(reset=True)
    # saturation: four submitting threads (packing runs in parallel in the
    # library), every request offered at once
    import concurrent.futures as cf
    t1 = time.perf_counter()
    with cf.ThreadPoolExecutor(4) as ex:
        sat_tickets = list(ex.map(submit, reqs))
    submit_s = time.perf_counter() - t1
    for t in sat_tickets:
        t.wait()
    sat_s = time.perf_counter() - t1
    sat_stats = ctx.serve_stats(reset=True)
    ctx.serve_stop()
    log(f"served: p50 {open_stats['p50_us']:.0f} us, p99 {open_stats['p99_us']:.0f} us at "
        f"{rate_hz:.0f} req/s; saturation {n_requests / sat_s:.0f} req/s "
        f"(mean batch {sat_stats['mean_batch']:.1f})")

    def alone(r):
        d = datas[r.dataset]
        p = ctx.pack_population(r.pop, d.n_features, d.n_classes)
        if r.kind == "fitness":
            c, m = ctx.eval_population(dss[r.dataset], p)
            out = dict(correct=c.cpu().numpy(), confusion=m.cpu().numpy())
        else:
            out = dict(pred=ctx.predict(p, r.rows, 0).cpu().numpy())
        ctx.release_population(p)
        return out

    for r in reqs[:64]:
        alone(r)
    torch.cuda.synchronize()
    lat = []
    t_start = time.perf_counter()
    identical = True
    for r, so in zip(reqs, served_out):
        pace(t_start, r.t_arrival)
        ao = alone(r)
        lat.append((time.perf_counter() - t_start - r.t_arrival) * 1e6)
        identical = identical and all(np.array_equal(ao[k], so[k]) for k in ao)
    alone_open_s = time.perf_counter() - t_start
    t1 = time.perf_counter()
    for r in reqs:
        alone(r)
    alone_sat_s = time.perf_counter() - t1
    lat = np.sort(np.array(lat))
    pct = lambda p: float(lat[max(0, int(np.ceil(p * len(lat))) - 1)])
    log(f"alone: p50 {pct(0.5):.0f} us, p99 {pct(0.99):.0f} us at {rate_hz:.0f} req/s; "
        f"saturation {n_requests / alone_sat_s:.0f} req/s; identical={identical}")
    served_rps = n_requests / sat_s
    alone_rps = n_requests / alone_sat_s
    return {
        "workload": f"{n_requests} requests, Poisson at {rate_hz:.0f}/s: 50% fitness (8-2048 rule "
                    "sets of 1-32 rules x 1-6 conditions; 90% on 569 x 30, 10% on 2^20 x 64), "
                    "50% prediction (1 rule set x 1-4096 rows of 64 features)",
        "nominal_cond_evals": nominal,
        "served": {"offered_req_per_s": rate_hz, "p50_us": open_stats["p50_us"],
                   "p99_us": open_stats["p99_us"], "mean_us": open_stats["mean_us"],
                   "mean_batch": open_stats["mean_batch"],
                   "saturation_req_per_s": served_rps,
                   "saturation_cond_evals_per_s": nominal / sat_s,
                   "saturation_mean_batch": sat_stats["mean_batch"],
                   "saturation_submit_s": submit_s, "saturation_total_s": sat_s,
                   "offered_fraction_of_saturation": rate_hz / served_rps},
        "alone": {"p50_us": pct(0.5), "p99_us": pct(0.99), "open_loop_s": alone_open_s,
                  "saturation_req_per_s": alone_rps,
                  "saturation_cond_evals_per_s": nominal / alone_sat_s},
        "speedup_vs_alone": served_rps / alone_rps,
        "results_identical_to_alone": identical,
    }


def trace_summary(path, first=None, last=None):
    """Per-kernel statistics and cross-stream overlap of a rocprofv3 kernel
    trace (its *_kernel_trace.csv), over the dispatches from the first one
    whose name starts with `first` through the last one whose name starts
    with `last` (the whole trace by default).  Overlap: the time during which
    kernels of two or more streams (hardware queues) run at once, and the
    dispatches that share some of their run time with a dispatch of another
    stream."""
    import csv
    with open(path) as fh:
        rows = list(csv.DictReader(fh))
    key = "Stream_Id" if rows and "Stream_Id" in rows[0] else "Queue_Id"

    def short(name):  # the kernel's name without namespaces or arguments
        name = name.replace("void ", "").replace("(anonymous namespace)::", "")
        return name.split("(")[0].replace("aerl::", "")[:60]

    ev = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short(r["Kernel_Name"]),
                 r[key]) for r in rows)
    if first:
        i0 = next(i for i, e in enumerate(ev) if e[2].startswith(first))
        ev = ev[i0:]
    if last:
        i1 = max(i for i, e in enumerate(ev) if e[2].startswith(last))
        ev = ev[:i1 + 1]
    stats = {}
    for t0, t1, name, _ in ev:
        st = stats.setdefault(name, [0, 0.0, float("inf"), 0.0])
        d = (t1 - t0) * 1e-3
        st[0] += 1
        st[1] += d
        st[2] = min(st[2], d)
        st[3] = max(st[3], d)
    # sweep line over (time, +1/-1, stream)
    pts = sorted([(t0, 1, q) for t0, _, _, q in ev] + [(t1, -1, q) for _, t1, _, q in ev])
    live, busy, multi, prev = {}, 0, 0, None
    for t, d, q in pts:
        if prev is not None and live:
            busy += t - prev
            if sum(1 for v in live.values() if v > 0) >= 2:
                multi += t - prev
        live[q] = live.get(q, 0) + d
        if live[q] == 0:
            del live[q]
        prev = t
    # dispatches overlapping one of another stream (sorted by start)
    overl = [False] * len(ev)
    active = []
    for i, (t0, t1, _, q) in enumerate(ev):
        active = [j for j in active if ev[j][1] > t0]
        for j in active:
            if ev[j][3] != q:
                overl[i] = overl[j] = True
        active.append(i)
    span = (max(e[1] for e in ev) - ev[0][0]) * 1e-6 if ev else 0.0
    out = {"dispatches": len(ev), "streams": len({e[3] for e in ev}), "span_ms": span,
           "busy_ms": busy * 1e-6, "multi_stream_ms": multi * 1e-6,
           "dispatches_overlapping_another_stream": int(sum(overl)),
           "kernels": {k: {"calls": v[0], "avg_us": v[1] / v[0], "min_us": v[2], "max_us": v[3],
                           "total_ms": v[1] * 1e-3} for k, v in
                       sorted(stats.items(), key=lambda kv: -kv[1][1])}}
    return out


def bench_serve_alone(ctx):
    """The serving section on its own (both datasets uploaded here)."""
    from paper_2406_01821_amd import synth
    small = synth.small_hard(0).data
    big = synth.scaled_hard(1).data
    ds_small, ds_big = ctx.upload_dataset(small), ctx.upload_dataset(big)
    out = bench_serve(ctx, small, ds_small, big, ds_big)
    ctx.release_dataset(ds_small)
    ctx.release_dataset(ds_big)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only-hard", action="store_true", help="time the hard path only")
    ap.add_argument("--only", default=None, help="one extra section alone: c1, finetune, evolve, softmax, categorical, soft, serve, ragged")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run only a plain 256 MiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--trace-summary", default=None, metavar="CSV",
                    help="summarize a rocprofv3 kernel trace (per kernel, cross-stream overlap)")
    ap.add_argument("--trace-from", default=None, help="with --trace-summary: first kernel name")
    ap.add_argument("--trace-to", default=None, help="with --trace-summary: last kernel name")
    args = ap.parse_args()
    if args.trace_summary:
        print(json.dumps(trace_summary(args.trace_summary, args.trace_from, args.trace_to),
                         indent=1))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(rule sets or samples would be split across GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2406_01821_amd import synth
    from paper_2406_01821_amd.aerl import Context

    if args.copy_probe:
        nbytes = 256 << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes,
                          "launches": 3}), flush=True)
        return

    if args.only:
        ctx = Context(0)
        fn = {"c1": lambda: bench_c1(ctx, args.steps, args.warmup, not args.no_cpu),
              "finetune": lambda: bench_finetune(ctx),
              "evolve": lambda: bench_evolve(ctx, not args.no_cpu),
              "softmax": lambda: bench_softmax(ctx, max(3, args.steps // 4), 1),
              "categorical": lambda: bench_categorical(ctx, args.steps, args.warmup),
              "soft": lambda: bench_soft(ctx, max(3, args.steps // 4), 1, not args.no_cpu),
              "serve": lambda: bench_serve_alone(ctx),
              "ragged": lambda: bench_ragged(ctx, max(3, args.steps // 4), 1)}
        print(json.dumps({args.only: fn[args.only]()}), flush=True)
        ctx.close()
        return

    t0 = time.time()
    w = synth.scaled_hard(1)
    log(f"generated {w.name} in {time.time() - t0:.1f}s")
    ctx = Context(0)
    ds = ctx.upload_dataset(w.data)
    pop = ctx.pack_population(w.pop, w.data.n_features, w.data.n_classes)
    out = ctx.eval_population(ds, pop)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ms, wall_ms = timed(lambda: ctx.eval_population(ds, pop, out=out), args.steps, args.warmup,
                        stream)
    log(f"hard eval: kernel+fills {ms:.3f} ms/step (wall {wall_ms:.3f} ms/step)")
    nominal = int(w.pop.nominal_conds_per_set().sum()) * w.data.n
    value = nominal / (wall_ms * 1e-3)

    rec = algorithmic_work(w)
    # per condition and sample: a folded threshold is one compare, a
    # feature-vs-feature condition two products and a compare
    lane_ops = 64.0 * (1.0 * rec["total_t"] + 3.0 * rec["total_ff"])
    achieved = lane_ops / (ms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                "unit": "Tlane-op/s", "frac": achieved / VALU_PEAK, "traffic": hard_traffic(),
                "kernel": "k_hard", "algorithmic_lane_ops": lane_ops,
                "traffic_reduce_kernel": hard_traffic("reduce_bytes"),
                "hbm_bytes_min": float(w.data.n * (w.data.n_features + 1) * 4)}
    result = {
        "metric": "rule-condition evals/s (hard fitness, nominal)",
        "value": value, "unit": "cond-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "hard fitness, 2^20 x 64 fp32 samples, 4 classes, 4096 rule sets "
                               "x 1-32 rules x 1-6 conditions, 30% feature-vs-feature",
                   "n_samples": w.data.n, "n_features": w.data.n_features,
                   "n_sets": w.pop.n_sets, "nominal_cond_evals": nominal},
        "kernel_ms": ms,
        "roofline": roofline,
    }
    result["call_level"] = time_call_level(ctx, ds, w)
    if not args.no_cpu:
        result["cpu_baseline"] = time_cpu_oracle_hard(w)
        result["cpu_oracle_detail"] = cpu_oracle_detail(w)
    ctx.release_population(pop)
    if not args.only_hard:
        small = synth.small_hard(0).data
        ds_small = ctx.upload_dataset(small)
        result["serving"] = bench_serve(ctx, small, ds_small, w.data, ds)
        ctx.release_dataset(ds_small)
    ctx.release_dataset(ds)
    del w
    if not args.only_hard:
        result["soft"] = bench_soft(ctx, max(3, args.steps // 4), 1, not args.no_cpu)
        result["finetune"] = bench_finetune(ctx)
        result["softmax"] = bench_softmax(ctx, max(3, args.steps // 4), 1)
        result["categorical"] = bench_categorical(ctx, args.steps, args.warmup)
        result["ragged"] = bench_ragged(ctx, max(3, args.steps // 4), 1)
        result["c1"] = bench_c1(ctx, args.steps, args.warmup, not args.no_cpu)
        result["evolution"] = bench_evolve(ctx, not args.no_cpu)
    print(json.dumps(result), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
