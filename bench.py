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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only-hard", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2406_01821_amd import synth
    from paper_2406_01821_amd.aerl import Context

    t0 = time.time()
    w = synth.scaled_hard(1)
    log(f"generated {w.name} in {time.time() - t0:.1f}s")
    ctx = Context(0)
    ds = ctx.upload_dataset(w.data)
    pop = ctx.pack_population(w.pop, w.data.n_features, w.data.n_classes)
    out = ctx.eval_population(ds, pop)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        ctx.eval_population(ds, pop, out=out)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        ctx.eval_population(ds, pop, out=out)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    step_ms = [a.elapsed_time(b) for a, b in ev]
    ms = float(np.mean(step_ms))
    log(f"hard eval: mean {ms:.3f} ms, min {min(step_ms):.3f}, max {max(step_ms):.3f} "
        f"(wall {wall / args.steps * 1e3:.3f} ms/step)")
    nominal = int(w.pop.nominal_conds_per_set().sum()) * w.data.n
    value = nominal / (wall / args.steps)

    rec = algorithmic_work(w)
    lane_ops = 64.0 * (2.0 * rec["total_t"] + 3.0 * rec["total_ff"])
    achieved = lane_ops / (ms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                "unit": "Tlane-op/s", "frac": achieved / VALU_PEAK, "traffic": None,
                "kernel": "k_hard", "algorithmic_lane_ops": lane_ops,
                "hbm_bytes_min": float(w.data.n * (w.data.n_features + 1) * 4)}
    result = {
        "metric": "rule-condition evals/s (hard fitness, nominal)",
        "value": value, "unit": "cond-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "hard fitness, 2^20 x 64 fp32 samples, 4 classes, 4096 rule sets "
                               "x 1-32 rules x 1-6 conditions, 30% feature-vs-feature",
                   "n_samples": w.data.n, "n_features": w.data.n_features,
                   "n_sets": w.pop.n_sets, "nominal_cond_evals": nominal},
        "kernel_ms": ms,
        "roofline": roofline,
    }
    if not args.no_cpu:
        result["cpu_baseline"] = time_cpu_oracle_hard(w)
    print(json.dumps(result), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
