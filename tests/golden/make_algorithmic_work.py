"""Writes algorithmic_work.json: the condition visits a 64-lane wave must make
(threshold and feature-vs-feature separately) to evaluate each benchmark
population under wave-uniform early exit, on 64-sample tiles of the
label-grouped sample order.  Computed by the oracle only.

Usage: python tests/golden/make_algorithmic_work.py [--quick]
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2406_01821_amd import synth  # noqa: E402


def digest(w) -> str:
    h = hashlib.sha256()
    for a in (w.data.x, w.data.y, w.pop.set_rule_off, w.pop.rule_cond_off, w.pop.op, w.pop.kind,
              w.pop.f, w.pop.g, w.pop.coef, w.pop.coef2, w.pop.theta, w.pop.rule_class,
              w.pop.set_default):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


def work_for(w):
    pop = w.pop.conds_kind_first()  # the library evaluates threshold conditions first
    ptr, idx = oracle.label_grouped_tiles(w.data.y, w.data.n_classes, 64)
    wt, wf = oracle.workcount(w.data.x, pop, ptr, idx)
    nominal = int(w.pop.nominal_conds_per_set().sum()) * w.data.n
    return dict(workload=w.name, digest=digest(w), n=w.data.n, n_sets=w.pop.n_sets,
                tiles64=len(ptr) - 1, nominal_cond_evals=nominal,
                work_t=[int(v) for v in wt], work_ff=[int(v) for v in wf],
                total_t=int(wt.sum()), total_ff=int(wf.sum()))


def main():
    out = {}
    for w in (synth.small_hard(0), synth.scaled_hard(1)):
        r = work_for(w)
        out[r["workload"]] = r
        print(r["workload"], r["total_t"], r["total_ff"], flush=True)
    with open(os.path.join(HERE, "algorithmic_work.json"), "w") as fh:
        json.dump(out, fh)


if __name__ == "__main__":
    main()
