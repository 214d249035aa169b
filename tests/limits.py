"""Inputs at the library's documented maxima, shared by the GPU parity
tests: a 512-feature table and rule sets with rules of 255 conditions and
1023 records (the closing record included), whose conditions each pass
about 99% of the samples, so that walks run deep into the long rules."""
import numpy as np

from paper_2406_01821_amd import synth
from paper_2406_01821_amd.population import Dataset, from_rule_lists


def widest_table(rng, n=2000, nf=512, nc=3):
    x = synth.lognormal_features(rng, n, nf)
    y = rng.integers(0, nc, n).astype(np.int32)
    return Dataset(x, y, nc)


def longest_sets_population(rng, data, n_extra=12, seed=513):
    """Three rule sets at or next to the record limit (every record kind:
    folded thresholds both ways, zero coefficients, feature-vs-feature,
    empty rules), then n_extra random rule sets of the synthetic recipe."""
    x, nf, nc = data.x, data.n_features, data.n_classes
    lo, hi = np.quantile(x, 0.01, axis=0), np.quantile(x, 0.99, axis=0)

    def cond():
        f = int(rng.integers(nf))
        k = int(rng.integers(4))
        if k == 0:
            return dict(op=3, f=f, coef=1.0, theta=np.float32(lo[f]))
        if k == 1:
            return dict(op=1, f=f, coef=1.0, theta=np.float32(hi[f]))
        if k == 2:  # zero coefficient: 0*x > -1 for every finite x
            return dict(op=2, f=f, coef=0.0, theta=-1.0)
        g = (f + 1 + int(rng.integers(nf - 1))) % nf
        return dict(op=2, kind=1, f=f, g=g, coef=1.0, coef2=np.float32(1e-3))

    def rule(k):
        return (int(rng.integers(nc)), [cond() for _ in range(k)])

    long_sets = [
        (0, [rule(255) for _ in range(4)] + [rule(2)]),              # 1022 conditions
        (1 % nc, [rule(255) for _ in range(4)] + [rule(1), (2 % nc, [])]),  # 1021 + an empty rule
        (2 % nc, [rule(255), (1 % nc, []), rule(64), rule(255), rule(255), rule(191)]),
    ]
    recs = [sum(max(len(c), 1) for _, c in rules) + 1 for _, rules in long_sets]
    assert recs == [1023, 1023, 1022]
    rest = synth.tiny(seed, n=data.n, nf=nf, n_classes=nc, n_sets=n_extra, rules=(0, 12),
                      conds=(0, 6), ff_frac=0.3).pop
    return from_rule_lists(long_sets + [rest.to_rule_list(s) for s in range(rest.n_sets)])
