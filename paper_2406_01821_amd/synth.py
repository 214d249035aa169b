"""Seeded synthetic workloads.

The paper measures on the UCI Breast Cancer data (569 samples x 30 numeric
features, binary label; Section 4.1) with a fixed pool of 100 candidate rule
sets.  That data is not shipped here; these generators stand in for it with
data of the same shape and of scaled-up shapes.  Every array is drawn from
``numpy.random.default_rng(seed)`` (PCG64) in the documented order, so both
the library's tests and the oracle's tests receive identical inputs.

This module only draws numbers.  Labels are planted with a small decision
list on raw feature values (``x[f] > q`` / ``x[f] < q`` at empirical
quantiles), which is data synthesis: the labels are inputs to both the
library and the oracle, so nothing here is shared arithmetic between them.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np

from .population import Dataset, Population


# ---------------------------------------------------------------- features
def lognormal_features(rng: np.random.Generator, n: int, nf: int) -> np.ndarray:
    """Per column ``mu ~ U(-1, 3)``, ``sigma ~ U(0.2, 0.8)``; entries
    ``exp(mu + sigma * N(0,1))`` drawn in float64 and rounded to float32.
    Draw order: mu[nf], sigma[nf], then the [n][nf] normals row by row."""
    mu = rng.uniform(-1.0, 3.0, size=nf)
    sigma = rng.uniform(0.2, 0.8, size=nf)
    x = np.empty((n, nf), dtype=np.float32)
    chunk = 1 << 16
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        z = rng.standard_normal((b - a, nf))
        x[a:b] = np.exp(mu + sigma * z).astype(np.float32)
    return x


# ---------------------------------------------------------------- labels
def planted_labels(x: np.ndarray, n_classes: int, n_rules: int, conds: tuple, noise: float,
                   seed: int, min_share: float = 0.10, max_attempts: int = 200) -> np.ndarray:
    """Labels from a random planted decision list over raw features, with an
    exact number ``round(noise * n)`` of labels flipped.

    Attempt ``a`` draws from ``default_rng(seed + 1000 * a)``: per rule a
    condition count in ``conds`` (inclusive), a class; per condition a
    feature, a direction and a quantile level ``U(0.2, 0.8)`` of that
    feature's column; then a default class.  The first attempt whose labels
    give every class at least ``min_share`` of the samples is kept.  Noise:
    ``round(noise*n)`` distinct samples (drawn without replacement) get a
    different class (the other one for two classes, otherwise a uniform
    other class)."""
    n, nf = x.shape
    for attempt in range(max_attempts):
        rng = np.random.default_rng(seed + 1000 * attempt)
        y = np.full(n, -1, dtype=np.int64)
        for _ in range(n_rules):
            k = int(rng.integers(conds[0], conds[1] + 1))
            cls = int(rng.integers(n_classes))
            hold = np.ones(n, dtype=bool)
            for _ in range(k):
                f = int(rng.integers(nf))
                greater = bool(rng.integers(2))
                q = np.float32(np.quantile(x[:, f], rng.uniform(0.2, 0.8)))
                hold &= (x[:, f] > q) if greater else (x[:, f] < q)
            y[(y < 0) & hold] = cls
        default = int(rng.integers(n_classes))
        y[y < 0] = default
        counts = np.bincount(y, minlength=n_classes)
        if counts.min() >= min_share * n:
            break
    else:
        raise RuntimeError("could not plant balanced labels")
    n_flip = int(round(noise * n))
    idx = rng.choice(n, size=n_flip, replace=False)
    if n_classes == 2:
        y[idx] = 1 - y[idx]
    else:
        y[idx] = (y[idx] + rng.integers(1, n_classes, size=n_flip)) % n_classes
    return y.astype(np.int32)


# ---------------------------------------------------------------- populations
def random_population(rng: np.random.Generator, x: np.ndarray, n_sets: int, rules: tuple,
                      conds: tuple, n_classes: int, ff_frac: float = 0.3,
                      kinds_allowed: str = "T+FF") -> Population:
    """Random rule sets in the form of the paper's candidate pool.

    Draw order (all vectors): rules per set ``U{rules}``, default class per
    set, conditions per rule ``U{conds}``, class per rule, then per
    condition: kind (feature-vs-feature with probability ``ff_frac``),
    feature ``f``, offset for ``g`` (``g = (f + U{1..nf-1}) % nf`` so
    ``g != f``), op ``U{<,<=,>,>=}``, ``coef ~ U(0,1)``, ``coef2 ~ U(0,1)``,
    threshold level ``u ~ U(0,1)``.  Thresholds are
    ``min_f + u * (max_f - min_f)`` over the column's empirical range,
    computed in float64 and rounded to float32.  Threshold conditions carry
    ``g = 0, coef2 = 0``; feature-vs-feature ones carry ``theta = 0``."""
    nf = x.shape[1]
    n_rules = rng.integers(rules[0], rules[1] + 1, size=n_sets)
    default = rng.integers(0, n_classes, size=n_sets)
    R = int(n_rules.sum())
    n_conds = rng.integers(conds[0], conds[1] + 1, size=R)
    rule_class = rng.integers(0, n_classes, size=R)
    K = int(n_conds.sum())
    kind = (rng.random(K) < ff_frac).astype(np.uint8)
    if kinds_allowed == "T":
        kind[:] = 0
    f = rng.integers(0, nf, size=K)
    goff = rng.integers(1, max(nf, 2), size=K)
    op = rng.integers(0, 4, size=K).astype(np.uint8)
    coef = rng.random(K).astype(np.float32)
    coef2 = rng.random(K).astype(np.float32)
    u = rng.random(K)
    cmin = x.min(axis=0).astype(np.float64)
    cmax = x.max(axis=0).astype(np.float64)
    theta = (cmin[f] + u * (cmax[f] - cmin[f])).astype(np.float32)
    g = (f + goff) % nf
    ff = kind == 1
    g = np.where(ff, g, 0)
    coef2 = np.where(ff, coef2, np.float32(0))
    theta = np.where(ff, np.float32(0), theta)
    set_rule_off = np.concatenate([[0], np.cumsum(n_rules)])
    rule_cond_off = np.concatenate([[0], np.cumsum(n_conds)])
    return Population(set_rule_off, default, rule_cond_off, rule_class, op, kind, f, g,
                      coef, coef2, theta)


# ---------------------------------------------------------------- workloads
@dataclass
class Workload:
    data: Dataset
    pop: Population
    name: str


def small_hard(seed: int = 0) -> Workload:
    """569 x 30 features, 2 classes, planted 3 rules x 2 conditions, 5% noise;
    100 rule sets of 1-8 rules x 1-4 conditions, 30% feature-vs-feature."""
    rng = np.random.default_rng(seed)
    x = lognormal_features(rng, 569, 30)
    y = planted_labels(x, 2, 3, (2, 2), 0.05, seed)
    pop = random_population(rng, x, 100, (1, 8), (1, 4), 2, 0.3)
    return Workload(Dataset(x, y, 2, "569x30"), pop, "hard-569x30-P100")


def small_hard_pools(n_pools: int = 64, seed0: int = 100) -> List[Population]:
    """Independent candidate pools of the 569 x 30 workload's shape (100 rule
    sets of 1-8 rules x 1-4 conditions, 30% feature-vs-feature), drawn on its
    dataset: pool i from ``default_rng(seed0 + i)``."""
    x = small_hard(0).data.x
    return [random_population(np.random.default_rng(seed0 + i), x, 100, (1, 8), (1, 4), 2, 0.3)
            for i in range(n_pools)]


def scaled_hard(seed: int = 1, n: int = 1 << 20, nf: int = 64, n_sets: int = 4096) -> Workload:
    """2^20 x 64 features, 4 classes, planted 12 rules x 1-4 conditions, 3%
    noise; 4096 rule sets of 1-32 rules x 1-6 conditions, 30%
    feature-vs-feature.  ``n`` / ``n_sets`` shrink it for tests."""
    rng = np.random.default_rng(seed)
    x = lognormal_features(rng, n, nf)
    y = planted_labels(x, 4, 12, (1, 4), 0.03, seed)
    pop = random_population(rng, x, n_sets, (1, 32), (1, 6), 4, 0.3)
    return Workload(Dataset(x, y, 4, f"{n}x{nf}"), pop, f"hard-{n}x{nf}-P{n_sets}")


def ragged_runs(n_runs: int = 64, seed0: int = 2000, n_range=(1000, 200_000),
                f_range=(16, 128), p_range=(16, 1024), rules=(1, 64), conds=(1, 8)) -> List[Workload]:
    """Independent runs, each with its own dataset and population.  Run i uses
    seed ``seed0 + i``: n log-uniform in ``n_range``, feature count uniform in
    ``f_range``, class count uniform in {2,3,4}, population size log-uniform
    in ``p_range``; labels planted with 4 rules x 1-3 conditions, 3% noise."""
    out = []
    for i in range(n_runs):
        rng = np.random.default_rng(seed0 + i)
        n = int(round(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1])))))
        nf = int(rng.integers(f_range[0], f_range[1] + 1))
        nc = int(rng.integers(2, 5))
        P = int(round(np.exp(rng.uniform(np.log(p_range[0]), np.log(p_range[1])))))
        x = lognormal_features(rng, n, nf)
        y = planted_labels(x, nc, 4, (1, 3), 0.03, seed0 + i)
        pop = random_population(rng, x, P, rules, conds, nc, 0.3)
        out.append(Workload(Dataset(x, y, nc, f"run{i}-{n}x{nf}"), pop, f"ragged-run{i}"))
    return out


def soft_workload(seed: int = 3, n: int = 262_144, nf: int = 32, n_sets: int = 1024,
                  n_rules: int = 16, n_conds: int = 4) -> Workload:
    """262,144 x 32 features, 2 classes, planted 4 rules x 1-3 conditions, 3%
    noise; 1024 rule sets of exactly 16 rules x 4 threshold conditions."""
    rng = np.random.default_rng(seed)
    x = lognormal_features(rng, n, nf)
    y = planted_labels(x, 2, 4, (1, 3), 0.03, seed)
    pop = random_population(rng, x, n_sets, (n_rules, n_rules), (n_conds, n_conds), 2, 0.0,
                            kinds_allowed="T")
    return Workload(Dataset(x, y, 2, f"{n}x{nf}"), pop, f"soft-{n}x{nf}-P{n_sets}")


def categorical_population(rng: np.random.Generator, x: np.ndarray, cat_cols: int, n_codes: int,
                           n_sets: int, rules: tuple, conds: tuple, n_classes: int,
                           cat_frac: float = 0.3, ff_frac: float = 0.2) -> Population:
    """Random rule sets over a table whose last ``cat_cols`` columns hold
    category codes 0..n_codes-1: a random population of the numeric columns
    (``random_population``), then each condition, with probability
    ``cat_frac``, becomes categorical on a uniform categorical column with a
    random code set (each code in with probability 1/2; one code, an
    equality test, with probability 1/4).  Draws after the population: per
    condition u (categorical?), column, equality?, code, set bits."""
    nf = x.shape[1]
    num = nf - cat_cols
    pop = random_population(rng, x[:, :num], n_sets, rules, conds, n_classes, ff_frac)
    K = pop.n_conds
    make = rng.random(K) < cat_frac
    col = num + rng.integers(0, cat_cols, size=K)
    eq = rng.random(K) < 0.25
    code = rng.integers(0, n_codes, size=K)
    bits = rng.integers(0, 2, size=(K, n_codes)).astype(np.uint64)
    weights = np.uint64(1) << np.arange(n_codes, dtype=np.uint64)
    sets_mask = (bits * weights).sum(axis=1).astype(np.uint64)
    mask = np.where(eq, np.uint64(1) << code.astype(np.uint64), sets_mask).astype(np.uint64)
    kind = np.where(make, 2, pop.kind).astype(np.uint8)
    f = np.where(make, col, pop.f).astype(np.int32)
    g = np.where(make, 0, pop.g).astype(np.int32)
    coef = np.where(make, np.float32(0), pop.coef).astype(np.float32)
    coef2 = np.where(make, np.float32(0), pop.coef2).astype(np.float32)
    theta = np.where(make, np.float32(0), pop.theta).astype(np.float32)
    return Population(pop.set_rule_off, pop.set_default, pop.rule_cond_off, pop.rule_class, pop.op,
                      kind, f, g, coef, coef2, theta, {}, np.where(make, mask, 0).astype(np.uint64))


def categorical_workload(seed: int = 5, n: int = 1 << 18, n_num: int = 24, cat_cols: int = 8,
                         n_codes: int = 12, n_classes: int = 3, n_sets: int = 1024,
                         rules=(1, 16), conds=(1, 4)) -> Workload:
    """A table of log-normal numeric columns followed by ``cat_cols``
    categorical columns of codes 0..n_codes-1 (Zipf-like code frequencies,
    stored as float32); labels planted on the numeric columns with the code
    of the first categorical column mixed in; rule sets with 30%
    categorical conditions."""
    rng = np.random.default_rng(seed)
    xn = lognormal_features(rng, n, n_num)
    w = 1.0 / np.arange(1, n_codes + 1)
    codes = rng.choice(n_codes, size=(n, cat_cols), p=w / w.sum()).astype(np.float32)
    x = np.concatenate([xn, codes], axis=1)
    y = planted_labels(xn, n_classes, 6, (1, 3), 0.03, seed)
    flip = codes[:, 0] == 0
    y = np.where(flip, (y + 1) % n_classes, y).astype(np.int32)
    pop = categorical_population(rng, x, cat_cols, n_codes, n_sets, rules, conds, n_classes)
    return Workload(Dataset(x, y, n_classes, f"{n}x{n_num}+{cat_cols}cat"), pop,
                    f"categorical-{n}x{n_num + cat_cols}-P{n_sets}")


def tiny(seed: int, n: int = 100, nf: int = 8, n_classes: int = 2, n_sets: int = 20,
         rules=(1, 6), conds=(1, 4), ff_frac: float = 0.3) -> Workload:
    """Small random case for tests (labels uniform, no planting)."""
    rng = np.random.default_rng(seed)
    x = lognormal_features(rng, n, nf)
    y = rng.integers(0, n_classes, size=n).astype(np.int32)
    pop = random_population(rng, x, n_sets, rules, conds, n_classes, ff_frac)
    return Workload(Dataset(x, y, n_classes, f"tiny{n}x{nf}"), pop, f"tiny-{seed}")


def special_values_population(seed: int, nf: int, n_classes: int, n_sets: int) -> Population:
    """Rule sets of 1-9 rules x 0-6 conditions whose coefficients and
    thresholds come from a list of special values (signed zeros, tiny and
    huge magnitudes, +-inf thresholds), 30% feature-vs-feature, empty rules
    anywhere (for edge-case tests)."""
    from .population import from_rule_lists
    rng = np.random.default_rng(seed)
    coefs = np.float32([0.0, -0.0, 1.0, -1.0, 0.5, -2.0, 1e-30, 3e38])
    thetas = np.float32([0.0, -0.0, 0.25, -1.5, np.inf, -np.inf, 1e-40])
    sets = []
    for _ in range(n_sets):
        rules = []
        for _ in range(int(rng.integers(1, 10))):
            conds = []
            for _ in range(int(rng.integers(0, 7))):
                op = int(rng.integers(4))
                f = int(rng.integers(nf))
                if rng.random() < 0.3:
                    g = int((f + 1 + rng.integers(nf - 1)) % nf)
                    conds.append(dict(op=op, kind=1, f=f, g=g, coef=rng.choice(coefs),
                                      coef2=rng.choice(coefs)))
                else:
                    conds.append(dict(op=op, kind=0, f=f, coef=rng.choice(coefs),
                                      theta=rng.choice(thetas)))
            rules.append((int(rng.integers(n_classes)), conds))
        sets.append((int(rng.integers(n_classes)), rules))
    return from_rule_lists(sets)


@dataclass
class Request:
    kind: str            # "fitness" or "predict"
    t_arrival: float     # seconds from start
    dataset: int         # 0 = small resident dataset, 1 = scaled one (fitness only)
    pop: Population
    rows: np.ndarray = None   # float32 [m][nf] for predict


def serving_mix(small: Dataset, big: Dataset, n_requests: int, rate_hz: float = 2000.0,
                seed: int = 4, p_range=(8, 2048), rows_range=(1, 4096),
                big_share: float = 0.1) -> List[Request]:
    """Poisson arrivals at ``rate_hz``: half fitness requests (small dataset
    with probability ``1 - big_share``, else the big one; population size
    log-uniform in ``p_range``; rule sets of 1-32 rules x 1-6 conditions),
    half prediction requests (one rule set, ``U`` log-uniform rows drawn from
    the big dataset's feature generator)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n_requests))
    out = []
    for i in range(n_requests):
        if rng.random() < 0.5:
            ds = 1 if rng.random() < big_share else 0
            d = big if ds == 1 else small
            P = int(round(np.exp(rng.uniform(np.log(p_range[0]), np.log(p_range[1])))))
            pop = random_population(rng, d.x[:4096], P, (1, 32), (1, 6), d.n_classes, 0.3)
            out.append(Request("fitness", float(t[i]), ds, pop))
        else:
            m = int(round(np.exp(rng.uniform(np.log(rows_range[0]), np.log(rows_range[1])))))
            start = int(rng.integers(0, max(1, big.n - m)))
            rows = big.x[start:start + m]
            pop = random_population(rng, big.x[:4096], 1, (1, 32), (1, 6), big.n_classes, 0.3)
            out.append(Request("predict", float(t[i]), 1, pop, rows))
    return out
