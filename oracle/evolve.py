"""Reference of the evolution step that feeds the library (test
infrastructure only).

Section 3 of the paper: evolution runs on the CPU, by tournament selection
and offspring generation with randomized coefficients; candidates go to the
GPU for evaluation, and (optionally) back-propagation refines each
candidate's fitness every generation, which steers evolution through the
Baldwin effect (the tuned fitness is used for selection, the offspring
inherit the untuned rule sets).  Section 4.1: a fixed pool of 100 candidate
rule sets.  The paper gives no operator details; the reading implemented
here (and, independently, by the library's host code) is:

Random stream: SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): a 64-bit counter advanced by
0x9e3779b97f4a7c15 per draw and mixed by two xor-shift-multiply rounds.
  below(n) = ((next() >> 32) * n) >> 32          an integer in [0, n)
  unit()   = (next() >> 40) * 2**-24             a float32 in [0, 1)

Random condition (F features, C classes, per-feature ranges lo, hi):
  feature-vs-feature if unit() < ff_frac (and F >= 2), else threshold;
  f = below(F); g = (f + 1 + below(F - 1)) % F for feature-vs-feature;
  op = below(4); coef = unit(); then coef2 = unit() (feature-vs-feature) or
  theta = float32(lo[f] + unit() * (hi[f] - lo[f])) in float64 (threshold).
Random rule: class = below(C), then one random condition.
Random pool: per rule set R = 1 + below(max_rules), default = below(C);
  per rule K = 1 + below(max_conds), class = below(C), K random conditions.

Next generation from a pool P with fitness F (higher is better):
  the elite best rule sets (fitness descending, ties by index) pass as they
  are; every other slot gets a child:
    tournament(): k draws i = below(n), the best of them (ties: lower index);
    child = copy of tournament();
    if unit() < p_crossover: B = tournament(); ca = below(R_A + 1),
      cb = below(R_B + 1); rules = A[:ca] + B[cb:] (A[:1] if that is
      empty), cut to max_rules; default of A;
    every condition in order: if unit() < p_coef: coef = unit(), then
      coef2 = unit() or theta from the range, as for a random condition;
    if unit() < p_struct: t = below(4):
      0 add a condition: r = below(R); if K_r < max_conds, append a random
        condition to rule r;
      1 drop a condition: r = below(R); if K_r >= 2, drop j = below(K_r);
      2 add a rule: if R < max_rules, insert a random rule at below(R + 1);
      3 drop a rule: if R >= 2, drop below(R).
A rule set is a list of rules [class, [conditions]]; a condition is a dict
with op, kind, f, g, coef, coef2, theta (float32 values).
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1


class SplitMix64:
    def __init__(self, state: int):
        self.state = state & MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def below(self, n: int) -> int:
        return ((self.next() >> 32) * n) >> 32

    def unit(self) -> np.float32:
        return np.float32((self.next() >> 40) * 2.0 ** -24)


def _range_theta(rng, lo, hi, f):
    u = float(rng.unit())
    return np.float32(float(lo[f]) + u * (float(hi[f]) - float(lo[f])))


def random_condition(rng, cfg, nf, lo, hi):
    ff = bool(rng.unit() < np.float32(cfg["ff_frac"])) and nf >= 2
    f = rng.below(nf)
    g = (f + 1 + rng.below(nf - 1)) % nf if ff else 0
    op = rng.below(4)
    coef = rng.unit()
    if ff:
        return dict(op=op, kind=1, f=f, g=g, coef=coef, coef2=rng.unit(), theta=np.float32(0))
    return dict(op=op, kind=0, f=f, g=0, coef=coef, coef2=np.float32(0),
                theta=_range_theta(rng, lo, hi, f))


def random_rule(rng, cfg, nf, nc, lo, hi):
    cls = rng.below(nc)
    return [cls, [random_condition(rng, cfg, nf, lo, hi)]]


def random_pool(rng, cfg, nf, nc, lo, hi):
    pool = []
    for _ in range(cfg["pool"]):
        R = 1 + rng.below(cfg["max_rules"])
        default = rng.below(nc)
        rules = []
        for _ in range(R):
            K = 1 + rng.below(cfg["max_conds"])
            cls = rng.below(nc)
            rules.append([cls, [random_condition(rng, cfg, nf, lo, hi) for _ in range(K)]])
        pool.append((default, rules))
    return pool


def _copy(rs):
    default, rules = rs
    return default, [[c, [dict(d) for d in conds]] for c, conds in rules]


def tournament(rng, fitness, k):
    best = -1
    for _ in range(k):
        i = rng.below(len(fitness))
        if best < 0 or fitness[i] > fitness[best] or (fitness[i] == fitness[best] and i < best):
            best = i
    return best


def next_generation(rng, pool, fitness, cfg, nf, nc, lo, hi):
    n = len(pool)
    order = sorted(range(n), key=lambda i: (-int(fitness[i]), i))
    out = [_copy(pool[i]) for i in order[:cfg["elite"]]]
    for _ in range(cfg["elite"], n):
        a = tournament(rng, fitness, cfg["tournament"])
        default, rules = _copy(pool[a])
        if rng.unit() < np.float32(cfg["p_crossover"]):
            b = tournament(rng, fitness, cfg["tournament"])
            rb = _copy(pool[b])[1]
            ca = rng.below(len(rules) + 1)
            cb = rng.below(len(rb) + 1)
            merged = rules[:ca] + rb[cb:]
            rules = (merged if merged else rules[:1])[:cfg["max_rules"]]
        for _, conds in rules:
            for c in conds:
                if rng.unit() < np.float32(cfg["p_coef"]):
                    c["coef"] = rng.unit()
                    if c["kind"] == 1:
                        c["coef2"] = rng.unit()
                    else:
                        c["theta"] = _range_theta(rng, lo, hi, c["f"])
        if rng.unit() < np.float32(cfg["p_struct"]):
            t = rng.below(4)
            if t == 0:
                r = rng.below(len(rules))
                if len(rules[r][1]) < cfg["max_conds"]:
                    rules[r][1].append(random_condition(rng, cfg, nf, lo, hi))
            elif t == 1:
                r = rng.below(len(rules))
                if len(rules[r][1]) >= 2:
                    del rules[r][1][rng.below(len(rules[r][1]))]
            elif t == 2:
                if len(rules) < cfg["max_rules"]:
                    pos = rng.below(len(rules) + 1)
                    rules.insert(pos, random_rule(rng, cfg, nf, nc, lo, hi))
            else:
                if len(rules) >= 2:
                    del rules[rng.below(len(rules))]
        out.append((default, rules))
    return out


def to_rule_lists(pool):
    """In the form of ``population.from_rule_lists``."""
    return [(d, [(c, conds) for c, conds in rules]) for d, rules in pool]


def from_population(pop):
    """A Population as this module's pool form."""
    out = []
    for s in range(pop.n_sets):
        d, rules = pop.to_rule_list(s)
        out.append((d, [[c, conds] for c, conds in rules]))
    return out
