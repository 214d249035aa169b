"""Host-side containers for datasets and rule-set populations.

A population is a list of rule sets in structure-of-arrays form.  Each rule set
is an ordered list of rules followed by a default class; each rule is an AND
of conditions and maps to one class.  This is the tensorized rule form of the
paper (Section 3, Fig. 1a) stored sparsely: a condition row of the paper's
rule tensor has one non-zero weight (a threshold condition) or two non-zero
weights with zero bias (a feature-versus-feature condition).

Condition encoding (one entry per condition, all arrays of length n_conds):

* ``op``    uint8: 0 ``<``, 1 ``<=``, 2 ``>``, 3 ``>=``
* ``kind``  uint8: 0 threshold ``coef*x[f] op theta``;
                   1 feature-vs-feature ``coef*x[f] op coef2*x[g]``
* ``f``, ``g`` int32 feature indices (``g`` ignored for kind 0)
* ``coef``, ``coef2``, ``theta`` float32 (``coef2`` ignored for kind 0,
  ``theta`` ignored for kind 1)

Nothing here evaluates a rule; the containers only hold and reshape arrays.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, List, Sequence

import numpy as np

OP_LT, OP_LE, OP_GT, OP_GE = 0, 1, 2, 3
KIND_T, KIND_FF = 0, 1


@dataclass
class Dataset:
    """Labeled samples: ``x`` float32 [n][f] row-major, ``y`` int32 [n]."""

    x: np.ndarray
    y: np.ndarray
    n_classes: int
    name: str = ""

    def __post_init__(self):
        self.x = np.ascontiguousarray(self.x, dtype=np.float32)
        self.y = np.ascontiguousarray(self.y, dtype=np.int32)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_features(self) -> int:
        return int(self.x.shape[1])


@dataclass
class Population:
    set_rule_off: np.ndarray   # int32 [n_sets+1]
    set_default: np.ndarray    # int32 [n_sets]
    rule_cond_off: np.ndarray  # int32 [n_rules+1]
    rule_class: np.ndarray     # int32 [n_rules]
    op: np.ndarray             # uint8 [n_conds]
    kind: np.ndarray           # uint8 [n_conds]
    f: np.ndarray              # int32 [n_conds]
    g: np.ndarray              # int32 [n_conds]
    coef: np.ndarray           # float32 [n_conds]
    coef2: np.ndarray          # float32 [n_conds]
    theta: np.ndarray          # float32 [n_conds]
    meta: dict = field(default_factory=dict)
    cat_mask: Optional[np.ndarray] = None  # uint64 [n_conds]: code set of kind-2 conditions

    def __post_init__(self):
        i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
        u8 = lambda a: np.ascontiguousarray(a, dtype=np.uint8)
        f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
        self.set_rule_off = i32(self.set_rule_off)
        self.set_default = i32(self.set_default)
        self.rule_cond_off = i32(self.rule_cond_off)
        self.rule_class = i32(self.rule_class)
        self.op, self.kind = u8(self.op), u8(self.kind)
        self.f, self.g = i32(self.f), i32(self.g)
        self.coef, self.coef2, self.theta = f32(self.coef), f32(self.coef2), f32(self.theta)
        self.cat_mask = (np.zeros(self.op.shape[0], np.uint64) if self.cat_mask is None
                         else np.ascontiguousarray(self.cat_mask, dtype=np.uint64))

    @property
    def n_sets(self) -> int:
        return int(self.set_default.shape[0])

    @property
    def n_rules(self) -> int:
        return int(self.rule_class.shape[0])

    @property
    def n_conds(self) -> int:
        return int(self.op.shape[0])

    def rules_of(self, s: int) -> range:
        return range(int(self.set_rule_off[s]), int(self.set_rule_off[s + 1]))

    def conds_of(self, r: int) -> range:
        return range(int(self.rule_cond_off[r]), int(self.rule_cond_off[r + 1]))

    def nominal_conds_per_set(self) -> np.ndarray:
        """Number of conditions in each rule set (int64 [n_sets])."""
        per_rule = np.diff(self.rule_cond_off.astype(np.int64))
        csum = np.concatenate([[0], np.cumsum(per_rule)])
        return csum[self.set_rule_off[1:]] - csum[self.set_rule_off[:-1]]

    def subset(self, sets: Sequence[int]) -> "Population":
        """A new population holding the given rule sets, in the given order."""
        return from_rule_lists([self.to_rule_list(s) for s in sets])

    def to_rule_list(self, s: int):
        """One rule set as ``(default, [(class, [cond_dict, ...]), ...])``."""
        rules = []
        for r in self.rules_of(s):
            conds = []
            for j in self.conds_of(r):
                d = dict(op=int(self.op[j]), kind=int(self.kind[j]), f=int(self.f[j]),
                         g=int(self.g[j]), coef=np.float32(self.coef[j]),
                         coef2=np.float32(self.coef2[j]), theta=np.float32(self.theta[j]))
                if self.kind[j] == 2:
                    d["mask"] = int(self.cat_mask[j])
                conds.append(d)
            rules.append((int(self.rule_class[r]), conds))
        return int(self.set_default[s]), rules

    def with_params(self, coef, coef2, theta) -> "Population":
        """The same structure with other coefficients and thresholds (fp32)."""
        return Population(self.set_rule_off.copy(), self.set_default.copy(),
                          self.rule_cond_off.copy(), self.rule_class.copy(), self.op.copy(),
                          self.kind.copy(), self.f.copy(), self.g.copy(),
                          np.asarray(coef, np.float32), np.asarray(coef2, np.float32),
                          np.asarray(theta, np.float32), dict(self.meta), self.cat_mask.copy())

    def conds_kind_first(self) -> "Population":
        """Same rule sets with each rule's conditions stably reordered so that
        threshold conditions come before feature-vs-feature ones.  A rule is an
        AND, so the order of its conditions never changes a result."""
        perm = np.arange(self.n_conds)
        for r in range(self.n_rules):
            a, b = int(self.rule_cond_off[r]), int(self.rule_cond_off[r + 1])
            seg = np.arange(a, b)
            perm[a:b] = seg[np.argsort(self.kind[a:b], kind="stable")]
        return Population(self.set_rule_off.copy(), self.set_default.copy(),
                          self.rule_cond_off.copy(), self.rule_class.copy(),
                          self.op[perm], self.kind[perm], self.f[perm], self.g[perm],
                          self.coef[perm], self.coef2[perm], self.theta[perm], dict(self.meta),
                          self.cat_mask[perm])


def from_rule_lists(sets: List) -> Population:
    """Build a population from ``[(default, [(class, [cond, ...]), ...]), ...]``
    where each cond is a dict with keys op, kind, f, g, coef, coef2, theta
    (missing keys default to 0)."""
    set_rule_off, set_default, rule_cond_off, rule_class = [0], [], [0], []
    cols = {k: [] for k in ("op", "kind", "f", "g", "coef", "coef2", "theta", "mask")}
    for default, rules in sets:
        set_default.append(int(default))
        for cls, conds in rules:
            rule_class.append(int(cls))
            for c in conds:
                for k in cols:
                    cols[k].append(c.get(k, 0))
            rule_cond_off.append(len(cols["op"]))
        set_rule_off.append(len(rule_class))
    return Population(np.array(set_rule_off), np.array(set_default), np.array(rule_cond_off),
                      np.array(rule_class, dtype=np.int32),
                      np.array(cols["op"], dtype=np.uint8), np.array(cols["kind"], dtype=np.uint8),
                      np.array(cols["f"], dtype=np.int32), np.array(cols["g"], dtype=np.int32),
                      np.array(cols["coef"], dtype=np.float32), np.array(cols["coef2"], dtype=np.float32),
                      np.array(cols["theta"], dtype=np.float32), {},
                      np.array([int(m) for m in cols["mask"]], dtype=np.uint64))


def concat(pops: Sequence[Population]) -> Population:
    """Concatenate populations (rule sets of the first come first)."""
    sets = []
    for p in pops:
        sets.extend(p.to_rule_list(s) for s in range(p.n_sets))
    return from_rule_lists(sets)
