"""Pins for the oracle's hard (first-firing) evaluation.

Each test checks the oracle against something other than itself: the worked
example of Fig. 1, the closed form of an fp32 product, an independent
exact-arithmetic evaluator on tiny inputs, and invariants of the method.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from oracle import naive
from paper_2406_01821_amd import synth
from paper_2406_01821_amd.population import from_rule_lists, Population

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
OPS = {"<": 0, "<=": 1, ">": 2, ">=": 3}


def tensor_row_to_condition(row, bias):
    """Section 3 / Fig. 1a: a row w with bias b is the test w.x + b > 0.
    One non-zero weight: c*x[f] > -b.  Two non-zero weights and zero bias:
    w_f*x[f] > -w_g*x[g]."""
    nz = [i for i, w in enumerate(row) if w != 0]
    if len(nz) == 1:
        f = nz[0]
        return dict(op=2, kind=0, f=f, g=0, coef=np.float32(row[f]), coef2=np.float32(0),
                    theta=np.float32(-bias))
    assert len(nz) == 2 and bias == 0
    f, g = nz
    return dict(op=2, kind=1, f=f, g=g, coef=np.float32(row[f]), coef2=np.float32(-row[g]),
                theta=np.float32(0))


def fig1():
    with open(os.path.join(GOLDEN, "fig1_ruleset.json")) as fh:
        return json.load(fh)


def fig1_population(default):
    d = fig1()
    cls = d["classes"]
    rules = []
    for name in ("rule1", "rule2"):
        r = d["panel_a_tensors"][name]
        conds = [tensor_row_to_condition(row, b) for row, b in zip(r["conditions"], r["biases"])]
        rules.append((cls[r["class"]], conds))
    return from_rule_lists([(default, rules)])


def reading_holds(reading, feats, row):
    """Evaluate a printed Fig. 1b reading 'feature > const [x feature2]'
    directly with float32 arithmetic."""
    f, op, const, f2 = reading
    lhs = np.float32(row[feats.index(f)])
    rhs = np.float32(const) if f2 is None else np.float32(np.float32(const) * np.float32(row[feats.index(f2)]))
    assert op == ">"
    return bool(lhs > rhs)


def fig1_probe_rows():
    """Rows that put each printed threshold exactly at, just below and just
    above its boundary while the other conditions hold."""
    base = np.array([3.0, 1.0, 1.0, 0.5, 0.5, 0.5], np.float32)
    rows = [base.copy()]
    edges = [(0, np.float32(2.02)), (3, np.float32(0.29)), (4, np.float32(0.43)), (5, np.float32(0.29))]
    for f, t in edges:
        for v in (np.nextafter(t, np.float32(-np.inf)), t, np.nextafter(t, np.float32(np.inf))):
            r = base.copy(); r[f] = v; rows.append(r)
    # feature-vs-feature: x1 against 0.38 * x2
    t = np.float32(np.float32(0.38) * np.float32(1.0))
    for v in (np.nextafter(t, np.float32(-np.inf)), t, np.nextafter(t, np.float32(np.inf))):
        r = base.copy(); r[1] = v; rows.append(r)
    r = base.copy(); r[2] = np.float32(7.0); r[1] = np.float32(2.0); rows.append(r)
    return np.array(rows, np.float32)


@pytest.mark.parametrize("default", [0, 1])
def test_fig1_tensor_form_matches_printed_readings(default):
    d = fig1()
    feats = d["features"]
    pop = fig1_population(default)
    rows = fig1_probe_rows()
    pred = oracle.predict(rows, pop, 0)
    cls = d["classes"]
    for i, row in enumerate(rows):
        expect = default
        for name in ("rule1", "rule2"):
            if all(reading_holds(rd, feats, row) for rd in d["panel_b_readings"][name]):
                expect = cls[d["panel_a_tensors"][name]["class"]]
                break
        assert pred[i] == expect, (i, row, pred[i], expect)


def test_fig1_bias_sign_and_strict_step():
    # bias -2.02 reads "mean radius > 2.02": a sample exactly at 2.02 does not fire
    pop = fig1_population(default=0)
    at = np.array([[2.02, 1.0, 1.0, 0.5, 0.1, 0.1]], np.float32)
    above = at.copy(); above[0, 0] = np.nextafter(np.float32(2.02), np.float32(9))
    assert oracle.predict(at, pop)[0] == 0
    assert oracle.predict(above, pop)[0] == 1


def test_fig1_tuned_readings_direction_flip():
    """Fig. 1c: '-perimeter error > -0.98' is perimeter error < 0.98, and
    '-fde > -7275.88 x wc' is fde < 7275.88 x wc; both stay single rows."""
    d = fig1()
    feats = d["features"]
    cls = d["classes"]
    rules = []
    for name in ("rule1", "rule2"):
        conds = []
        for sgn, f, op, const, f2 in d["panel_c_readings_after_tuning"][name]:
            if f2 is None:
                conds.append(dict(op=OPS[op], kind=0, f=feats.index(f), coef=np.float32(sgn),
                                  theta=np.float32(const)))
            else:
                conds.append(dict(op=OPS[op], kind=1, f=feats.index(f), g=feats.index(f2),
                                  coef=np.float32(sgn), coef2=np.float32(const)))
        rules.append((cls[d["panel_a_tensors"][name]["class"]], conds))
    pop = from_rule_lists([(0, rules)])
    rng = np.random.default_rng(7)
    rows = rng.uniform(-5, 5, size=(4000, 6)).astype(np.float32)
    rows[:, 2] = rng.uniform(-1e-3, 1e-3, size=4000).astype(np.float32)
    pred = oracle.predict(rows, pop)
    x = rows.astype(np.float64)
    r1 = (x[:, 0] > np.float32(0.06)) & (rows[:, 1] < np.float32(np.float32(7275.88) * rows[:, 2])) \
        & (x[:, 3] > np.float32(-3.69))
    r2 = (rows[:, 4] < np.float32(0.98)) & (rows[:, 5] < np.float32(0.24))
    expect = np.where(r1, 1, np.where(r2, 0, 0))
    np.testing.assert_array_equal(pred, expect)
    assert r1.sum() > 50 and (~r1 & r2).sum() > 50


def test_paper_accuracies_are_fractions_of_a_30_percent_split():
    """Fig. 1 / Section 3: 21.05% and 92.40% are both k/171 to two decimals
    (171 = ceil(0.3 * 569)); the data and split are not available, so this
    only records the consistency of the printed numbers."""
    before, after = fig1()["accuracy_before_after_percent"]
    assert round(100 * 36 / 171, 2) == before and round(100 * 158 / 171, 2) == after


def _single_condition_pop(conds):
    """One rule set per condition: rule of class 1 holding that condition,
    default 0, so the prediction is the condition's truth."""
    return from_rule_lists([(0, [(1, [c])]) for c in conds])


def test_fp32_product_closed_form_and_exact_rounding():
    """fl32(c*x) == float32(float64(c)*float64(x)) (the fp64 product of two
    float32 values is exact), checked through the oracle's decisions against
    an exact-rational evaluator, including subnormal and overflowing products."""
    np.seterr(over="ignore")
    rng = np.random.default_rng(11)
    xs = np.concatenate([
        rng.uniform(-4, 4, 40), np.ldexp(rng.uniform(0.5, 1, 10), -140),
        np.ldexp(rng.uniform(0.5, 1, 10), 120), [0.0, -0.0, 1e-45, 3.4e38]]).astype(np.float32)
    cs = np.concatenate([rng.uniform(-2, 2, 12), [1.0, -1.0, 0.0, 1e-30, 7.5e30]]).astype(np.float32)
    conds, expect_rows = [], []
    x = xs.reshape(-1, 1).repeat(2, axis=1)
    x[:, 1] = np.roll(xs, 7)
    for c in cs:
        for op in range(4):
            for t_src in ("at", "mid"):
                prod = (np.float64(c) * x[:, 0].astype(np.float64)).astype(np.float32)
                theta = prod[5] if t_src == "at" else np.float32(0.37)
                conds.append(dict(op=op, kind=0, f=0, coef=c, theta=theta))
            conds.append(dict(op=op, kind=1, f=0, g=1, coef=c, coef2=np.float32(cs[3])))
    pop = _single_condition_pop(conds)
    y = np.zeros(len(xs), np.int32)
    _, conf = oracle.hard_eval(x, y, 2, pop)
    for s, cnd in enumerate(conds):
        lhs = (np.float64(cnd["coef"]) * x[:, 0].astype(np.float64)).astype(np.float32)
        if cnd["kind"] == 1:
            rhs = (np.float64(cnd["coef2"]) * x[:, 1].astype(np.float64)).astype(np.float32)
        else:
            rhs = np.full(len(xs), cnd["theta"], np.float32)
        truth = {0: lhs < rhs, 1: lhs <= rhs, 2: lhs > rhs, 3: lhs >= rhs}[cnd["op"]]
        assert conf[s, 0, 1] == truth.sum(), (s, cnd)
    # exact-rational rounding on a subset, row by row, through predict
    for s in range(0, len(conds), 5):
        pred = oracle.predict(x, pop, s)
        for i in range(len(xs)):
            assert pred[i] == int(naive.condition(conds[s], x[i])), (s, i, conds[s], x[i])


def _alphabet():
    """Small condition alphabet over 3 features with thresholds at sample
    values (ties) and between them, every op, both kinds."""
    conds = []
    for op in range(4):
        for f, t in ((0, 1.0), (1, 0.5), (2, 2.0), (0, 1.5)):
            conds.append(dict(op=op, kind=0, f=f, coef=np.float32(1.0), theta=np.float32(t)))
        conds.append(dict(op=op, kind=1, f=0, g=1, coef=np.float32(0.5), coef2=np.float32(1.0)))
        conds.append(dict(op=op, kind=1, f=2, g=0, coef=np.float32(1.0), coef2=np.float32(2.0)))
    return conds


def test_bruteforce_tiny_against_exact_recursive_evaluator():
    x = np.array([[1.0, 0.5, 2.0], [2.0, 1.0, 1.0], [1.5, 0.75, 3.0], [0.5, 0.25, 1.0],
                  [3.0, 2.0, 0.5]], np.float32)
    y = np.array([0, 1, 1, 0, 1], np.int32)
    alpha = _alphabet()
    rng = np.random.default_rng(5)
    rules = [[c] for c in alpha] + [[alpha[i], alpha[j]] for i, j in itertools.product(range(len(alpha)), repeat=2)]
    sets = []
    for default in (0, 1):
        for r in rules:
            sets.append((default, [(1 - default, r)]))
    for _ in range(3000):
        k = int(rng.integers(1, 3))
        chosen = [(int(rng.integers(2)), rules[int(rng.integers(len(rules)))]) for _ in range(k)]
        sets.append((int(rng.integers(2)), chosen))
    pop = from_rule_lists(sets)
    correct, conf = oracle.hard_eval(x, y, 2, pop)
    for s, rs in enumerate(sets):
        c, m = naive.evaluate(rs, x, y, 2)
        assert correct[s] == c and np.array_equal(conf[s], m), (s, rs)


@pytest.fixture(scope="module")
def small():
    return synth.small_hard(0)


def test_confusion_invariants(small):
    d, pop = small.data, small.pop
    correct, conf = oracle.hard_eval(d.x, d.y, d.n_classes, pop)
    hist = np.bincount(d.y, minlength=d.n_classes)
    assert np.all(conf.sum(axis=(1, 2)) == d.n)
    assert np.array_equal(np.trace(conf, axis1=1, axis2=2), correct)
    assert np.all(conf.sum(axis=2) == hist)


def test_permuting_samples_leaves_counts(small):
    d, pop = small.data, small.pop
    c0, m0 = oracle.hard_eval(d.x, d.y, d.n_classes, pop)
    perm = np.random.default_rng(3).permutation(d.n)
    c1, m1 = oracle.hard_eval(d.x[perm], d.y[perm], d.n_classes, pop)
    assert np.array_equal(c0, c1) and np.array_equal(m0, m1)


def test_default_only_scores_class_prior(small):
    d = small.data
    pop = from_rule_lists([(c, []) for c in range(d.n_classes)])
    correct, _ = oracle.hard_eval(d.x, d.y, d.n_classes, pop)
    assert np.array_equal(correct, np.bincount(d.y, minlength=d.n_classes))


def test_unreachable_and_always_firing_rules(small):
    d, pop = small.data, small.pop
    base, base_conf = oracle.hard_eval(d.x, d.y, d.n_classes, pop)
    never = dict(op=2, kind=0, f=0, coef=np.float32(1.0), theta=np.float32(np.inf))
    always = dict(op=0, kind=0, f=0, coef=np.float32(1.0), theta=np.float32(np.inf))
    appended, prepended, after_always = [], [], []
    for s in range(pop.n_sets):
        default, rules = pop.to_rule_list(s)
        appended.append((default, rules + [(1, [never])]))
        prepended.append((default, [(s % d.n_classes, [always])] + rules))
        after_always.append((default, rules + [(0, [always]), (1, [never])]))
    c1, m1 = oracle.hard_eval(d.x, d.y, d.n_classes, from_rule_lists(appended))
    assert np.array_equal(c1, base) and np.array_equal(m1, base_conf)
    c2, _ = oracle.hard_eval(d.x, d.y, d.n_classes, from_rule_lists(prepended))
    hist = np.bincount(d.y, minlength=d.n_classes)
    assert np.array_equal(c2, hist[np.arange(pop.n_sets) % d.n_classes])
    c3, _ = oracle.hard_eval(d.x, d.y, d.n_classes, from_rule_lists(after_always))
    c4, _ = oracle.hard_eval(d.x, d.y, d.n_classes,
                             from_rule_lists([(0, r + [(0, [always])]) for _, r in
                                              (pop.to_rule_list(s) for s in range(pop.n_sets))]))
    assert np.array_equal(c3, c4)


def test_predict_agrees_with_confusion(small):
    d, pop = small.data, small.pop
    _, conf = oracle.hard_eval(d.x, d.y, d.n_classes, pop)
    for s in (0, 17, 99):
        pred = oracle.predict(d.x, pop, s)
        m = np.zeros((d.n_classes, d.n_classes), np.int64)
        np.add.at(m, (d.y, pred), 1)
        assert np.array_equal(m, conf[s])


def test_threads_do_not_change_results(small):
    d, pop = small.data, small.pop
    a = oracle.hard_eval(d.x, d.y, d.n_classes, pop, nthreads=1)
    b = oracle.hard_eval(d.x, d.y, d.n_classes, pop, nthreads=4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ------------------------------------------------------------- work count
def _naive_work(x, rule_set, tile_rows):
    """Wave-uniform early exit, written as set operations on one tile."""
    default, rules = rule_set
    work_t = work_ff = 0
    undecided = set(tile_rows)
    for _, conds in rules:
        if not undecided:
            break
        alive = set(undecided)
        for c in conds:
            if not alive:
                break
            work_ff += c["kind"] == 1
            work_t += c["kind"] == 0
            alive = {i for i in alive if naive.condition(c, x[i])}
        undecided -= alive
    return work_t, work_ff


def test_workcount_matches_set_simulation():
    w = synth.tiny(21, n=48, nf=4, n_sets=12, rules=(1, 5), conds=(1, 3))
    x, pop = w.data.x, w.pop
    ptr, idx = oracle.label_grouped_tiles(w.data.y, 2, tile=8)
    wt, wf = oracle.workcount(x, pop, ptr, idx)
    for s in range(pop.n_sets):
        rs = pop.to_rule_list(s)
        et = ef = 0
        for t in range(len(ptr) - 1):
            a, b = _naive_work(x, rs, list(idx[ptr[t]:ptr[t + 1]]))
            et += a; ef += b
        assert (wt[s], wf[s]) == (et, ef), s


def test_workcount_bounds_and_first_rule_always_fires(small):
    d, pop = small.data, small.pop
    ptr, idx = oracle.label_grouped_tiles(d.y, d.n_classes, tile=64)
    wt, wf = oracle.workcount(d.x, pop, ptr, idx)
    nominal = pop.nominal_conds_per_set() * (len(ptr) - 1)
    assert np.all(wt + wf <= nominal) and np.all(wt + wf >= 1)
    always = dict(op=0, kind=0, f=0, coef=np.float32(1.0), theta=np.float32(np.inf))
    pop2 = from_rule_lists([(0, [(1, [always, always])] + pop.to_rule_list(s)[1])
                            for s in range(pop.n_sets)])
    wt2, wf2 = oracle.workcount(d.x, pop2, ptr, idx)
    assert np.all(wt2 == 2 * (len(ptr) - 1)) and np.all(wf2 == 0)
