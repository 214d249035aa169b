"""Pins of categorical conditions in the oracle (Section 5 names categorical
features as an extension): the code-set test against the exact-rational
evaluator on every special value, equality as a one-code set, and, in both
soft heads, a categorical condition acting as its truth: one that holds for
every sample changes no loss, one that holds for none removes its rule, and
it has no gradient."""
import numpy as np
import pytest

import oracle
from oracle import naive
from paper_2406_01821_amd import synth
from paper_2406_01821_amd.population import from_rule_lists

SPECIAL = np.array([0.0, -0.0, 1.0, 2.5, -1.0, 63.0, 64.0, 62.999996, 1e9, 3.0000002, 7.0],
                   np.float32)


def table(seed, n=120, num=3, cat=2):
    rng = np.random.default_rng(seed)
    xn = synth.lognormal_features(rng, n, num)
    codes = rng.choice(SPECIAL, size=(n, cat)).astype(np.float32)
    x = np.concatenate([xn, codes], axis=1)
    y = rng.integers(0, 3, size=n).astype(np.int32)
    return x, y


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_code_sets_against_the_exact_evaluator(seed):
    x, y = table(seed)
    rng = np.random.default_rng(100 + seed)
    pop = synth.categorical_population(rng, x, 2, 64, 25, (1, 4), (1, 3), 3, cat_frac=0.6)
    c, m = oracle.hard_eval(x, y, 3, pop)
    for s in range(pop.n_sets):
        rc, rm = naive.evaluate(pop.to_rule_list(s), x, y, 3)
        assert c[s] == rc and np.array_equal(m[s], rm), s


def test_equality_is_a_one_code_set_and_predict_takes_any_value():
    x = np.array([[v] for v in [0.0, -0.0, 1.0, 2.0, 2.5, 63.0, 64.0, np.inf, -np.inf, np.nan]],
                 np.float32)
    for code in (0, 1, 2, 63):
        pop = from_rule_lists([(0, [(1, [dict(kind=2, f=0, mask=1 << code)])])])
        pred = oracle.predict(x, pop, 0)
        with np.errstate(invalid="ignore"):
            want = (x[:, 0] == code).astype(np.int32)
        np.testing.assert_array_equal(pred, want)
    everything = from_rule_lists([(0, [(1, [dict(kind=2, f=0, mask=(1 << 64) - 1)])])])
    np.testing.assert_array_equal(oracle.predict(x, everything, 0), [1, 1, 1, 1, 0, 1, 0, 0, 0, 0])


@pytest.mark.parametrize("head", ["first", "softmax"])
def test_soft_heads_take_the_truth_of_a_categorical_condition(head):
    w = synth.tiny(50, n=200, nf=4, n_classes=3, n_sets=6, rules=(2, 4), conds=(1, 2))
    x = np.concatenate([w.data.x, np.full((200, 1), 5.0, np.float32)], axis=1)
    y = w.data.y
    tau = oracle.tau(x)
    fwd = ((lambda p: oracle.soft_forward(x, y, tau, 3, p)) if head == "first"
           else (lambda p: oracle.smax_forward(x, y, tau, 3, p, 2.0)))
    bwd = ((lambda p: oracle.soft_backward(x, y, tau, 3, p)) if head == "first"
           else (lambda p: oracle.smax_backward(x, y, tau, 3, p, 2.0)))
    base = [w.pop.to_rule_list(s) for s in range(w.pop.n_sets)]
    always = dict(kind=2, f=4, mask=1 << 5)   # every sample holds code 5
    never = dict(kind=2, f=4, mask=1 << 6)
    with_true = [(d, [(c, conds + [always]) for c, conds in rules]) for d, rules in base]
    with_false = [(d, rules[:1] + [(rules[1][0], rules[1][1] + [never])] + rules[2:])
                  for d, rules in base]
    without = [(d, rules[:1] + rules[2:]) for d, rules in base]
    l0 = fwd(from_rule_lists(base))
    np.testing.assert_allclose(fwd(from_rule_lists(with_true)), l0, rtol=1e-14)
    np.testing.assert_allclose(fwd(from_rule_lists(with_false)),
                               fwd(from_rule_lists(without)), rtol=1e-14)
    p = from_rule_lists(with_true)
    g = bwd(p)
    cat = p.kind == 2
    assert all(np.all(a[cat] == 0.0) for a in g)
