"""Pins of the softmax head in the oracle (rule votes through a softmax,
the probabilistic-output variant of the paper's Section 5): the closed form
of one rule with one condition, normalisation, indifference to the order of
the rules, beta = 0, a vectorised numpy evaluation written separately from
the C code, and fp64 central finite differences of the gradient."""
import numpy as np
import pytest

import oracle
from paper_2406_01821_amd import synth
from paper_2406_01821_amd.population import from_rule_lists


def _numpy_votes(x, tau, pop, s, coef, coef2, theta):
    """Votes [n][C] from the definition, vectorised over samples."""
    n = x.shape[0]
    C = int(max(pop.rule_class.max(initial=0), pop.set_default.max())) + 1
    v = np.zeros((n, max(C, 2)))
    none = np.ones(n)
    for k in pop.rules_of(s):
        r = np.ones(n)
        for j in pop.conds_of(k):
            f = pop.f[j]
            rhs = coef2[j] * x[:, pop.g[j]].astype(np.float64) if pop.kind[j] else theta[j]
            z = (1.0 if pop.op[j] >= 2 else -1.0) * (coef[j] * x[:, f].astype(np.float64) - rhs) / tau[f]
            r = r * (1.0 / (1.0 + np.exp(-z)))
        v[:, pop.rule_class[k]] += r
        none = none * (1.0 - r)
    v[:, pop.set_default[s]] += none
    return v


def test_one_rule_one_condition_closed_form():
    x = np.array([[0.3], [1.7], [2.5]], np.float32)
    tau = np.array([0.8], np.float32)
    pop = from_rule_lists([(0, [(1, [dict(op=2, kind=0, f=0, coef=np.float32(1.5),
                                          theta=np.float32(2.0))])])])
    for beta in (0.5, 3.0):
        P = oracle.smax_probs(x, tau, 2, pop, 0, beta)
        z = (1.5 * x[:, 0].astype(np.float64) - 2.0) / np.float64(tau[0])
        sig = 1.0 / (1.0 + np.exp(-z))
        p1 = 1.0 / (1.0 + np.exp(beta * (1.0 - 2.0 * sig)))  # votes sig vs 1 - sig
        np.testing.assert_allclose(P[:, 1], p1, rtol=1e-13)
        np.testing.assert_allclose(P.sum(axis=1), 1.0, rtol=1e-14)
        y = np.array([1, 0, 1], np.int32)
        L = oracle.smax_forward(x, y, tau, 2, pop, beta)
        want = np.mean(-np.log(np.where(y == 1, p1, 1.0 - p1)))
        np.testing.assert_allclose(L[0], want, rtol=1e-13)


def test_matches_a_separate_numpy_evaluation_and_sums_to_one():
    w = synth.tiny(41, n=200, nf=7, n_classes=3, n_sets=12, rules=(1, 6), conds=(1, 3), ff_frac=0.4)
    tau = oracle.tau(w.data.x)
    c = [a.astype(np.float64) for a in (w.pop.coef, w.pop.coef2, w.pop.theta)]
    for s in range(w.pop.n_sets):
        v = _numpy_votes(w.data.x, tau, w.pop, s, *c)[:, :3]
        e = np.exp(2.0 * v - (2.0 * v).max(axis=1, keepdims=True))
        want = e / e.sum(axis=1, keepdims=True)
        got = oracle.smax_probs(w.data.x, tau, 3, w.pop, s, 2.0)
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(got.sum(axis=1), 1.0, rtol=1e-14)


def test_rule_order_does_not_matter_and_beta_zero_is_uniform():
    w = synth.tiny(42, n=150, nf=6, n_classes=3, n_sets=8, rules=(2, 6), conds=(1, 3))
    tau = oracle.tau(w.data.x)
    rng = np.random.default_rng(0)
    sets = []
    for s in range(w.pop.n_sets):
        d, rules = w.pop.to_rule_list(s)
        sets.append((d, [rules[i] for i in rng.permutation(len(rules))]))
    perm = from_rule_lists(sets)
    a = oracle.smax_forward(w.data.x, w.data.y, tau, 3, w.pop, 1.5)
    b = oracle.smax_forward(w.data.x, w.data.y, tau, 3, perm, 1.5)
    np.testing.assert_allclose(a, b, rtol=1e-13)
    np.testing.assert_allclose(oracle.smax_forward(w.data.x, w.data.y, tau, 3, w.pop, 0.0),
                               np.log(3.0), rtol=1e-14)
    g = oracle.smax_backward(w.data.x, w.data.y, tau, 3, w.pop, 0.0)
    assert all(np.all(x == 0.0) for x in g)


@pytest.mark.parametrize("beta", [1.0, 4.0])
def test_gradient_against_central_differences(beta):
    w = synth.tiny(43, n=64, nf=8, n_classes=3, n_sets=5, rules=(1, 5), conds=(1, 3), ff_frac=0.3)
    x, y, pop = w.data.x, w.data.y, w.pop
    tau = oracle.tau(x)
    base = [pop.coef.astype(np.float64), pop.coef2.astype(np.float64), pop.theta.astype(np.float64)]
    g = oracle.smax_backward(x, y, tau, 3, pop, beta)
    meanabs = np.abs(x.astype(np.float64)).mean(axis=0)
    for j in range(pop.n_conds):
        f = pop.f[j]
        for k in ([0, 1] if pop.kind[j] else [0, 2]):
            h = 1e-6 * float(tau[f]) / (meanabs[pop.g[j] if k == 1 else f] if k < 2 else 1.0)
            plus = [b.copy() for b in base]
            minus = [b.copy() for b in base]
            plus[k][j] += h
            minus[k][j] -= h
            # the parameter moves only its own rule set's loss
            s = int(np.searchsorted(pop.rule_cond_off, j, side="right")) - 1
            s = int(np.searchsorted(pop.set_rule_off, s, side="right")) - 1
            lp = oracle.smax_forward(x, y, tau, 3, pop, beta, *plus)[s]
            lm = oracle.smax_forward(x, y, tau, 3, pop, beta, *minus)[s]
            fd = (lp - lm) / (2 * h)
            scale = max(abs(fd), 1e-3 * max(np.abs(gg).max() for gg in g))
            roundoff = 8 * np.finfo(np.float64).eps * abs(lp) / h
            assert abs(g[k][j] - fd) <= 1e-5 * scale + roundoff, (j, k, g[k][j], fd)
