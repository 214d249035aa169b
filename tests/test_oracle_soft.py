"""Pins for the oracle's soft (sigmoid-relaxed) loss and its gradient.

The paper only says that a sigmoid replaces the step for back-propagation
(Section 3); the exact relaxation is this project's reading (first-firing
probabilities, cross-entropy, tau = 0.05 std).  These tests pin the fp64
oracle to closed forms, to normalisation, to the hard path in the tau -> 0
limit, to a naive probability-space evaluation and to finite differences.
"""
import numpy as np
import pytest
from scipy.special import expit, logsumexp

import oracle
from paper_2406_01821_amd import synth
from paper_2406_01821_amd.population import from_rule_lists


def z_of(cond, x, tau):
    """Soft margin of one condition for every row, written out directly."""
    s = 1.0 if cond["op"] >= 2 else -1.0
    lhs = np.float64(cond["coef"]) * x[:, cond["f"]].astype(np.float64)
    if cond.get("kind", 0) == 1:
        rhs = np.float64(cond["coef2"]) * x[:, cond["g"]].astype(np.float64)
    else:
        rhs = np.float64(cond["theta"])
    return s * (lhs - rhs) / np.float64(tau[cond["f"]])


@pytest.fixture(scope="module")
def sub():
    w = synth.tiny(31, n=64, nf=8, n_sets=6, rules=(1, 5), conds=(1, 3), ff_frac=0.3)
    t = oracle.tau(w.data.x)
    return w, t


def test_tau_is_five_percent_of_population_std():
    w = synth.tiny(2, n=500, nf=6)
    x = w.data.x.copy()
    x[:, 3] = 2.5  # constant column -> tau 1
    t = oracle.tau(x)
    expect = (0.05 * np.std(x.astype(np.float64), axis=0)).astype(np.float32)
    expect[3] = 1.0
    np.testing.assert_array_equal(t, expect)


@pytest.mark.parametrize("op", [0, 1, 2, 3])
@pytest.mark.parametrize("kind", [0, 1])
def test_single_rule_single_condition_closed_form(op, kind):
    rng = np.random.default_rng(op + 4 * kind)
    x = rng.uniform(0.5, 3.0, size=(300, 3)).astype(np.float32)
    y = rng.integers(0, 2, size=300).astype(np.int32)
    tau = np.array([0.3, 0.2, 0.25], np.float32)
    cond = dict(op=op, kind=kind, f=0, g=1, coef=np.float32(0.8), coef2=np.float32(0.9),
                theta=np.float32(1.4) if kind == 0 else np.float32(0))
    for cls, default in ((1, 0), (0, 1)):
        pop = from_rule_lists([(default, [(cls, [cond])])])
        loss = oracle.soft_forward(x, y, tau, 2, pop)[0]
        z = z_of(cond, x, tau)
        # P(rule class) = sigmoid(z); P(default) = sigmoid(-z)
        L = np.where(y == cls, np.logaddexp(0, -z), np.logaddexp(0, z))
        assert loss == pytest.approx(np.minimum(L, 100).mean(), rel=1e-13)
        g1, g2, g3 = oracle.soft_backward(x, y, tau, 2, pop)
        dLdz = np.where(y == cls, -expit(-z), expit(z))
        s = 1.0 if op >= 2 else -1.0
        dz_dc = s * x[:, 0].astype(np.float64) / np.float64(tau[0])
        assert g1[0] == pytest.approx((dLdz * dz_dc).mean(), rel=1e-12)
        if kind == 0:
            assert g3[0] == pytest.approx((dLdz * -s / np.float64(tau[0])).mean(), rel=1e-12)
            assert g2[0] == 0
        else:
            dz_dc2 = -s * x[:, 1].astype(np.float64) / np.float64(tau[0])
            assert g2[0] == pytest.approx((dLdz * dz_dc2).mean(), rel=1e-12)
            assert g3[0] == 0


def test_class_probabilities_sum_to_one(sub):
    w, tau = sub
    for s in range(w.pop.n_sets):
        lp = oracle.soft_logprobs(w.data.x, tau, 2, w.pop, s)
        np.testing.assert_allclose(logsumexp(lp, axis=1), 0.0, atol=1e-12)


def test_log_space_matches_naive_probability_space(sub):
    w, tau = sub
    wide = tau * np.float32(50)  # keeps every sigmoid away from saturation
    a = oracle.soft_forward(w.data.x, w.data.y, wide, 2, w.pop)
    b = oracle.soft_forward_naive(w.data.x, w.data.y, wide, 2, w.pop)
    np.testing.assert_allclose(a, b, rtol=1e-12)


def test_small_tau_limit_recovers_hard_prediction():
    w = synth.tiny(8, n=400, nf=6, n_sets=15, rules=(1, 6), conds=(1, 3), n_classes=3)
    x, pop = w.data.x, w.pop
    tau = oracle.tau(x) * np.float32(1e-3)
    for s in range(pop.n_sets):
        lp = oracle.soft_logprobs(x, tau, 3, pop, s)
        hard = oracle.predict(x, pop, s)
        margins = np.full(x.shape[0], np.inf)
        default, rules = pop.to_rule_list(s)
        for _, conds in rules:
            for c in conds:
                margins = np.minimum(margins, np.abs(z_of(c, x, tau)))
        ok = margins > 30
        assert ok.sum() > 100
        np.testing.assert_array_equal(lp.argmax(axis=1)[ok], hard[ok])


def test_unsatisfiable_rule_changes_nothing(sub):
    w, tau = sub
    never = dict(op=2, kind=0, f=1, coef=np.float32(1.0), theta=np.float32(np.inf))
    sets = [w.pop.to_rule_list(s) for s in range(w.pop.n_sets)]
    pop2 = from_rule_lists([(d, rules[:1] + [(1, [never])] + rules[1:]) for d, rules in sets])
    a = oracle.soft_forward(w.data.x, w.data.y, tau, 2, w.pop)
    b = oracle.soft_forward(w.data.x, w.data.y, tau, 2, pop2)
    np.testing.assert_array_equal(a, b)


def test_gradient_matches_central_finite_differences(sub):
    w, tau = sub
    x, y, pop = w.data.x, w.data.y, w.pop
    for s in range(pop.n_sets):
        lp = oracle.soft_logprobs(x, tau, 2, pop, s)
        nll = -lp[np.arange(len(y)), y]
        assert not np.any(np.abs(nll - 100) < 1e-3)
    dloss = np.linspace(0.5, 1.5, pop.n_sets)
    g1, g2, g3 = oracle.soft_backward(x, y, tau, 2, pop, dloss=dloss)
    base = [pop.coef.astype(np.float64), pop.coef2.astype(np.float64), pop.theta.astype(np.float64)]
    meanabs = np.abs(x.astype(np.float64)).mean(axis=0)

    def total(params):
        return float(np.dot(dloss, oracle.soft_forward(x, y, tau, 2, pop, *params)))

    checked = 0
    for j in range(pop.n_conds):
        f = pop.f[j]
        which = [0, 1 if pop.kind[j] else 2]
        for w_idx in which:
            h = 1e-4 * float(tau[f]) / (meanabs[f] if w_idx < 2 else 1.0)
            if w_idx == 1:
                h = 1e-4 * float(tau[f]) / meanabs[pop.g[j]]
            plus = [p.copy() for p in base]; minus = [p.copy() for p in base]
            plus[w_idx][j] += h; minus[w_idx][j] -= h
            fd = (total(plus) - total(minus)) / (2 * h)
            an = (g1, g2, g3)[w_idx][j]
            assert an == pytest.approx(fd, rel=1e-6, abs=1e-9), (j, w_idx, an, fd)
            checked += 1
    assert checked > 30


def test_mirror_symmetry_single_condition():
    """Swapping the rule's class with the default and flipping the op's
    direction (z -> -z) leaves the loss and the threshold gradient unchanged."""
    rng = np.random.default_rng(9)
    x = rng.uniform(0.5, 3.0, size=(200, 2)).astype(np.float32)
    y = rng.integers(0, 2, size=200).astype(np.int32)
    tau = np.array([0.2, 0.3], np.float32)
    c1 = dict(op=2, kind=0, f=0, coef=np.float32(0.7), theta=np.float32(1.1))
    c2 = dict(c1, op=0)
    p1 = from_rule_lists([(0, [(1, [c1])])])
    p2 = from_rule_lists([(1, [(0, [c2])])])
    l1 = oracle.soft_forward(x, y, tau, 2, p1)
    l2 = oracle.soft_forward(x, y, tau, 2, p2)
    assert l1[0] == pytest.approx(l2[0], rel=1e-14)
    g1 = oracle.soft_backward(x, y, tau, 2, p1)
    g2 = oracle.soft_backward(x, y, tau, 2, p2)
    assert g1[2][0] == pytest.approx(g2[2][0], rel=1e-12)
    assert g1[0][0] == pytest.approx(g2[0][0], rel=1e-12)


def test_clamped_samples_have_zero_gradient():
    x = np.array([[10.0], [10.0]], np.float32)
    y = np.array([0, 0], np.int32)
    tau = np.array([0.01], np.float32)
    # rule of class 1 fires with certainty (z = 900), label 0: P_y ~ exp(-900)
    pop = from_rule_lists([(0, [(1, [dict(op=2, kind=0, f=0, coef=np.float32(1), theta=np.float32(1))])])])
    assert oracle.soft_forward(x, y, tau, 2, pop)[0] == 100.0
    g = oracle.soft_backward(x, y, tau, 2, pop)
    assert g[0][0] == 0 and g[2][0] == 0
