"""Pins of the fine-tuning reference (oracle/tune.py) against closed forms:
Adam's first step and its steps under a constant gradient, plain gradient
descent, parameters that are not parameters never moving, and one step of
the loop on a single rule with a single condition, whose gradient has a
closed form (no call to the oracle's adjoint)."""
import numpy as np

import oracle
from oracle import tune
from paper_2406_01821_amd.population import from_rule_lists


def test_adam_first_step_is_lr_times_g_over_abs_g_plus_eps():
    rng = np.random.default_rng(0)
    g = [rng.normal(size=7) * 10.0 ** rng.integers(-6, 3, size=7) for _ in range(3)]
    p0 = [rng.normal(size=7) for _ in range(3)]
    mask = [np.ones(7, bool)] * 3
    z = [np.zeros(7)] * 3
    p1, m1, m2 = tune.adam_step(p0, g, mask, z, z, 1, 0.05, 0.9, 0.999, 1e-8)
    for a, b, gg in zip(p0, p1, g):
        np.testing.assert_allclose(a - b, 0.05 * gg / (np.abs(gg) + 1e-8), rtol=1e-12, atol=1e-15)


def test_adam_constant_gradient_moves_the_same_each_step():
    """With a constant gradient the bias-corrected moments are g and g^2, so
    every step is lr * g / (|g| + eps)."""
    g = [np.array([3.0, -0.25, 1e-3])] * 3
    mask = [np.ones(3, bool)] * 3
    p = [np.zeros(3)] * 3
    m1 = [np.zeros(3)] * 3
    m2 = [np.zeros(3)] * 3
    for t in range(1, 6):
        p, m1, m2 = tune.adam_step(p, g, mask, m1, m2, t, 0.01, 0.9, 0.999, 1e-8)
    step = 0.01 * g[0] / (np.abs(g[0]) + 1e-8)
    for a in p:
        np.testing.assert_allclose(a, -5 * step, rtol=1e-12)


def test_sgd_and_mask():
    p = [np.array([1.0, 2.0]), np.array([3.0, 4.0]), np.array([5.0, 6.0])]
    g = [np.array([1.0, -1.0])] * 3
    mask = [np.array([True, True]), np.array([False, True]), np.array([True, False])]
    q = tune.sgd_step(p, g, mask, 0.5)
    np.testing.assert_array_equal(q[0], [0.5, 2.5])
    np.testing.assert_array_equal(q[1], [3.0, 4.5])
    np.testing.assert_array_equal(q[2], [4.5, 6.0])
    z = [np.zeros(2)] * 3
    r, _, _ = tune.adam_step(p, g, mask, z, z, 1, 0.5, 0.9, 0.999, 1e-8)
    assert r[1][0] == 3.0 and r[2][1] == 6.0


def test_loop_step_on_one_condition_matches_the_closed_form():
    """One rule of class 1 with x > theta, default class 0, one sample of
    label 1: L = softplus(-z), z = (c x - theta) / tau, so
    dL/dtheta = sigmoid(-z) / tau and dL/dc = -x sigmoid(-z) / tau."""
    x = np.array([[2.0]], np.float32)
    y = np.array([1], np.int32)
    tau = np.array([0.5], np.float32)
    c0, t0 = 0.75, 1.25
    pop = from_rule_lists([(0, [(1, [dict(op=2, kind=0, f=0, coef=np.float32(c0),
                                          theta=np.float32(t0))])])])
    ps, ls = tune.finetune(x, y, tau, 2, pop, 1, optimizer="sgd", lr=0.1)
    z = (np.float64(np.float32(c0)) * 2.0 - np.float64(np.float32(t0))) / 0.5
    sig = 1.0 / (1.0 + np.exp(z))  # sigmoid(-z)
    np.testing.assert_allclose(ls[0][0], np.log1p(np.exp(-z)), rtol=1e-12)
    np.testing.assert_allclose(ps[1][2][0], np.float32(t0) - 0.1 * sig / 0.5, rtol=1e-12)
    np.testing.assert_allclose(ps[1][0][0], np.float32(c0) + 0.1 * 2.0 * sig / 0.5, rtol=1e-12)
    assert ps[1][1][0] == 0.0  # a threshold condition has no second coefficient
    assert ls[1][0] < ls[0][0]


def test_zero_epochs_and_descent():
    from paper_2406_01821_amd import synth
    w = synth.tiny(3, n=300, nf=6, n_classes=2, n_sets=6, rules=(1, 4), conds=(1, 3), ff_frac=0.3)
    tau = oracle.tau(w.data.x)
    ps, ls = tune.finetune(w.data.x, w.data.y, tau, 2, w.pop, 0)
    assert len(ps) == 1
    np.testing.assert_array_equal(ps[0][0], w.pop.coef.astype(np.float64))
    ps, ls = tune.finetune(w.data.x, w.data.y, tau, 2, w.pop, 3, optimizer="sgd", lr=1e-4)
    # small steps along the negative gradient do not raise any rule set's loss
    assert np.all(ls[3] <= ls[0] + 1e-12)
    ff = w.pop.kind == 1
    np.testing.assert_array_equal(ps[3][1][~ff], w.pop.coef2[~ff])
    np.testing.assert_array_equal(ps[3][2][ff], w.pop.theta[ff])
