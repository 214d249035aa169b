"""Fine-tuning of rule coefficients by gradient descent (test infrastructure).

Section 3 of the paper: the sigmoid relaxation gives gradients with respect
to the rule coefficients, which back-propagation uses to adjust them without
changing the logical structure; Section 4.1 applies 50 epochs of gradient
updates per candidate.  The paper names no update rule, so both common ones
are written out here in fp64, plainly, one full-batch step per epoch, with
the gradients of the fp64 oracle (``oracle.soft_backward``, every rule set
weighted 1, i.e. each rule set's own mean loss).

Parameters per condition: the coefficient, plus the threshold of a
threshold condition or the second coefficient of a feature-vs-feature
condition (the other one of that pair is not a parameter and never moves).

Adam follows Kingma & Ba (2015), Algorithm 1: first and second moment
estimates with bias correction, step lr * mhat / (sqrt(vhat) + eps).
"""
from __future__ import annotations

import numpy as np

from .oracle import soft_backward, soft_forward


def _mask(pop):
    """Which entries of (coef, coef2, theta) are parameters."""
    ff = np.asarray(pop.kind) == 1
    return [np.ones(len(ff), bool), ff, ~ff]


def sgd_step(params, grads, mask, lr):
    """p <- p - lr * g on the parameter entries."""
    return [np.where(m, p - lr * g, p) for p, g, m in zip(params, grads, mask)]


def adam_step(params, grads, mask, m1, m2, t, lr, beta1, beta2, eps):
    """One Adam step (t counts from 1); returns (params, m1, m2)."""
    out_p, out_m1, out_m2 = [], [], []
    for p, g, m, a, b in zip(params, grads, mask, m1, m2):
        a = beta1 * a + (1.0 - beta1) * g
        b = beta2 * b + (1.0 - beta2) * g * g
        mhat = a / (1.0 - beta1 ** t)
        vhat = b / (1.0 - beta2 ** t)
        out_p.append(np.where(m, p - lr * mhat / (np.sqrt(vhat) + eps), p))
        out_m1.append(a)
        out_m2.append(b)
    return out_p, out_m1, out_m2


def finetune(x, y, tau, n_classes, pop, epochs, optimizer="adam", lr=0.01, betas=(0.9, 0.999),
             eps=1e-8, start=None, nthreads=0):
    """Runs ``epochs`` full-batch steps from ``start`` (default: the
    population's own parameters).  Returns (params per epoch, losses per
    epoch): params[e] and losses[e] are the values after e updates,
    e = 0..epochs, in fp64."""
    params = [np.asarray(a, np.float64).copy() for a in
              (start if start is not None else (pop.coef, pop.coef2, pop.theta))]
    mask = _mask(pop)
    m1 = [np.zeros_like(p) for p in params]
    m2 = [np.zeros_like(p) for p in params]
    hist_p, hist_l = [], []
    for e in range(epochs + 1):
        hist_p.append([p.copy() for p in params])
        hist_l.append(soft_forward(x, y, tau, n_classes, pop, *params, nthreads=nthreads))
        if e == epochs:
            break
        g = soft_backward(x, y, tau, n_classes, pop, None, *params, nthreads=nthreads)
        if optimizer == "adam":
            params, m1, m2 = adam_step(params, g, mask, m1, m2, e + 1, lr, betas[0], betas[1], eps)
        else:
            params = sgd_step(params, g, mask, lr)
    return hist_p, hist_l
