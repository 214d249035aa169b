"""GPU parity of on-device fine-tuning (aerl_finetune) against the fp64
reference loop of oracle/tune.py, which takes its gradients from the fp64
oracle adjoint:
  * the fused optimizer update itself, fed the library's own gradients,
    agrees with fp64 Adam to fp32 rounding;
  * plain gradient descent, epoch by epoch, stays within the drift that the
    soft-path gradient tolerance allows, and the loss history within the
    forward tolerance;
  * Adam over several epochs: loss history within tolerance, parameters
    within the drift the gradient tolerance allows (an entry whose gradient
    is below that tolerance may step either way, Adam's step being
    sign-like);
  * the structure never moves, and the tuned rule sets scored with the step
    activation are bit-exact against the oracle."""
import numpy as np
import pytest

import oracle
from oracle import tune
from paper_2406_01821_amd import synth

pytestmark = pytest.mark.gpu

LR = 0.01


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2406_01821_amd.aerl import Context
    c = Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _dev(ctx, pop):
    import torch
    return [torch.tensor(a, device=ctx.device) for a in (pop.coef, pop.coef2, pop.theta)]


def _host(ts):
    return [t.detach().cpu().numpy().astype(np.float64) for t in ts]


def _grad_tol(g64):
    """The soft-path gradient tolerance, per entry."""
    out = []
    for g in g64:
        s = np.abs(g).max() if g.size else 0.0
        out.append(1e-4 * np.maximum(np.abs(g), 1e-3 * s))
    return out


def _setup(ctx, w):
    ds = ctx.upload_dataset(w.data)
    p = ctx.pack_population(w.pop, w.data.n_features, w.data.n_classes)
    return ds, p, oracle.tau(w.data.x)


def test_adam_update_matches_fp64_adam_on_the_same_gradients(ctx):
    import torch
    w = synth.tiny(21, n=2500, nf=9, n_classes=3, n_sets=30, rules=(1, 6), conds=(1, 4),
                   ff_frac=0.4)
    ds, p, _ = _setup(ctx, w)
    par = _dev(ctx, w.pop)
    ones = torch.ones(w.pop.n_sets, device=ctx.device)
    mask = tune._mask(w.pop)
    ref = [a.astype(np.float64) for a in (w.pop.coef, w.pop.coef2, w.pop.theta)]
    m1 = [np.zeros(w.pop.n_conds)] * 3
    m2 = [np.zeros(w.pop.n_conds)] * 3
    for e in range(1, 4):
        # the library's own gradient at the current parameters (the adjoint
        # is deterministic, so this is the gradient the update consumes)
        cur = [t.clone() for t in par]
        g = _host(ctx.soft_backward(ds, p, *cur, ones))
        start = _host(cur)
        # one epoch from each epoch's start needs the moments of the earlier
        # ones: rerun all e epochs from the beginning
        run = _dev(ctx, w.pop)
        ctx.finetune(ds, p, *run, epochs=e, optimizer="adam", lr=LR)
        ref, m1, m2 = tune.adam_step(start, g, mask, m1, m2, e, LR, 0.9, 0.999, 1e-8)
        got = _host(run)
        for a, b in zip(got, ref):
            np.testing.assert_allclose(a, b, rtol=2e-6, atol=1e-7)
        par = run


def test_sgd_epoch_by_epoch(ctx):
    w = synth.tiny(22, n=3000, nf=9, n_classes=2, n_sets=40, rules=(1, 8), conds=(1, 4),
                   ff_frac=0.3)
    ds, p, tau = _setup(ctx, w)
    E = 4
    ps, ls = tune.finetune(w.data.x, w.data.y, tau, 2, w.pop, E, optimizer="sgd", lr=LR)
    par = _dev(ctx, w.pop)
    hist = _host([ctx.finetune(ds, p, *par, epochs=E, optimizer="sgd", lr=LR,
                               loss_history=True)])[0]
    drift = [np.zeros(w.pop.n_conds) for _ in range(3)]
    gpu = _dev(ctx, w.pop)
    for e in range(1, E + 1):
        g64 = oracle.soft_backward(w.data.x, w.data.y, tau, 2, w.pop, None, *ps[e - 1])
        drift = [d + LR * t + 2e-7 * np.abs(q) for d, t, q in zip(drift, _grad_tol(g64), ps[e])]
        ctx.finetune(ds, p, *gpu, epochs=1, optimizer="sgd", lr=LR)
        for a, b, d in zip(_host(gpu), ps[e], drift):
            assert np.all(np.abs(a - b) <= 1.5 * d + 1e-7), (e, np.abs(a - b).max())
        np.testing.assert_allclose(hist[e], ls[e], rtol=2e-5, atol=1e-6)
    # one call of E epochs equals E calls of one (no optimizer state)
    for a, b in zip(_host(par), _host(gpu)):
        np.testing.assert_array_equal(a, b)


def test_adam_trajectory_and_structure(ctx):
    w = synth.tiny(23, n=3000, nf=9, n_classes=3, n_sets=40, rules=(1, 8), conds=(1, 4),
                   ff_frac=0.3)
    ds, p, tau = _setup(ctx, w)
    E = 5
    ps, ls = tune.finetune(w.data.x, w.data.y, tau, 3, w.pop, E, optimizer="adam", lr=LR)
    par = _dev(ctx, w.pop)
    hist = _host([ctx.finetune(ds, p, *par, epochs=E, optimizer="adam", lr=LR,
                               loss_history=True)])[0]
    for e in range(E + 1):
        np.testing.assert_allclose(hist[e], ls[e], rtol=1e-4, atol=1e-6)
    # an entry whose fp64 gradient stays at or above 1e-5 of its array's
    # largest at every epoch carries a gradient error of at most 1e-2
    # relative, small against the step; an entry below that may step either
    # way (Adam's step is sign-like), by at most lr per epoch
    clear = [np.ones(w.pop.n_conds, bool) for _ in range(3)]
    for e in range(E):
        g64 = oracle.soft_backward(w.data.x, w.data.y, tau, 3, w.pop, None, *ps[e])
        for k, g in enumerate(g64):
            clear[k] &= np.abs(g) >= 1e-5 * np.abs(g).max()
    got = _host(par)
    mask = tune._mask(w.pop)
    for k in range(3):
        d = np.abs(got[k] - ps[E][k])
        sel = clear[k] & mask[k]
        close = d[mask[k]] <= 1e-3 * LR * E + 1e-6
        print(f"array {k}: {sel.sum()} of {mask[k].sum()} clear, worst drift of a clear entry "
              f"{d[sel].max() / (LR * E) if sel.any() else 0:.2e} x lr*E; "
              f"{close.mean():.4f} of all entries within 1e-3 lr*E")
        assert np.all(d[sel] <= 1e-2 * LR * E + 1e-6), (k, d[sel].max())
        assert np.all(d <= 2 * LR * E + 1e-6), (k, d.max())
        assert close.mean() >= 0.95
    # the structure is untouched: no threshold on feature-vs-feature
    # conditions, no second coefficient on threshold ones
    ff = w.pop.kind == 1
    np.testing.assert_array_equal(got[1][~ff], w.pop.coef2[~ff])
    np.testing.assert_array_equal(got[2][ff], w.pop.theta[ff])


def test_fifty_epochs_on_the_breast_cancer_shape_then_hard_rescore(ctx):
    """569 x 30, 100 rule sets, 50 Adam epochs (Section 4.1's count); the
    tuned rule sets, repacked, score bit-exactly as the oracle scores them,
    and the soft loss of the pool goes down."""
    import torch
    w = synth.small_hard(0)
    ds, p, tau = _setup(ctx, w)
    par = _dev(ctx, w.pop)
    hist = _host([ctx.finetune(ds, p, *par, epochs=50, optimizer="adam", lr=0.05,
                               loss_history=True)])[0]
    assert hist.shape == (51, w.pop.n_sets)
    assert hist[50].mean() < hist[0].mean()
    tuned = w.pop.with_params(*[t.cpu().numpy() for t in par])
    np.testing.assert_allclose(hist[50], oracle.soft_forward(w.data.x, w.data.y, tau, 2, tuned),
                               rtol=1e-5, atol=1e-6)
    pt = ctx.pack_population(tuned, 30, 2)
    c, m = ctx.eval_population(ds, pt)
    torch.cuda.synchronize()
    rc, rm = oracle.hard_eval(w.data.x, w.data.y, 2, tuned)
    np.testing.assert_array_equal(c.cpu().numpy(), rc)
    np.testing.assert_array_equal(m.cpu().numpy(), rm)
    c0, _ = oracle.hard_eval(w.data.x, w.data.y, 2, w.pop)
    print(f"mean accuracy {c0.mean() / 569:.4f} -> {rc.mean() / 569:.4f} after 50 epochs")


def test_bad_configurations_are_refused(ctx):
    from paper_2406_01821_amd.aerl import AerlError, AERL_EINVAL
    w = synth.tiny(24, n=200, nf=5, n_sets=3)
    ds, p, _ = _setup(ctx, w)
    par = _dev(ctx, w.pop)
    for kw in (dict(lr=0.0), dict(lr=float("nan")), dict(betas=(1.0, 0.9)), dict(eps=0.0),
               dict(epochs=-1)):
        args = dict(epochs=2, optimizer="adam", lr=LR)
        args.update(kw)
        with pytest.raises(AerlError) as e:
            ctx.finetune(ds, p, *par, **args)
        assert e.value.status == AERL_EINVAL
