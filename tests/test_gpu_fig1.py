"""The paper's worked example (Fig. 1: the rule tensors of panel a, the
readings of panel b and the tuned readings of panel c, kept in
tests/golden/fig1_ruleset.json) on the GPU: predictions on rows placed just
below, at and just above every printed threshold, fitness counts of those
rows, the tuned rule set's direction flips on random rows, and the soft loss
of the rule set, each against the oracle (which the oracle tests pin to the
printed readings)."""
import numpy as np
import pytest

import oracle
from paper_2406_01821_amd.population import Dataset, from_rule_lists
from test_oracle_hard import OPS, fig1, fig1_population, fig1_probe_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2406_01821_amd.aerl import Context
    c = Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.mark.parametrize("default", [0, 1])
def test_fig1_predictions_and_counts_at_every_printed_threshold(ctx, default):
    import torch
    pop = fig1_population(default)
    rows = fig1_probe_rows()
    p = ctx.pack_population(pop, 6, 2)
    got = ctx.predict(p, rows, 0)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), oracle.predict(rows, pop, 0))
    y = (np.arange(len(rows)) % 2).astype(np.int32)
    data = Dataset(rows, y, 2, "fig1-probes")
    ds = ctx.upload_dataset(data)
    c, m = ctx.eval_population(ds, p)
    torch.cuda.synchronize()
    rc, rm = oracle.hard_eval(rows, y, 2, pop)
    np.testing.assert_array_equal(c.cpu().numpy(), rc)
    np.testing.assert_array_equal(m.cpu().numpy(), rm)


def test_fig1_tuned_rule_set_on_random_rows(ctx):
    """Panel c's readings ('-perimeter error > -0.98' and the like) on 4000
    random rows, predicted on the GPU and compared with the readings
    evaluated directly."""
    import torch
    d = fig1()
    feats, cls = d["features"], d["classes"]
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
    p = ctx.pack_population(pop, 6, 2)
    got = ctx.predict(p, rows, 0)
    torch.cuda.synchronize()
    x = rows.astype(np.float64)
    r1 = (x[:, 0] > np.float32(0.06)) & (rows[:, 1] < np.float32(np.float32(7275.88) * rows[:, 2])) \
        & (x[:, 3] > np.float32(-3.69))
    r2 = (rows[:, 4] < np.float32(0.98)) & (rows[:, 5] < np.float32(0.24))
    np.testing.assert_array_equal(got.cpu().numpy(), np.where(r1, 1, np.where(r2, 0, 0)))


def test_fig1_soft_loss(ctx):
    import torch
    pop = fig1_population(0)
    rng = np.random.default_rng(11)
    rows = rng.uniform(0.0, 4.0, size=(3000, 6)).astype(np.float32)
    y = rng.integers(0, 2, size=3000).astype(np.int32)
    data = Dataset(rows, y, 2, "fig1-soft")
    ds = ctx.upload_dataset(data)
    p = ctx.pack_population(pop, 6, 2)
    par = [torch.tensor(a, device=ctx.device) for a in (pop.coef, pop.coef2, pop.theta)]
    loss = ctx.soft_forward(ds, p, *par)
    torch.cuda.synchronize()
    ref = oracle.soft_forward(rows, y, oracle.tau(rows), 2, pop)
    got = loss.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref) <= 1e-5 * np.abs(ref) + 1e-6), (got, ref)
