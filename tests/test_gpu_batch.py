"""GPU parity of the ragged batch: many (dataset, population) evaluations in
one persistent launch, optionally captured in a hipGraph, give the same
integer counts as the oracle and as the one-launch-per-population path, for
every work split (Section 3 semantics; Section 5: CPU and GPU results are
equivalent)."""
import numpy as np
import pytest

import limits
import oracle
from paper_2406_01821_amd import synth
from paper_2406_01821_amd.population import from_rule_lists

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2406_01821_amd.aerl import Context
    c = Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def small_runs():
    """Twelve runs of mixed shapes: tiny and mid-sized datasets, 16-128
    features, 2-4 classes, rule sets of 1-64 rules x 1-8 conditions."""
    return synth.ragged_runs(12, seed0=3100, n_range=(1, 12_000), p_range=(1, 200))


@pytest.fixture(scope="module")
def runs(ctx):
    ws = small_runs()
    devs = []
    for w in ws:
        ds = ctx.upload_dataset(w.data)
        p = ctx.pack_population(w.pop, w.data.n_features, w.data.n_classes)
        devs.append((ds, p))
    refs = [oracle.hard_eval(w.data.x, w.data.y, w.data.n_classes, w.pop) for w in ws]
    yield ws, devs, refs
    for ds, p in devs:
        ctx.release_population(p)
        ctx.release_dataset(ds)


def make_items(ctx, devs, confusion=True):
    items = []
    for ds, p in devs:
        c, m = ctx.batch_outputs(ds, p, confusion)
        items.append((ds, p, c, m))
    return items


def check_items(items, refs, confusion=True):
    for k, ((ds, p, c, m), (rc, rm)) in enumerate(zip(items, refs)):
        np.testing.assert_array_equal(c.cpu().numpy(), rc, err_msg=f"item {k} correct")
        if confusion:
            np.testing.assert_array_equal(m.cpu().numpy(), rm, err_msg=f"item {k} confusion")


@pytest.mark.parametrize("cfg", [None, (1, 1), (3, 2), (16, 1), (64, 4), (128, 16), (1000, 1),
                                 (64, 4, 128), (7, 3, 32), (16, 2, 1)])
def test_batch_bit_exact_every_split(ctx, runs, cfg):
    import torch
    ws_, devs, refs = runs
    items = make_items(ctx, devs)
    ws = ctx.batch_workspace(items, cfg)
    plan = ctx.batch_plan(items, ws, cfg)
    plan.run()
    torch.cuda.synchronize()
    check_items(items, refs)
    plan.release()


def test_batch_without_confusion(ctx, runs):
    import torch
    ws_, devs, refs = runs
    items = make_items(ctx, devs, confusion=False)
    ws = ctx.batch_workspace(items)
    plan = ctx.batch_plan(items, ws)
    plan.run()
    torch.cuda.synchronize()
    check_items(items, refs, confusion=False)
    plan.release()


def test_batch_matches_plain_path(ctx, runs):
    import torch
    ws_, devs, refs = runs
    items = make_items(ctx, devs)
    ws = ctx.batch_workspace(items)
    plan = ctx.batch_plan(items, ws)
    plan.run()
    plain = [ctx.eval_population(ds, p) for ds, p in devs]
    torch.cuda.synchronize()
    for (ds, p, c, m), (pc, pm) in zip(items, plain):
        assert torch.equal(c, pc) and torch.equal(m, pm)
    plan.release()


def test_graph_replays_with_eager_work_between(ctx, runs):
    """The captured graph is replayed several times; between replays the
    outputs are overwritten by eager work and the host synchronizes.  Every
    replay must reproduce the oracle's counts (the graph holds no memset node:
    outputs and the work counter are cleared by a kernel)."""
    import torch
    ws_, devs, refs = runs
    items = make_items(ctx, devs)
    ws = ctx.batch_workspace(items)
    plan = ctx.batch_plan(items, ws, graph=True)
    for rep in range(4):
        for _, _, c, m in items:
            c.fill_(-7 - rep)
            m.fill_(123)
        scratch = torch.randn(1 << 16, device=ctx.device).sum()
        torch.cuda.synchronize()
        plan.run()
        torch.cuda.synchronize()
        check_items(items, refs)
        assert torch.isfinite(scratch)
    plan.release()


def test_graph_on_side_stream(ctx, runs):
    import torch
    ws_, devs, refs = runs
    items = make_items(ctx, devs)
    ws = ctx.batch_workspace(items)
    s = torch.cuda.Stream(device=ctx.device)
    plan = ctx.batch_plan(items, ws, graph=True, stream=s)
    with torch.cuda.stream(s):
        plan.run(stream=s)
        plan.run(stream=s)
    s.synchronize()
    check_items(items, refs)
    plan.release()


def test_shared_dataset_and_population(ctx, runs):
    """Several items may name the same dataset or the same population."""
    import torch
    ws_, devs, refs = runs
    pairs = [devs[0], devs[0], devs[1], devs[0]]
    want = [refs[0], refs[0], refs[1], refs[0]]
    items = make_items(ctx, pairs)
    ws = ctx.batch_workspace(items)
    plan = ctx.batch_plan(items, ws, graph=True)
    plan.run()
    torch.cuda.synchronize()
    check_items(items, want)
    plan.release()


def test_empty_population_and_single_sample(ctx):
    import torch
    w1 = synth.tiny(40, n=1, nf=16, n_classes=2, n_sets=5)
    w2 = synth.tiny(41, n=700, nf=20, n_classes=3, n_sets=9)
    empty = from_rule_lists([])
    ds1 = ctx.upload_dataset(w1.data)
    ds2 = ctx.upload_dataset(w2.data)
    p1 = ctx.pack_population(w1.pop, 16, 2)
    p2 = ctx.pack_population(w2.pop, 20, 3)
    pe = ctx.pack_population(empty, 20, 3)
    items = make_items(ctx, [(ds1, p1), (ds2, pe), (ds2, p2)])
    ws = ctx.batch_workspace(items)
    plan = ctx.batch_plan(items, ws, graph=True)
    plan.run()
    torch.cuda.synchronize()
    refs = [oracle.hard_eval(w1.data.x, w1.data.y, 2, w1.pop), None,
            oracle.hard_eval(w2.data.x, w2.data.y, 3, w2.pop)]
    check_items([items[0], items[2]], [refs[0], refs[2]])
    assert items[1][2].numel() == 0
    plan.release()
    for p in (p1, p2, pe):
        ctx.release_population(p)
    for d in (ds1, ds2):
        ctx.release_dataset(d)


@pytest.mark.parametrize("cfg", [None, (7, 3)])
def test_mixed_widths_at_the_limits(ctx, cfg):
    """One batch holding a 512-feature table with rule sets of 1023 records
    (rules of 255 conditions), the paper's 569 x 30 shape and a 129-feature
    table: the launch sizes its LDS for the widest item; every item against
    the oracle, replayed from a graph."""
    import torch
    rng = np.random.default_rng(5125)
    wide = limits.widest_table(rng, n=1500)
    wide_pop = limits.longest_sets_population(rng, wide, n_extra=6, seed=5126)
    c1 = synth.small_hard(0)
    mid = synth.tiny(5127, n=900, nf=129, n_classes=4, n_sets=20, rules=(0, 16), conds=(0, 6))
    cases = [(wide, wide_pop), (c1.data, c1.pop), (mid.data, mid.pop)]
    devs = []
    for d, pop in cases:
        devs.append((ctx.upload_dataset(d), ctx.pack_population(pop, d.n_features, d.n_classes)))
    items = make_items(ctx, devs)
    ws = ctx.batch_workspace(items, cfg)
    plan = ctx.batch_plan(items, ws, cfg, graph=True)
    refs = [oracle.hard_eval(d.x, d.y, d.n_classes, pop) for d, pop in cases]
    for _ in range(2):
        plan.run()
        torch.cuda.synchronize()
        check_items(items, refs)
    plan.release()
    for ds, p in devs:
        ctx.release_population(p)
        ctx.release_dataset(ds)


def test_empty_batch(ctx):
    import torch
    ws = ctx.batch_workspace([])
    plan = ctx.batch_plan([], ws, graph=True)
    plan.run()
    torch.cuda.synchronize()
    plan.release()


def test_autotune_picks_a_candidate_and_plans_use_it(ctx, runs):
    import torch
    ws_, devs, refs = runs
    items = make_items(ctx, devs)
    ws = ctx.batch_workspace(items, (1, 1))
    (q, tg, kib), ms = ctx.autotune(items, ws)
    assert q in (64, 128, 256, 512, 1024, 2048) and tg in (1, 2, 4, 8) and kib in (64, 128)
    assert ms > 0
    check_items(items, refs)  # autotune leaves valid outputs behind
    for _, _, c, m in items:
        c.zero_()
    plan = ctx.batch_plan(items, ws)
    plan.run()
    torch.cuda.synchronize()
    check_items(items, refs)
    plan.release()


def test_batch_errors(ctx, runs):
    import torch
    from paper_2406_01821_amd.aerl import (AerlError, AERL_ENOENT, AERL_ENOMEM, AERL_EINVAL,
                                           DeviceDataset)
    ws_, devs, refs = runs
    items = make_items(ctx, devs[:2])
    ws = ctx.batch_workspace(items)
    small = torch.empty(256, dtype=torch.uint8, device=ctx.device)
    with pytest.raises(AerlError) as e:
        ctx.batch_plan(items, small)
    assert e.value.status == AERL_ENOMEM
    bad = [(DeviceDataset(987654, None, 1, 1, 1),) + items[0][1:]]
    with pytest.raises(AerlError) as e:
        ctx.batch_plan(bad, ws)
    assert e.value.status == AERL_ENOENT
    swapped = [(items[1][0], items[0][1], items[0][2], items[0][3])]
    if (devs[0][0].n_features, devs[0][0].n_classes) != (devs[1][0].n_features,
                                                         devs[1][0].n_classes):
        with pytest.raises(AerlError) as e:
            ctx.batch_plan(swapped, ws)
        assert e.value.status == AERL_EINVAL
    nulls = [(items[0][0], items[0][1], None, None)]
    with pytest.raises(AerlError) as e:
        ctx.batch_plan(nulls, ws)
    assert e.value.status == AERL_EINVAL


def test_released_population_is_refused_at_run(ctx):
    from paper_2406_01821_amd.aerl import AerlError, AERL_ENOENT
    w = synth.tiny(42, n=300, nf=16, n_classes=2, n_sets=4)
    ds = ctx.upload_dataset(w.data)
    p = ctx.pack_population(w.pop, 16, 2)
    items = make_items(ctx, [(ds, p)])
    ws = ctx.batch_workspace(items)
    plan = ctx.batch_plan(items, ws, graph=True)
    ctx.release_population(p)
    with pytest.raises(AerlError) as e:
        plan.run()
    assert e.value.status == AERL_ENOENT
    plan.release()
    ctx.release_dataset(ds)


def test_ragged_64_runs_full_size(ctx):
    """The full 64-run ragged workload (1k-200k samples, 16-128 features,
    16-1024 rule sets of 1-64 rules x 1-8 conditions) in one graph-captured
    persistent launch: bit-exact against the per-run plain path on every
    count, and against the oracle on three sampled rule sets of every run."""
    import torch
    ws_ = synth.ragged_runs()
    devs = []
    for w in ws_:
        devs.append((ctx.upload_dataset(w.data),
                     ctx.pack_population(w.pop, w.data.n_features, w.data.n_classes)))
    items = make_items(ctx, devs)
    ws = ctx.batch_workspace(items)
    plan = ctx.batch_plan(items, ws, graph=True)
    plan.run()
    plain = [ctx.eval_population(ds, p) for ds, p in devs]
    torch.cuda.synchronize()
    for k, ((ds, p, c, m), (pc, pm), w) in enumerate(zip(items, plain, ws_)):
        assert torch.equal(c, pc) and torch.equal(m, pm), f"run {k}"
        P = w.pop.n_sets
        sample = sorted({0, P // 2, P - 1})
        rc, rm = oracle.hard_eval(w.data.x, w.data.y, w.data.n_classes, w.pop.subset(sample))
        np.testing.assert_array_equal(c.cpu().numpy()[sample], rc, err_msg=f"run {k}")
        np.testing.assert_array_equal(m.cpu().numpy()[sample], rm, err_msg=f"run {k}")
    plan.release()
    for ds, p in devs:
        ctx.release_population(p)
        ctx.release_dataset(ds)
