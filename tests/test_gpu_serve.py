"""GPU tests of the serving loop: requests submitted while others are on the
device are batched into shared launches, admitted by the arena budget, and
every result equals the same request evaluated alone (plain entry points)
and the oracle, bit for bit (Section 3 semantics; Section 5: CPU and GPU
results are equivalent)."""
import threading

import numpy as np
import pytest

import oracle
from paper_2406_01821_amd import synth
from paper_2406_01821_amd.population import Dataset, from_rule_lists

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2406_01821_amd.aerl import Context
    c = Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.fixture(scope="module")
def resident(ctx):
    """Two resident datasets: the 569 x 30 two-class table and a mid-sized
    65,536 x 64 four-class one (the scaled generator at 1/16 of its rows)."""
    small = synth.small_hard(0).data
    rng = np.random.default_rng(77)
    x = synth.lognormal_features(rng, 65536, 64)
    y = synth.planted_labels(x, 4, 12, (1, 4), 0.03, 77)
    big = Dataset(x, y, 4, "mid-65536x64")
    ds_small = ctx.upload_dataset(small)
    ds_big = ctx.upload_dataset(big)
    yield (small, ds_small), (big, ds_big)
    ctx.release_dataset(ds_small)
    ctx.release_dataset(ds_big)


def make_requests(small, big, n, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        if rng.random() < 0.5:
            which = 1 if rng.random() < 0.3 else 0
            d = big if which else small
            P = int(round(np.exp(rng.uniform(np.log(1), np.log(300)))))
            pop = synth.random_population(rng, d.x[:4096], P, (1, 32), (1, 6), d.n_classes, 0.3)
            reqs.append(("fitness", which, pop, None))
        else:
            m = int(round(np.exp(rng.uniform(np.log(1), np.log(4096)))))
            start = int(rng.integers(0, big.n - m))
            pop = synth.random_population(rng, big.x[:4096], 2, (1, 32), (1, 6), big.n_classes, 0.3)
            reqs.append(("predict", 1, pop, big.x[start:start + m]))
    return reqs


def submit(ctx, dss, r):
    kind, which, pop, rows = r
    if kind == "fitness":
        return ctx.serve_submit_fitness(dss[which], pop)
    return ctx.serve_submit_predict(pop, rows, 64, 4, set_index=1)


def check_result(ctx, datas, dss, r, out, alone=True):
    import torch
    kind, which, pop, rows = r
    if kind == "fitness":
        d = datas[which]
        rc, rm = oracle.hard_eval(d.x, d.y, d.n_classes, pop)
        np.testing.assert_array_equal(out["correct"], rc)
        np.testing.assert_array_equal(out["confusion"], rm)
        if alone:
            p = ctx.pack_population(pop, d.n_features, d.n_classes)
            c, m = ctx.eval_population(dss[which], p)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(out["correct"], c.cpu().numpy())
            np.testing.assert_array_equal(out["confusion"], m.cpu().numpy())
            ctx.release_population(p)
    else:
        np.testing.assert_array_equal(out["pred"], oracle.predict(rows, pop, 1))
        if alone:
            p = ctx.pack_population(pop, 64, 4)
            got = ctx.predict(p, rows, 1)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(out["pred"], got.cpu().numpy())
            ctx.release_population(p)


def test_mix_from_two_threads_equals_alone_and_oracle(ctx, resident):
    (small, ds_small), (big, ds_big) = resident
    datas, dss = (small, big), (ds_small, ds_big)
    reqs = make_requests(small, big, 80, 5)
    ctx.serve_start(256 << 20)
    tickets = [None] * len(reqs)

    def worker(k):
        for i in range(k, len(reqs), 2):
            tickets[i] = submit(ctx, dss, reqs[i])

    th = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    outs = [t.wait() for t in tickets]
    stats = ctx.serve_stats()
    ctx.serve_stop()
    assert stats["completed"] == len(reqs) == stats["submitted"]
    assert stats["mean_batch"] > 1.0, stats  # requests shared launches
    assert 0 < stats["p50_us"] <= stats["p99_us"] <= stats["max_us"]
    assert stats["arena_peak"] <= 256 << 20
    for r, o, t in zip(reqs, outs, tickets):
        assert t.result["status"] == 0 and t.result["batch_size"] >= 1
        check_result(ctx, datas, dss, r, o)


def test_small_arena_admits_in_turn(ctx, resident):
    """An arena that holds only a few requests at once: requests wait for
    space, all complete, and peak use stays inside the arena."""
    (small, ds_small), (big, ds_big) = resident
    datas, dss = (small, big), (ds_small, ds_big)
    reqs = make_requests(small, big, 24, 6)
    arena = 2 << 20
    ctx.serve_start(arena, max_batch=4, max_inflight=2)
    tickets = [submit(ctx, dss, r) for r in reqs]
    outs = [t.wait() for t in tickets]
    stats = ctx.serve_stats()
    ctx.serve_stop()
    assert stats["arena_peak"] <= arena
    assert stats["launches"] >= len(reqs) / 4
    for r, o in zip(reqs, outs):
        check_result(ctx, datas, dss, r, o, alone=False)


def test_predict_edges_and_wide_rows(ctx):
    """Zero rows, one row, a ragged tile tail, and 200 features (one sample
    per lane)."""
    from paper_2406_01821_amd.aerl import AERL_OK
    rng = np.random.default_rng(9)
    x = synth.lognormal_features(rng, 2000, 200)
    pop = synth.random_population(rng, x, 3, (1, 20), (1, 6), 3, 0.3)
    ctx.serve_start(64 << 20)
    cases = [0, 1, 257, 2000]
    ts = [ctx.serve_submit_predict(pop, x[:m], 200, 3, set_index=2) for m in cases]
    outs = [t.wait() for t in ts]
    ctx.serve_stop()
    for m, o, t in zip(cases, outs, ts):
        assert t.result["status"] == AERL_OK
        np.testing.assert_array_equal(o["pred"], oracle.predict(x[:m], pop, 2))


def test_empty_population_and_default_only(ctx, resident):
    (small, ds_small), _ = resident
    empty = from_rule_lists([])
    default_only = from_rule_lists([(1, [])])
    ctx.serve_start(16 << 20)
    t1 = ctx.serve_submit_fitness(ds_small, empty)
    t2 = ctx.serve_submit_fitness(ds_small, default_only)
    o1, o2 = t1.wait(), t2.wait()
    ctx.serve_stop()
    assert o1["correct"].size == 0
    assert o2["correct"][0] == int((small.y == 1).sum())


def test_serving_errors(ctx, resident):
    from paper_2406_01821_amd.aerl import (AerlError, AERL_ENOENT, AERL_EINVAL, AERL_ENOMEM,
                                           AERL_ESTATE, DeviceDataset)
    (small, ds_small), (big, ds_big) = resident
    pop = synth.random_population(np.random.default_rng(3), small.x, 4, (1, 4), (1, 3), 2, 0.3)
    with pytest.raises(AerlError) as e:
        ctx.serve_submit_fitness(ds_small, pop)
    assert e.value.status == AERL_ESTATE
    with pytest.raises(AerlError) as e:
        ctx.serve_stop()
    assert e.value.status == AERL_ESTATE
    ctx.serve_start(1 << 20)
    try:
        with pytest.raises(AerlError) as e:
            ctx.serve_start(1 << 20)
        assert e.value.status == AERL_ESTATE
        with pytest.raises(AerlError) as e:
            ctx.serve_submit_fitness(DeviceDataset(424242, None, 1, 30, 2), pop)
        assert e.value.status == AERL_ENOENT
        pop4 = synth.random_population(np.random.default_rng(5), big.x[:4096], 8, (1, 8), (1, 4),
                                       4, 0.3)
        with pytest.raises(AerlError) as e:
            ctx.serve_submit_fitness(ds_small, pop4)  # features >= 30, classes >= 2
        assert e.value.status == AERL_EINVAL
        with pytest.raises(AerlError) as e:
            ctx.serve_submit_predict(pop, small.x[:5], 30, 2, set_index=4)
        assert e.value.status == AERL_EINVAL
        huge = synth.random_population(np.random.default_rng(4), big.x[:4096], 2048, (1, 32),
                                       (1, 6), 4, 0.3)
        with pytest.raises(AerlError) as e:
            ctx.serve_submit_fitness(ds_big, huge)  # needs more than the 1 MiB arena
        assert e.value.status == AERL_ENOMEM
        t = ctx.serve_submit_fitness(ds_small, pop)
        t.wait()
        from paper_2406_01821_amd.aerl import aerl_serve_wait
        assert aerl_serve_wait(ctx.h, t.ticket, 0, None) == AERL_ENOENT  # already collected
    finally:
        ctx.serve_stop()


def test_dataset_in_use_cannot_be_released(ctx, resident):
    from paper_2406_01821_amd.aerl import AERL_ESTATE, aerl_release_dataset
    _, (big, _) = resident
    ds = ctx.upload_dataset(big)
    rng = np.random.default_rng(8)
    pops = [synth.random_population(rng, big.x[:4096], 512, (1, 32), (1, 6), 4, 0.3)
            for _ in range(6)]
    ctx.serve_start(128 << 20, max_inflight=1)
    ts = [ctx.serve_submit_fitness(ds, p) for p in pops]
    st = aerl_release_dataset(ctx.h, ds.id)
    for t in ts:
        t.wait()
    ctx.serve_stop()
    if st != 0:
        assert st == AERL_ESTATE
        ctx.release_dataset(ds)  # nothing in flight any more
    else:
        pytest.skip("requests finished before the release attempt")


def test_trace_span_log(ctx, resident, tmp_path, monkeypatch):
    """AERL_TRACE names a file at start: one JSON line per completed request
    with its host spans (pack, queue, launch, copy-out) and its launch's
    device spans (upload, kernels, download), consistent with one another
    and with the request's own result; without it nothing is written."""
    import json
    (small, ds_small), (big, ds_big) = resident
    datas, dss = (small, big), (ds_small, ds_big)
    reqs = make_requests(small, big, 30, 9)
    path = tmp_path / "spans.jsonl"
    monkeypatch.setenv("AERL_TRACE", str(path))
    ctx.serve_start(64 << 20, max_inflight=2)
    tickets = [submit(ctx, dss, r) for r in reqs]
    outs = [t.wait() for t in tickets]
    ctx.serve_stop()
    lines = [json.loads(s) for s in path.read_text().splitlines()]
    assert len(lines) == len(reqs)
    by_ticket = {d["ticket"]: d for d in lines}
    assert sorted(by_ticket) == sorted(t.ticket for t in tickets)
    for r, t, o in zip(reqs, tickets, outs):
        d = by_ticket[t.ticket]
        assert d["kind"] == r[0] and d["status"] == 0 and d["slot"] in (0, 1)
        assert d["batch"] == t.result["batch_size"] >= 1
        for k in ("pack_us", "queue_us", "launch_us", "copy_out_us", "h2d_us", "kernels_us",
                  "d2h_us"):
            assert d[k] >= 0.0, (k, d)
        parts = d["pack_us"] + d["queue_us"] + d["launch_us"] + d["copy_out_us"]
        assert abs(parts - d["total_us"]) <= 1.0 + 1e-3 * d["total_us"], d
        assert abs(d["total_us"] - t.result["latency_us"]) <= 1.0 + 1e-3 * d["total_us"], d
        # the launch's device work ends before the scheduler sees it done
        assert d["h2d_us"] + d["kernels_us"] + d["d2h_us"] <= d["launch_us"] + 50.0, d
        check_result(ctx, datas, dss, r, o, alone=False)
    monkeypatch.delenv("AERL_TRACE")
    size = path.stat().st_size
    ctx.serve_start(16 << 20)
    submit(ctx, dss, reqs[0]).wait()
    ctx.serve_stop()
    assert path.stat().st_size == size
