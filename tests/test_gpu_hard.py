"""GPU parity of the hard path: dataset layout, fitness counts, confusion and
predictions are bit-exact against the CPU oracle (Section 3 / Fig. 1
semantics; Section 5: CPU and GPU results are equivalent)."""
import numpy as np
import pytest

import limits
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


def run_hard(ctx, data, pop, cfg=None, confusion=True):
    import torch
    ds = ctx.upload_dataset(data)
    p = ctx.pack_population(pop, data.n_features, data.n_classes)
    correct, conf = ctx.eval_population(ds, p, confusion=confusion, cfg=cfg)
    torch.cuda.synchronize()
    return correct.cpu().numpy(), (conf.cpu().numpy() if conf is not None else None)


def check_against_oracle(ctx, data, pop, cfg=None):
    c, m = run_hard(ctx, data, pop, cfg)
    rc, rm = oracle.hard_eval(data.x, data.y, data.n_classes, pop)
    np.testing.assert_array_equal(c, rc)
    np.testing.assert_array_equal(m, rm)


def test_upload_layout_groups_labels_and_computes_tau(ctx):
    import torch
    w = synth.tiny(1, n=1000, nf=7, n_classes=3)
    ds = ctx.upload_dataset(w.data)
    info = ctx.dataset_info(ds)
    torch.cuda.synchronize()
    y_pad = info["y_pad"].cpu().numpy()
    perm = info["perm"].cpu().numpy()
    x_fm = info["x_fm"].cpu().numpy()
    counts = np.bincount(w.data.y, minlength=3)
    assert info["class_count"] == list(counts)
    valid = perm >= 0
    assert valid.sum() == w.data.n
    assert np.array_equal(np.sort(perm[valid]), np.arange(w.data.n))
    assert np.array_equal(y_pad[valid], w.data.y[perm[valid]])
    assert np.all(y_pad[~valid] == -1)
    # stable grouping: within each class the original order is kept
    for c in range(3):
        idx = perm[y_pad == c]
        assert np.all(np.diff(idx) > 0)
    assert np.array_equal(x_fm[:, valid].T, w.data.x[perm[valid]])
    assert info["n_pad"] % 256 == 0
    tau = info["tau"].cpu().numpy()
    ref = oracle.tau(w.data.x)
    ulps = np.abs(tau.view(np.int32) - ref.view(np.int32))
    assert ulps.max() <= 1


@pytest.mark.parametrize("n", [5, 300_001])
def test_tau_over_many_slices_is_exact_and_repeatable(ctx, n):
    """tau over a row split into many slices (and over fewer tiles than
    slices): within 1 ulp of the fp64 oracle, 1 for a constant column, and
    the same bits on a second upload."""
    import torch
    rng = np.random.default_rng(n)
    x = synth.lognormal_features(rng, n, 6)
    x[:, 2] = 3.5
    x[:, 4] *= 1e4
    data = Dataset(x, rng.integers(0, 4, size=n).astype(np.int32), 4, "tau")
    taus = []
    for _ in range(2):
        ds = ctx.upload_dataset(data)
        info = ctx.dataset_info(ds)
        torch.cuda.synchronize()
        taus.append(info["tau"].cpu().numpy().copy())
        ctx.release_dataset(ds)
    ref = oracle.tau(x)
    assert np.array_equal(taus[0], taus[1])
    assert np.abs(taus[0].view(np.int32) - ref.view(np.int32)).max() <= 1
    assert taus[0][2] == 1.0


def test_small_workload_bit_exact(ctx):
    w = synth.small_hard(0)
    check_against_oracle(ctx, w.data, w.pop)


@pytest.mark.parametrize("cfg", [(1, 1, 1), (2, 3, 1), (4, 7, 2), (4, 100, 5), (1, 64, 3), (2, 256, 1)])
def test_every_launch_configuration_bit_exact(ctx, cfg):
    w = synth.tiny(12, n=3000, nf=13, n_classes=3, n_sets=150, rules=(0, 9), conds=(0, 5))
    check_against_oracle(ctx, w.data, w.pop, cfg)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 255, 256, 257, 511, 1000, 4097])
def test_ragged_sample_counts(ctx, n):
    w = synth.tiny(100 + n, n=n, nf=5, n_classes=2, n_sets=40)
    check_against_oracle(ctx, w.data, w.pop)


@pytest.mark.parametrize("nc", [1, 2, 4, 5, 64])
def test_class_counts(ctx, nc):
    w = synth.tiny(7 + nc, n=2000, nf=6, n_classes=nc, n_sets=30)
    check_against_oracle(ctx, w.data, w.pop)


def test_missing_classes_and_single_class(ctx):
    w = synth.tiny(9, n=700, nf=4, n_classes=4, n_sets=25)
    y = np.where(w.data.y == 2, 0, w.data.y).astype(np.int32)  # class 2 absent
    check_against_oracle(ctx, Dataset(w.data.x, y, 4), w.pop)
    check_against_oracle(ctx, Dataset(w.data.x, np.zeros_like(y), 4), w.pop)


def test_edge_values_subnormals_infinities_ties(ctx):
    rng = np.random.default_rng(5)
    n = 900
    x = rng.uniform(-2, 2, size=(n, 4)).astype(np.float32)
    x[:100, 0] = np.ldexp(rng.uniform(-1, 1, 100), -130).astype(np.float32)  # subnormal
    x[100:150, 0] = 0.0
    x[150:200, 0] = -0.0
    x[200:260, 1] = np.float32(3e38)
    x[260:300, 1] = np.float32(-3e38)
    x[300:400, 2] = np.float32(0.75)
    y = rng.integers(0, 2, n).astype(np.int32)
    conds = []
    for op in range(4):
        for t in (0.75, 0.0, -0.0, np.inf, -np.inf, 1e-40, -1e-40, 1e-45, 3.4e38):
            for c in (1.0, -1.0, 0.0, 1e-3, 4.0):
                for f in (0, 1, 2):
                    conds.append(dict(op=op, kind=0, f=f, coef=np.float32(c), theta=np.float32(t)))
        for c, c2 in ((1.0, 1.0), (-1.0, 1e-38), (0.0, 0.0), (2.0, -3.0), (1e-20, 1e-20)):
            conds.append(dict(op=op, kind=1, f=0, g=1, coef=np.float32(c), coef2=np.float32(c2)))
            conds.append(dict(op=op, kind=1, f=2, g=0, coef=np.float32(c), coef2=np.float32(c2)))
    pop = from_rule_lists([(0, [(1, [c])]) for c in conds])
    check_against_oracle(ctx, Dataset(x, y, 2), pop)


def test_special_records_inside_long_rules(ctx):
    """Rules of up to 6 conditions mixing every record kind at every
    position of the paired walk: folded thresholds in both directions, zero
    coefficients (product form), +-inf thresholds, feature-vs-feature, and
    empty rules anywhere in a set; fitness against the oracle, and
    prediction on rows holding +-inf and NaN."""
    import torch
    rng = np.random.default_rng(21)
    n, nf = 3000, 6
    x = rng.uniform(-2, 2, size=(n, nf)).astype(np.float32)
    x[:200, 0] = 0.0
    x[200:300, 1] = np.float32(-0.0)
    x[300:400, 2] = np.float32(1e-40)
    y = rng.integers(0, 3, n).astype(np.int32)
    pop = synth.special_values_population(22, nf, 3, 80)
    check_against_oracle(ctx, Dataset(x, y, 3), pop)
    rows = x[:500].copy()
    rows[::7, 0] = np.inf
    rows[::11, 1] = -np.inf
    rows[::13, 2] = np.nan
    p = ctx.pack_population(pop, nf, 3)
    for s in range(0, pop.n_sets, 5):
        got = ctx.predict(p, rows, s)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), oracle.predict(rows, pop, s),
                                      err_msg=f"set {s}")


@pytest.mark.parametrize("nf", [65, 129, 300])
def test_wide_datasets_default_launch(ctx, nf):
    """Feature counts that move the default launch to two and one samples
    per lane (and, at 300, one block per CU)."""
    w = synth.tiny(70 + nf, n=2500, nf=nf, n_classes=3, n_sets=64, rules=(0, 9), conds=(0, 6))
    check_against_oracle(ctx, w.data, w.pop)


def test_limits_widest_table_and_longest_rule_set(ctx):
    """The documented maxima together: 512 features (one sample per lane, a
    128 KiB tile per block), rules of 255 conditions and rule sets of 1023
    records, whose next-rule offsets fill their field; the conditions pass
    about 99% of the samples each, so the walks run through every record
    kind deep into the long rules.  Fitness against the oracle, under the
    default launch and a forced one, and predictions of the longest sets."""
    import torch
    rng = np.random.default_rng(512)
    data = limits.widest_table(rng)
    pop = limits.longest_sets_population(rng, data)
    for cfg in (None, (1, 5, 3)):
        check_against_oracle(ctx, data, pop, cfg)
    p = ctx.pack_population(pop, data.n_features, data.n_classes)
    rows = data.x[:700]
    for s in range(3):
        got = ctx.predict(p, rows, s)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), oracle.predict(rows, pop, s),
                                      err_msg=f"set {s}")


def test_empty_population_rules_and_sets(ctx):
    w = synth.tiny(3, n=500, nf=5)
    pop = from_rule_lists([(1, []), (0, [(1, [])]), (1, [(0, []), (1, [])])] +
                          [w.pop.to_rule_list(s) for s in range(5)])
    check_against_oracle(ctx, w.data, pop)


def test_permutation_invariance_on_device(ctx):
    w = synth.tiny(15, n=3000, nf=6, n_sets=60)
    c0, m0 = run_hard(ctx, w.data, w.pop)
    perm = np.random.default_rng(1).permutation(w.data.n)
    c1, m1 = run_hard(ctx, Dataset(w.data.x[perm], w.data.y[perm], 2), w.pop)
    assert np.array_equal(c0, c1) and np.array_equal(m0, m1)


def test_repeated_calls_are_identical_and_outputs_overwritten(ctx):
    import torch
    w = synth.tiny(16, n=5000, nf=9, n_sets=120)
    ds = ctx.upload_dataset(w.data)
    p = ctx.pack_population(w.pop, 9, 2)
    out = ctx.eval_population(ds, p)
    first = [t.clone() for t in out]
    for _ in range(3):
        ctx.eval_population(ds, p, out=out)
    torch.cuda.synchronize()
    assert torch.equal(first[0], out[0]) and torch.equal(first[1], out[1])


def test_scaled_workload_slice_bit_exact(ctx):
    w = synth.scaled_hard(1, n=1 << 16, nf=64, n_sets=256)
    check_against_oracle(ctx, w.data, w.pop)


def test_scaled_workload_full_size_every_set(ctx):
    """2^20 x 64, 4096 rule sets, in the benchmark's launch configuration;
    the oracle recomputes every rule set (a few seconds on the host's
    cores)."""
    w = synth.scaled_hard(1)
    c, m = run_hard(ctx, w.data, w.pop)
    rc, rm = oracle.hard_eval(w.data.x, w.data.y, 4, w.pop)
    np.testing.assert_array_equal(c, rc)
    np.testing.assert_array_equal(m, rm)
    assert np.all(m.sum(axis=(1, 2)) == w.data.n)
    assert np.array_equal(np.trace(m, axis1=1, axis2=2), c)


@pytest.mark.parametrize("nc", [2, 3, 4])
def test_per_tile_counts_every_class_count(ctx, nc):
    """Launches of at least 4 Mi (tile, rule set) pairs (here about 1,200
    tiles x 4,096 rule sets) store the blocks' 10-bit counter words per tile
    and a second kernel sums them: two to four classes (one to three counted
    fields per set, so sets share words or straddle two), a ragged last tile
    per class, every rule set against the oracle; the same counts from
    1001-set chunks (a short last chunk, chunks ending inside a word) and
    from a launch that flushes per block (two-tile groups)."""
    w = synth.tiny(300 + nc, n=300_001, nf=9, n_classes=nc, n_sets=4096, rules=(0, 10),
                   conds=(0, 4))
    assert (w.data.n + 255) // 256 * 4096 >= 4 << 20
    c, m = run_hard(ctx, w.data, w.pop)
    rc, rm = oracle.hard_eval(w.data.x, w.data.y, nc, w.pop)
    np.testing.assert_array_equal(c, rc)
    np.testing.assert_array_equal(m, rm)
    for cfg in ((4, 1001, 1), (4, 2048, 2)):
        c2, m2 = run_hard(ctx, w.data, w.pop, cfg=cfg)
        np.testing.assert_array_equal(c2, rc)
        np.testing.assert_array_equal(m2, rm)


def test_dataset_past_65535_tiles(ctx):
    """2^24 + 1000 samples x 4 features in two classes: 65,540 layout tiles,
    more than one grid dimension could index; every rule set is checked
    against the oracle."""
    w = synth.tiny(77, n=(1 << 24) + 1000, nf=4, n_classes=2, n_sets=8, rules=(1, 6),
                   conds=(1, 3))
    check_against_oracle(ctx, w.data, w.pop)


@pytest.mark.parametrize("n", [1, 63, 64, 255, 256, 257, 4096])
def test_predict_matches_oracle(ctx, n):
    import torch
    w = synth.tiny(40 + n, n=max(n, 10), nf=11, n_sets=6, rules=(1, 12), conds=(1, 5))
    rows = w.data.x[:n]
    p = ctx.pack_population(w.pop, 11, 2)
    for s in range(w.pop.n_sets):
        got = ctx.predict(p, rows, s)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), oracle.predict(rows, w.pop, s))


def test_invalid_inputs_raise(ctx):
    from paper_2406_01821_amd.aerl import AerlError
    w = synth.tiny(2, n=50, nf=3)
    bad = Dataset(w.data.x.copy(), w.data.y, 2)
    bad.x[3, 1] = np.nan
    with pytest.raises(AerlError):
        ctx.upload_dataset(bad)
    with pytest.raises(AerlError):
        ctx.upload_dataset(Dataset(w.data.x, np.full(50, 2, np.int32), 2))
    ds = ctx.upload_dataset(w.data)
    p = ctx.pack_population(w.pop, 3, 2)
    other = synth.tiny(2, n=50, nf=4)
    p4 = ctx.pack_population(other.pop, 4, 2)
    with pytest.raises(AerlError):
        ctx.eval_population(ds, p4)
    with pytest.raises(AerlError):
        ctx.predict(p, w.data.x, set_index=w.pop.n_sets)


def test_block_counters_at_their_widest(ctx):
    """A block may cover up to 255 layout tiles; its per-(set, class)
    counters then reach 255 x 256 = 65,280 (16-bit counters in LDS)."""
    import torch
    from paper_2406_01821_amd.aerl import AerlError
    n = 255 * 256
    rng = np.random.default_rng(5)
    x = synth.lognormal_features(rng, n, 4)
    data = Dataset(x, np.zeros(n, np.int32), 1)
    pop = from_rule_lists([(0, []), (0, [(0, [dict(op=2, kind=0, f=0, g=0, coef=np.float32(1),
                                                     coef2=np.float32(0), theta=np.float32(-1))])])])
    check_against_oracle(ctx, data, pop, (4, 2, 255))
    c, _ = run_hard(ctx, data, pop, (4, 2, 255))
    assert list(c) == [n, n]
    with pytest.raises(AerlError):
        run_hard(ctx, data, pop, (4, 2, 256))


def _layout_tiles(y, n_classes, tile=256):
    """Sample indices of each layout tile: samples grouped by label (stable),
    each class region cut into tiles of 256."""
    tiles = []
    for c in range(n_classes):
        idx = np.flatnonzero(y == c)
        tiles += [idx[i:i + tile] for i in range(0, len(idx), tile)]
    return tiles


@pytest.mark.parametrize("cfg", [None, (4, 64, 1), (2, 33, 2), (1, 7, 1)])
def test_tile_test_at_the_tile_extremes(ctx, cfg):
    """Rules whose first or second condition sits exactly at a tile's largest
    or smallest value (x >= max passes one sample, x > max none; x <= min
    one, x < min none; also through coefficient 0.5 and through negated
    coefficients, and signed zeros), in rule sets of up to 63 rules (tile
    test) and of 64 and more (which walk every rule), against the oracle on
    every set."""
    rng = np.random.default_rng(71)
    n, nf = 2500, 6
    x = synth.lognormal_features(rng, n, nf)
    x[:40, 2] = 0.0
    x[40:80, 2] = -0.0
    x[80:120, 3] = -x[80:120, 3]
    y = rng.integers(0, 2, n).astype(np.int32)
    data = Dataset(x, y, 2)
    ext = []
    for t in _layout_tiles(y, 2):
        ext += [(f, x[t, f].max(), x[t, f].min()) for f in range(nf)]

    def cond(op, f, theta, coef=1.0):
        return dict(op=op, kind=0, f=f, g=0, coef=np.float32(coef), coef2=np.float32(0),
                    theta=np.float32(theta))

    def boundary_cond():
        f, hi, lo = ext[rng.integers(len(ext))]
        k = rng.integers(8)
        if k == 0: return cond(3, f, hi)               # x >= max
        if k == 1: return cond(2, f, hi)               # x > max
        if k == 2: return cond(1, f, lo)               # x <= min
        if k == 3: return cond(0, f, lo)               # x < min
        if k == 4: return cond(3, f, np.float32(0.5) * hi, 0.5)
        if k == 5: return cond(1, f, -hi, -1.0)        # -x <= -max
        if k == 6: return cond(2, 2, 0.0)              # x > 0 (signed zeros)
        return cond(0, 2, -0.0)                        # x < -0

    sets = []
    # 62 and 63 rules: the tile test's largest sets (up to 64 head entries
    # with the closing record); 64 and more: every rule walked
    sizes = [62, 63, 64, 65]
    for s in range(64):
        if s < len(sizes):
            n_rules = sizes[s]
        else:
            n_rules = int(rng.integers(1, 20)) if s % 6 else int(rng.integers(66, 90))
        rules = []
        for _ in range(n_rules):
            conds = [boundary_cond()]
            if rng.random() < 0.5:
                conds.append(boundary_cond())
            for _ in range(int(rng.integers(0, 3))):
                f = int(rng.integers(nf))
                conds.append(cond(int(rng.integers(4)), f, np.float32(rng.choice(x[:, f]))))
            rules.append((int(rng.integers(2)), conds))
        sets.append((int(rng.integers(2)), rules))
    pop = from_rule_lists(sets)
    check_against_oracle(ctx, data, pop, cfg)


@pytest.mark.parametrize("seed", range(6))
def test_tile_test_random_shapes(ctx, seed):
    """Random shapes on heavy-tailed data: 8-100 features (four or two
    samples per lane by default), 2-5 classes, rule sets of 1-70 rules x 1-8
    conditions (30% feature-vs-feature), so that tile-tested sets and sets
    walked rule by rule share launches, and thresholds over each column's
    range that sit above or below many tiles' extremes; bit-exact against
    the oracle."""
    rng = np.random.default_rng(900 + seed)
    nf = int(rng.integers(8, 101))
    nc = int(rng.integers(2, 6))
    n = int(rng.integers(700, 3000))
    x = synth.lognormal_features(rng, n, nf)
    y = rng.integers(0, nc, n).astype(np.int32)
    data = Dataset(x, y, nc)
    pop = synth.random_population(rng, x, 48, (1, 70), (1, 8), nc, 0.3)
    check_against_oracle(ctx, data, pop)
