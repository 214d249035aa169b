"""Host-side tests of libaerl (no GPU): the library loads and exports every
entry point the header declares, argument validation, and the exact rewriting
of conditions done by the packer (checked against the oracle on CPU)."""
import os
import re

import numpy as np
import pytest

import oracle
from paper_2406_01821_amd import synth
from paper_2406_01821_amd.population import from_rule_lists

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def aerl():
    from paper_2406_01821_amd import aerl as mod
    return mod


def header_symbols():
    text = open(os.path.join(ROOT, "include", "aerl.h")).read()
    return sorted(set(re.findall(r"^\s*(?:aerl_status|void|int64_t|const char \*)\s*(aerl_\w+)\(", text, re.M)))


def test_library_exports_every_declared_symbol(aerl):
    names = header_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(aerl.lib, n), n
        assert n in aerl.EXPORTED, n


def test_dataset_bytes_validation(aerl):
    import ctypes as C
    out = C.c_size_t()
    assert aerl.aerl_dataset_bytes(569, 30, 2, C.byref(out)) == 0
    # features [30][(3 tiles + 2 classes) * 256] + labels, perm, tiles, tau, scratch
    assert out.value >= 30 * 5 * 256 * 4
    assert aerl.aerl_dataset_bytes(-1, 30, 2, C.byref(out)) == aerl.AERL_EINVAL
    assert aerl.aerl_dataset_bytes(10, 0, 2, C.byref(out)) == aerl.AERL_EINVAL
    assert aerl.aerl_dataset_bytes(10, 513, 2, C.byref(out)) == aerl.AERL_EINVAL
    assert aerl.aerl_dataset_bytes(10, 4, 65, C.byref(out)) == aerl.AERL_EINVAL
    assert aerl.aerl_dataset_bytes(0, 4, 2, C.byref(out)) == 0


def test_sample_limit_keeps_the_padded_layout_in_int32(aerl):
    """The label-grouped layout pads every class region to whole 256-sample
    tiles and indexes the padded samples with int32: the largest accepted n
    pads to at most 2^31 - 1 samples, one more sample is refused (host
    arithmetic only; nothing of that size is allocated)."""
    import ctypes as C
    out = C.c_size_t()
    for nc in (1, 2, 4, 64):
        m = aerl.max_samples(nc)
        assert ((m + 255) // 256 + nc) * 256 <= 2**31 - 1
        assert ((m + 1 + 255) // 256 + nc) * 256 > 2**31 - 1
        assert aerl.aerl_dataset_bytes(m, 1, nc, C.byref(out)) == 0
        assert aerl.aerl_dataset_bytes(m + 1, 1, nc, C.byref(out)) == aerl.AERL_EINVAL
    # the case where a 2^31-sample upload's last class base wrapped to INT32_MIN
    assert aerl.aerl_dataset_bytes(2**31, 1, 2, C.byref(out)) == aerl.AERL_EINVAL
    assert aerl.max_samples(0) == 0 and aerl.max_samples(65) == 0


@pytest.mark.parametrize("counts", [[569 - 212, 212], [1 << 18] * 4, [(1 << 24) + 1000, 7],
                                    [(1 << 30) - 300_000, (1 << 30) - 3], [(1 << 31) - 300_000, 1]])
def test_hard_launch_plan_fits_the_grid(aerl, counts):
    """The planner's one-dimensional grid (one 1024-thread workgroup per set
    chunk and tile group) keeps its work-item count within 32 bits for every
    dataset size up to the sample limit, and covers every tile."""
    tiles = sum((c + 255) // 256 for c in counts)
    for n_sets in (1, 100, 4096, 100_000):
        p = aerl.eval_plan(counts, 8, n_sets, 256)
        assert p["samples_per_lane"] in (1, 2, 4)
        assert 1 <= p["tiles_per_group"] <= 255
        groups = sum(-(-((c + 255) // 256) // p["tiles_per_group"]) for c in counts)
        chunks = -(-n_sets // p["sets_per_chunk"])
        assert p["workgroups"] == groups * chunks
        assert p["workgroups"] * 1024 <= 2**32 - 1
        assert groups * p["tiles_per_group"] >= tiles
        if tiles * chunks * 1024 <= 2**32 - 1:
            assert p["tiles_per_group"] == 1  # single tiles while they fit
    with pytest.raises(aerl.AerlError):
        aerl.eval_plan([aerl.max_samples(2), 300], 8, 10, 256)


def _cond(**kw):
    d = dict(op=2, kind=0, f=0, g=0, coef=np.float32(1), coef2=np.float32(0), theta=np.float32(0))
    d.update(kw)
    return d


@pytest.mark.parametrize("bad", [
    dict(op=4), dict(kind=3), dict(f=5), dict(f=-1), dict(kind=1, g=0), dict(kind=1, g=7),
    dict(coef=np.float32(np.nan)), dict(coef=np.float32(np.inf)), dict(theta=np.float32(np.nan)),
    dict(kind=1, g=1, coef2=np.float32(np.inf))])
def test_population_validation_rejects(aerl, bad):
    pop = from_rule_lists([(0, [(1, [_cond(), _cond(**bad)])])])
    assert aerl.population_status(pop, 5, 2) == aerl.AERL_EINVAL


@pytest.mark.parametrize("field,value", [
    ("op", 4), ("kind", 3), ("f", 9), ("f", -1), ("coef", np.float32(np.nan)),
    ("theta", np.float32(np.nan)), ("g", -5)])
def test_large_population_validation_finds_one_fault(aerl, field, value):
    """A population of about 150k conditions is checked in several parallel
    parts: one fault anywhere in it (first, last or in between, in a
    threshold or a feature-vs-feature condition) is still found, and the
    population without it passes."""
    rng = np.random.default_rng(31)
    x = synth.lognormal_features(rng, 200, 9)
    pop = synth.random_population(rng, x, 12000, (1, 8), (1, 4), 3, 0.3)
    assert pop.n_conds > 4 * 32768
    assert aerl.population_status(pop, 9, 3) == 0
    ff = np.nonzero(pop.kind == 1)[0]
    t = np.nonzero(pop.kind == 0)[0]
    for j in (0, pop.n_conds - 1, int(rng.integers(pop.n_conds)), int(t[len(t) // 2]),
              int(ff[len(ff) // 3])):
        if field == "theta" and pop.kind[j] != 0:
            continue  # a feature-vs-feature condition has no theta
        if field == "g" and pop.kind[j] != 1:
            continue
        arr = getattr(pop, field)
        old = arr[j]
        arr[j] = value
        try:
            assert aerl.population_status(pop, 9, 3) == aerl.AERL_EINVAL, (field, j)
        finally:
            arr[j] = old
    assert aerl.population_status(pop, 9, 3) == 0


def test_population_validation_rejects_structure(aerl):
    ok = from_rule_lists([(0, [(1, [_cond()])]), (1, [])])
    assert aerl.population_status(ok, 5, 2) == 0
    bad_cls = from_rule_lists([(0, [(2, [_cond()])])])
    assert aerl.population_status(bad_cls, 5, 2) == aerl.AERL_EINVAL
    bad_default = from_rule_lists([(3, [])])
    assert aerl.population_status(bad_default, 5, 2) == aerl.AERL_EINVAL
    big = from_rule_lists([(0, [(1, [_cond()] * 256)])])
    assert aerl.population_status(big, 5, 2) == aerl.AERL_EINVAL
    # at most 1022 records per set (conditions, +1 per empty rule) besides
    # the closing default record
    many = from_rule_lists([(0, [(1, [_cond()] * 200)] * 5 + [(0, [])] * 23)])
    assert aerl.population_status(many, 5, 2) == aerl.AERL_EINVAL
    ok_many = from_rule_lists([(0, [(1, [_cond()] * 200)] * 5 + [(0, [])] * 22)])
    assert aerl.population_status(ok_many, 5, 2) == 0
    inf_theta = from_rule_lists([(0, [(1, [_cond(theta=np.float32(np.inf))])])])
    assert aerl.population_status(inf_theta, 5, 2) == 0


def _align(v):
    return (v + 255) & ~255


def decode_packed(img, n_sets, n_rules, n_conds, heads=False):
    """Splits the packed image into set records (record count in column 1),
    the hard record stream and, with heads=True, the head table and each
    set's head count."""
    sets_off = 0
    ssets_off = _align(sets_off + 16 * max(n_sets, 1))
    rules_off = _align(ssets_off + 16 * max(n_sets, 1))
    hc_off = _align(rules_off + 16 * max(n_rules, 1))
    raw = img[sets_off:sets_off + 16 * n_sets].view(np.int32).reshape(-1, 4)
    sets = raw.copy()
    sets[:, 1] &= 0xffff
    n_rec = n_conds + n_rules + n_sets + 1
    hc = img[hc_off:hc_off + 16 * n_rec].view(np.uint32).reshape(-1, 4)
    if not heads:
        return sets, hc
    sc_off = _align(hc_off + 16 * n_rec)
    hd_off = _align(sc_off + 4 * max(n_conds, 1))
    hd = img[hd_off:hd_off + 16 * n_rec].view(np.uint32).reshape(-1, 4)
    return sets, hc, hd, raw[:, 1] >> 16


FF, GE_LE, LAST, MUL, ALWAYS, CAT = 1 << 9, 1 << 10, 1 << 11, 1 << 0, 1 << 1, 1 << 3


def record_mask(x, r):
    """Samples of x for which packed record r holds, in float32 numpy
    arithmetic: x[f] >= y, x[f] <= y, y*x[f] > z, always, y*x[f] > z*x[g] or
    y*x[f] >= z*x[g]."""
    f1024, a, b, w = r
    if not w & FF and w & CAT:  # x[f] a code k in 0..63 with bit k of {a, b} set
        v = x[:, f1024 // 1024].astype(np.float64)
        with np.errstate(invalid="ignore"):
            ok = (v >= 0) & (v <= 63) & (v == np.floor(v))
        code = np.where(ok, v, 0).astype(np.uint64)
        mask = np.uint64(a) | (np.uint64(b) << np.uint64(32))
        return ok & (((mask >> code) & np.uint64(1)) == 1)
    a = np.uint32(a).view(np.float32)
    b = np.uint32(b).view(np.float32)
    xf = x[:, f1024 // 1024]
    if w & FF:
        lhs = np.float32(a) * xf
        rhs = np.float32(b) * x[:, w & 0x1ff]
        return lhs >= rhs if w & GE_LE else lhs > rhs
    if w & ALWAYS:
        return np.ones(x.shape[0], bool)
    if w & MUL:
        return np.float32(a) * xf > b
    return xf <= a if w & GE_LE else xf >= a


def eval_packed(x, sets, hc, s):
    """Walks the packed record stream of rule set s: a rule whose records all
    hold for a sample gives that sample its class; the set's closing record
    (always true, default class) takes the samples no rule fired for."""
    n = x.shape[0]
    first, count, default, _ = sets[s]
    pred = np.full(n, -1, np.int32)
    und = np.ones(n, bool)
    fire = und.copy()
    o = 0
    last = tuple(int(v) for v in hc[first + count - 1])
    assert last[3] & (ALWAYS | LAST) == ALWAYS | LAST and (last[3] >> 12) & 63 == default
    while o < count * 16:
        r = tuple(int(v) for v in hc[first + o // 16])
        w = r[3]
        fire &= record_mask(x, r)
        nxt = o + 16
        if w & LAST:
            assert nxt == w >> 18
        if not fire.any():
            nxt = w >> 18
            fire = und.copy()
        elif w & LAST:
            pred[fire] = (w >> 12) & 63
            und &= ~fire
            fire = und.copy()
        o = nxt
    assert not und.any()
    return pred


def test_packed_rewrite_is_exact_against_oracle(aerl):
    np.seterr(over="ignore")
    rng = np.random.default_rng(3)
    x = rng.uniform(-3, 3, size=(400, 4)).astype(np.float32)
    x[:20, 0] = 0.0
    x[20:40, 0] = -0.0
    x[40:60, 1] = np.float32(1.5)
    x[60:70, 2] = np.float32(3e38)
    x[70:75, 3] = np.inf
    x[75:80, 3] = -np.inf
    x[80:85, 3] = np.nan
    x[85:90, 1] = np.float32(1e-45)
    x[90:95, 1] = np.float32(-3.4e38)
    conds = []
    for op in range(4):
        for t in (1.5, 0.0, -0.0, np.inf, -np.inf, 1e-45, -1e-45, 3.4e38, -2.25):
            for c in (1.0, -1.0, 0.0, -0.0, 0.5, 2.0, 1e-45, -3e38):
                conds.append(_cond(op=op, f=int(rng.integers(4)), coef=np.float32(c), theta=np.float32(t)))
        for c, c2 in ((1.0, 1.0), (-1.0, 0.5), (0.0, 0.0), (2.0, -3.0)):
            conds.append(_cond(op=op, kind=1, f=1, g=2, coef=np.float32(c), coef2=np.float32(c2)))
    sets = [(0, [(1, [c])]) for c in conds]
    w = synth.tiny(4, n=300, nf=4, n_sets=40, rules=(1, 6), conds=(1, 4))
    sets += [w.pop.to_rule_list(s) for s in range(w.pop.n_sets)]
    pop = from_rule_lists(sets)
    img = aerl.pack_host(pop, 4, 2)
    S, H = decode_packed(img, pop.n_sets, pop.n_rules, pop.n_conds)
    xx = np.concatenate([x, w.data.x[:, :4]])
    for s in range(pop.n_sets):
        np.testing.assert_array_equal(eval_packed(xx, S, H, s), oracle.predict(xx, pop, s),
                                      err_msg=str(s))


def test_categorical_records_are_exact_against_oracle(aerl):
    """Categorical conditions pack into records whose code-set test, walked
    on the host, matches the oracle on every special value of a code
    column (and the soft condition words flag them with their masks)."""
    rng = np.random.default_rng(9)
    special = np.array([0.0, -0.0, 1.0, 2.5, -1.0, 31.0, 32.0, 63.0, 64.0, 1e9, np.inf, -np.inf,
                        np.nan, 5.0], np.float32)
    x = np.concatenate([rng.uniform(-3, 3, size=(300, 3)).astype(np.float32),
                        rng.choice(special, size=(300, 2)).astype(np.float32)], axis=1)
    pop = synth.categorical_population(rng, x, 2, 64, 60, (1, 6), (1, 4), 3, cat_frac=0.5)
    extra = [(0, [(1, [dict(kind=2, f=3, mask=m)])]) for m in
             (0, 1, 1 << 31, 1 << 32, 1 << 63, (1 << 64) - 1, 0x5555_5555_5555_5555)]
    pop = from_rule_lists([pop.to_rule_list(s) for s in range(pop.n_sets)] + extra)
    assert (pop.kind == 2).sum() > 50
    img = aerl.pack_host(pop, 5, 3)
    S, H = decode_packed(img, pop.n_sets, pop.n_rules, pop.n_conds)
    for s in range(pop.n_sets):
        np.testing.assert_array_equal(eval_packed(x, S, H, s), oracle.predict(x, pop, s),
                                      err_msg=str(s))


@pytest.mark.parametrize("seed", range(3))
def test_threshold_folding_is_exact_at_the_boundary(aerl, seed):
    """Folded thresholds (x >= t or x <= t) against the oracle's fp32
    product compare on the floats around every boundary: for random
    coefficients and thresholds over many binades and both signs, the
    samples are t/c and its 8 nearest floats on each side, plus +-0, +-inf
    and NaN, for all four operators."""
    np.seterr(all="ignore")
    rng = np.random.default_rng(100 + seed)
    n_cond = 120
    c = (rng.choice([-1.0, 1.0], n_cond) * 10.0 ** rng.uniform(-30, 30, n_cond)).astype(np.float32)
    t = (rng.choice([-1.0, 1.0], n_cond) * 10.0 ** rng.uniform(-30, 30, n_cond)).astype(np.float32)
    c[:4] = np.float32([1e-45, -1e-45, 3e38, -3e38])
    t[4:8] = np.float32([0.0, -0.0, 3.4e38, -3.4e38])
    cols = []
    for j in range(n_cond):
        q = np.float32(np.float64(t[j]) / np.float64(c[j]))
        near = [q]
        up = down = q
        for _ in range(8):
            up = np.nextafter(up, np.float32(np.inf))
            down = np.nextafter(down, np.float32(-np.inf))
            near += [up, down]
        cols.append(near)
    col = np.concatenate([np.array(v, np.float32) for v in cols] +
                         [np.float32([0.0, -0.0, np.inf, -np.inf, np.nan, 1e-45, -1e-45])])
    x = col[:, None].astype(np.float32)
    conds = [_cond(op=op, f=0, coef=c[j], theta=t[j]) for j in range(n_cond) for op in range(4)]
    pop = from_rule_lists([(0, [(1, [cd])]) for cd in conds])
    img = aerl.pack_host(pop, 1, 2)
    S, H = decode_packed(img, pop.n_sets, pop.n_rules, pop.n_conds)
    for s in range(pop.n_sets):
        np.testing.assert_array_equal(eval_packed(x, S, H, s), oracle.predict(x, pop, s),
                                      err_msg=f"set {s}: {conds[s]}")


DIRCHG = 1 << 2


def walk_s4_pairs(x, sets, hc, s, n_records, n_classes):
    """Label-for-label model of the hard kernel's record walk, which loads
    records two at a time into register quads A (offset o) and B (o+16): a
    rule that goes on past an A record, or starts right after one, continues
    from B without a load.  Non-last folded threshold records take the fast
    path of the walk's direction: >= from a rule's start, <= from the rule's
    flagged first <= record on; special records (feature, zero coefficient,
    always true, last) branch out.  Checks that every compare uses the record
    at its offset and that a fast record's direction is the walk's, that
    every pair read stays inside the stream, that always-true records only
    start rules, and that the walk ends.  Returns per-class prediction counts
    for the rows of x."""
    first, count, default, _ = (int(v) for v in sets[s])
    u = np.ones(x.shape[0], bool)
    f = None
    counts = np.zeros(n_classes, np.int64)
    quad = {}

    def rec(off):
        assert 0 <= first + off // 16 < n_records, "read outside the stream"
        return tuple(int(v) for v in hc[first + off // 16])

    o = 0
    if not u.any():
        return counts
    state, le = "load", False
    for _ in range(4 * count + 8):
        if state in ("load", "next_load"):
            if state == "next_load":
                o += 32
            else:
                le = False  # a rule starts at A
            quad["A"], quad["B"] = rec(o), rec(o + 16)
            state = ("A", "start" if state == "load" else "next")
            continue
        X, mode = state
        r = quad[X]
        assert r == rec(o if X == "A" else o + 16), "compared a stale record"
        w = r[3]
        if mode == "start":
            le = False
        src = u if mode == "start" else f
        cls = (w >> 12) & 63
        fast = not w & (0xa03 if le else 0xa07)
        if not fast and not w & 0xa03:  # a rule's first <= record
            assert w & GE_LE and not le and not w & FF
            le, fast = True, True
        if fast:
            assert not w & FF and bool(w & GE_LE) == le, "compare in the wrong direction"
            f = src & record_mask(x, r)
            if f.any():
                state = ("B", "next") if X == "A" else "next_load"
            else:
                o = w >> 18
                state = "load"
            continue
        le = False  # after a special record the >= labels serve
        if not w & FF and w & ALWAYS:
            assert mode == "start", "always-true record inside a rule"
            counts[cls] += int(u.sum())
            return counts
        f = src & record_mask(x, r)
        alive, last = f.any(), bool(w & LAST)
        if alive and last:
            counts[cls] += int(f.sum())
            u &= ~f
            if not u.any():
                return counts
        if X == "A":
            if alive and not last:
                state = ("B", "next")
            elif last:
                state = ("B", "start")
            else:
                o = w >> 18
                state = "load"
        else:
            if alive and not last:
                state = "next_load"
            elif alive:
                o += 32
                state = "load"
            else:
                o = w >> 18
                state = "load"
    raise AssertionError("record walk did not end")


@pytest.mark.parametrize("seed", range(4))
def test_paired_record_walk_matches_oracle(aerl, seed):
    """The paired-load record walk, run on the packed stream with numpy fp32
    arithmetic over label-uniform 256-sample tiles, reproduces the oracle's
    confusion counts (random populations with empty rules, 1-12 rules of
    1-9 conditions, both kinds, all operators)."""
    from paper_2406_01821_amd import synth
    w = synth.tiny(600 + seed, n=700, nf=9, n_classes=3, n_sets=25, rules=(0, 12),
                   conds=(0, 9), ff_frac=0.4)
    x, y, pop = w.data.x, w.data.y, w.pop
    img = aerl.pack_host(pop, 9, 3)
    sets, hc = decode_packed(img, pop.n_sets, pop.n_rules, pop.n_conds)
    n_records = pop.n_conds + pop.n_rules + pop.n_sets + 1
    _, ref = oracle.hard_eval(x, y, 3, pop)
    for s in range(pop.n_sets):
        got = np.zeros((3, 3), np.int64)
        for c in range(3):
            rows = x[y == c]
            for t in range(0, len(rows), 256):
                got[c] += walk_s4_pairs(rows[t:t + 256], sets, hc, s, n_records, 3)
        np.testing.assert_array_equal(got, ref[s], err_msg=f"set {s}")


def test_record_walk_with_special_values(aerl):
    """The walk model on rule sets mixing every record kind at every pair
    position (signed zeros, zero coefficients, +-inf thresholds, empty
    rules), against the oracle."""
    np.seterr(all="ignore")
    rng = np.random.default_rng(23)
    x = rng.uniform(-2, 2, size=(512, 6)).astype(np.float32)
    x[:60, 0] = 0.0
    x[60:90, 1] = np.float32(-0.0)
    y = np.repeat(np.arange(2, dtype=np.int32), 256)
    pop = synth.special_values_population(24, 6, 2, 60)
    img = aerl.pack_host(pop, 6, 2)
    sets, hc = decode_packed(img, pop.n_sets, pop.n_rules, pop.n_conds)
    n_records = pop.n_conds + pop.n_rules + pop.n_sets + 1
    _, ref = oracle.hard_eval(x, y, 2, pop)
    for s in range(pop.n_sets):
        got = np.zeros((2, 2), np.int64)
        for c in range(2):
            got[c] = walk_s4_pairs(x[y == c], sets, hc, s, n_records, 2)
        np.testing.assert_array_equal(got, ref[s], err_msg=f"set {s}")
    rows = x[:200].copy()
    rows[::7, 0] = np.inf
    rows[::11, 1] = -np.inf
    rows[::13, 2] = np.nan
    for s in range(pop.n_sets):  # prediction rows may be non-finite
        np.testing.assert_array_equal(eval_packed(rows, sets, hc, s), oracle.predict(rows, pop, s),
                                      err_msg=f"set {s}")


def test_hard_kernels_fit_two_blocks_per_cu(tmp_path):
    """The 1024-thread hard-eval kernels must keep a wave's SGPR count at or
    below 80, or two blocks no longer share a CU (half the resident waves);
    a compile of the sources checks the kernel metadata."""
    from paper_2406_01821_amd import build_lib
    counts = {}
    for src in ("hard.hip", "ragged.hip"):
        out = tmp_path / (src + ".s")
        build_lib.asm(src, str(out))
        name = None
        for line in out.read_text().splitlines():
            m = re.match(r"\s+\.name:\s+(\S+)", line)
            if m:
                name = m.group(1)
            m = re.match(r"\s+\.sgpr_count:\s+(\d+)", line)
            if m and name:
                counts[name] = int(m.group(1))
    hard = {k: v for k, v in counts.items() if "k_hardILi" in k or "k_hard_batch" in k}
    # k_hard<4>, <2>, <1> (each with 10- and 16-bit counters) and
    # k_hard_batch, each with and without the categorical walk
    assert len(hard) == 14, counts
    assert all(v <= 80 for v in hard.values()), hard


NO_TEST = int(np.float32(-np.inf).view(np.uint32))


def head_tests(entry):
    """The (table offset, t') pairs of a head entry."""
    hx, hy, hz, hw = (int(v) for v in entry)
    return [(hx >> 14, hy), (hz, hw)]


def eval_packed_filtered(x, sets, hc, hd, nh, s):
    """Model of the filtered walk over the rows of x taken as one tile: with
    the table {max x[f], -min x[f]} at byte offsets 8f and 8f + 4, a rule is
    skipped when table[e] < t' for one of its head entry's two tests; the
    others are walked from their start offset, in order; the closing record
    is always visited.  Returns the predictions and the number of rules
    skipped."""
    first, count, default, _ = (int(v) for v in sets[s])
    n_heads = int(nh[s])
    assert 1 <= n_heads <= count
    table = np.empty(2 * x.shape[1], np.float32)
    table[0::2] = x.max(axis=0)
    table[1::2] = -x.min(axis=0)
    pred = np.full(x.shape[0], -1, np.int32)
    und = np.ones(x.shape[0], bool)
    skipped = 0
    for k in range(n_heads):
        if k < n_heads - 1 and any(table[e // 4] < np.uint32(t).view(np.float32)
                                   for e, t in head_tests(hd[first + k])):
            skipped += 1
            continue
        o = int(hd[first + k][0]) & 0x3fff
        fire = und.copy()
        while True:
            r = tuple(int(v) for v in hc[first + o // 16])
            fire &= record_mask(x, r)
            if r[3] & LAST:
                break
            o += 16
        if fire.any():
            pred[fire] = (r[3] >> 12) & 63
            und &= ~fire
        if not und.any():
            break
    assert not und.any()
    return pred, skipped


def test_head_table_describes_every_rule(aerl):
    """One head entry per rule and one for the closing record: the rule's
    first-record offset and, for each of its first two records that is a
    folded threshold, that record's feature, direction and threshold in the
    table-compare form (no test otherwise)."""
    pop = synth.special_values_population(31, 6, 3, 80)
    img = aerl.pack_host(pop, 6, 3)
    sets, hc, hd, nh = decode_packed(img, pop.n_sets, pop.n_rules, pop.n_conds, heads=True)
    for s in range(pop.n_sets):
        first, count, _, _ = (int(v) for v in sets[s])
        n_rules = int(pop.set_rule_off[s + 1] - pop.set_rule_off[s])
        assert nh[s] == n_rules + 1
        starts = [0]
        for i in range(count - 1):
            if hc[first + i][3] & LAST:
                starts.append(16 * (i + 1))
        assert len(starts) == n_rules + 1 and starts[-1] == 16 * (count - 1)
        for k, o in enumerate(starts):
            assert int(hd[first + k][0]) & 0x3fff == o
            for i, (e, t) in enumerate(head_tests(hd[first + k])):
                r = [int(v) for v in hc[first + o // 16 + i]]
                same_rule = all(not int(hc[first + o // 16 + j][3]) & LAST for j in range(i))
                threshold = same_rule and not r[3] & (FF | MUL | ALWAYS | CAT)
                if not threshold:
                    assert (e, t) == (0, NO_TEST), (s, k, i)
                    continue
                le = bool(r[3] & GE_LE)
                assert e == 8 * (r[0] // 1024) + (4 if le else 0), (s, k, i)
                y = np.uint32(r[1]).view(np.float32)
                assert t == int((-y if le else y).view(np.uint32)), (s, k, i)


@pytest.mark.parametrize("seed", range(3))
def test_head_filter_skips_only_rules_that_cannot_fire(aerl, seed):
    """The filtered walk on tiles of 1-256 rows gives the oracle's
    predictions, and the heavy-tailed workload's thresholds let it skip
    rules."""
    rng = np.random.default_rng(40 + seed)
    w = synth.tiny(50 + seed, n=2048, nf=12, n_classes=3, n_sets=60, rules=(1, 16), conds=(1, 5))
    pops = [w.pop, synth.special_values_population(60 + seed, 12, 3, 40)]
    skipped = 0
    for pop in pops:
        img = aerl.pack_host(pop, 12, 3)
        sets, hc, hd, nh = decode_packed(img, pop.n_sets, pop.n_rules, pop.n_conds, heads=True)
        for n in (1, 7, 64, 256):
            rows = w.data.x[rng.choice(w.data.n, n, replace=False)]
            for s in range(pop.n_sets):
                got, k = eval_packed_filtered(rows, sets, hc, hd, nh, s)
                np.testing.assert_array_equal(got, oracle.predict(rows, pop, s), err_msg=f"set {s}")
                skipped += k
    assert skipped > 0


def test_large_population_packs_like_each_set_alone(aerl):
    """A population large enough to be packed by several host threads (about
    16k conditions per thread) gives, for every rule set, the same records,
    head entries and set fields as that rule set packed on its own."""
    rng = np.random.default_rng(77)
    x = synth.lognormal_features(rng, 500, 24)
    pop = synth.random_population(rng, x, 400, (0, 70), (0, 8), 3, 0.3)
    assert pop.n_conds > 3 * 16384
    img = aerl.pack_host(pop, 24, 3)
    sets, hc, hd, nh = decode_packed(img, pop.n_sets, pop.n_rules, pop.n_conds, heads=True)
    for s in range(0, pop.n_sets, 7):
        one = pop.subset([s])
        img1 = aerl.pack_host(one, 24, 3)
        s1, hc1, hd1, nh1 = decode_packed(img1, 1, one.n_rules, one.n_conds, heads=True)
        first, count = int(sets[s][0]), int(sets[s][1])
        assert int(s1[0][1]) == count and nh1[0] == nh[s]
        assert list(s1[0][2:]) == list(sets[s][2:])
        np.testing.assert_array_equal(hc[first:first + count], hc1[:count], err_msg=f"set {s}")
        np.testing.assert_array_equal(hd[first:first + count], hd1[:count], err_msg=f"set {s}")


def _pool_arrays(pop):
    return [pop.set_rule_off, pop.set_default, pop.rule_cond_off, pop.rule_class, pop.op, pop.kind,
            pop.f, pop.g, pop.coef.view(np.uint32), pop.coef2.view(np.uint32),
            pop.theta.view(np.uint32)]


@pytest.mark.parametrize("nf,nc,kw", [(30, 2, {}), (1, 3, dict(ff_frac=1.0)),
                                      (6, 4, dict(max_rules=1, max_conds=1, elite=0)),
                                      (9, 2, dict(p_crossover=1.0, p_struct=1.0, tournament=1)),
                                      (5, 3, dict(max_rules=3, max_conds=2, p_struct=1.0,
                                                  p_crossover=0.8, p_coef=0.5))])
def test_breeding_matches_the_reference_bit_for_bit(aerl, nf, nc, kw):
    """The library's host-side random pool and next generation (SplitMix64
    draws, tournament selection, crossover, coefficient and structure
    mutation) against oracle/evolve.py over twenty generations of arbitrary
    fitness: identical pools, float bits included, and random states (one
    case keeps rule sets at their rule and condition caps, so that every
    structural change meets its limit)."""
    from oracle import evolve as ev
    from paper_2406_01821_amd.population import from_rule_lists
    c = dict(pool=24, tournament=3, elite=2, max_rules=6, max_conds=4, ff_frac=0.3,
             p_crossover=0.5, p_coef=0.3, p_struct=0.6)
    c.update(kw)
    cfg = aerl.evolve_cfg(**c, seed=11)
    rng = np.random.default_rng(nf)
    lo = rng.normal(size=nf).astype(np.float32)
    hi = (lo + rng.random(nf) * 5).astype(np.float32)
    pop, state = aerl.random_pool(cfg, nf, nc, lo, hi, 11)
    r = ev.SplitMix64(11)
    ref = ev.random_pool(r, c, nf, nc, lo, hi)
    for gen in range(20):
        want = from_rule_lists(ev.to_rule_lists(ref))
        for a, b in zip(_pool_arrays(pop), _pool_arrays(want)):
            np.testing.assert_array_equal(a, b)
        assert state == r.state
        fit = np.random.default_rng(100 + gen).integers(0, 40, size=c["pool"]).astype(np.int32)
        pop, state = aerl.breed(pop, fit, cfg, nf, nc, lo, hi, state)
        ref = ev.next_generation(r, ref, fit, c, nf, nc, lo, hi)


def test_breeding_rejects_bad_input(aerl):
    cfg = aerl.evolve_cfg(pool=4, max_rules=2, max_conds=2)
    lo, hi = np.zeros(3, np.float32), np.ones(3, np.float32)
    pop, st = aerl.random_pool(cfg, 3, 2, lo, hi, 1)
    with pytest.raises(aerl.AerlError):
        aerl.breed(pop, np.zeros(3, np.int32), aerl.evolve_cfg(pool=3, max_rules=2, max_conds=2),
                   3, 2, lo, hi, st)
    with pytest.raises(aerl.AerlError):
        aerl.random_pool(aerl.evolve_cfg(pool=4, elite=4), 3, 2, lo, hi, 1)
    with pytest.raises(aerl.AerlError):
        aerl.random_pool(cfg, 3, 2, hi, lo - 1, 1)
    with pytest.raises(aerl.AerlError):
        aerl.random_pool(aerl.evolve_cfg(pool=4, max_rules=100), 3, 2, lo, hi, 1)
