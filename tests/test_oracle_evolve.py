"""Pins of the evolution reference (oracle/evolve.py): SplitMix64 against
its published first outputs, the ranges of its derived draws, tournament
selection against a replay of the same draws, elitism, and the limits every
child respects."""
import numpy as np

from oracle import evolve as ev


def cfg(**kw):
    c = dict(pool=20, tournament=3, elite=2, max_rules=5, max_conds=3, ff_frac=0.3,
             p_crossover=0.5, p_coef=0.2, p_struct=0.5)
    c.update(kw)
    return c


def test_splitmix64_published_outputs():
    r = ev.SplitMix64(0)
    assert [r.next() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                            0x06C45D188009454F]


def test_draw_ranges_and_exact_floats():
    r = ev.SplitMix64(12345)
    b = [r.below(7) for _ in range(7000)]
    assert min(b) == 0 and max(b) == 6
    counts = np.bincount(b, minlength=7)
    assert counts.min() > 850 and counts.max() < 1150
    for _ in range(1000):
        u = r.unit()
        assert isinstance(u, np.float32) and 0.0 <= u < 1.0
        assert float(u) * 2 ** 24 == int(float(u) * 2 ** 24)


def test_tournament_is_the_best_of_its_draws():
    fit = np.array([5, 9, 9, 1, 7, 9, 0, 3])
    for seed in range(50):
        a, b = ev.SplitMix64(seed), ev.SplitMix64(seed)
        got = ev.tournament(a, fit, 4)
        draws = [b.below(len(fit)) for _ in range(4)]
        best = max(draws, key=lambda i: (fit[i], -i))
        assert got == best


def test_copies_only_generation_replays_the_draws():
    """No variation and no elite: each child is P[i] for the tournament's
    single draw i, and each child consumes exactly the draws the
    specification lists (tournament, crossover test, one test per condition,
    structure test)."""
    rng0 = ev.SplitMix64(7)
    c = cfg(elite=0, tournament=1, p_crossover=0.0, p_coef=0.0, p_struct=0.0)
    lo, hi = np.zeros(4), np.ones(4)
    pool = ev.random_pool(rng0, c, 4, 3, lo, hi)
    fit = np.arange(20)
    a = ev.SplitMix64(99)
    out = ev.next_generation(a, pool, fit, c, 4, 3, lo, hi)
    b = ev.SplitMix64(99)
    for child in out:
        i = b.below(20)
        assert child == pool[i]
        b.unit()  # crossover test
        for _, conds in pool[i][1]:
            for _ in conds:
                b.unit()
        b.unit()  # structure test
    assert a.state == b.state


def test_elite_and_limits():
    lo, hi = np.array([0.0, -1.0, 5.0]), np.array([1.0, 1.0, 5.0])
    c = cfg()
    r = ev.SplitMix64(3)
    pool = ev.random_pool(r, c, 3, 4, lo, hi)
    for gen in range(30):
        fit = np.array([ev.SplitMix64(gen * 100 + i).below(50) for i in range(c["pool"])])
        order = sorted(range(c["pool"]), key=lambda i: (-fit[i], i))
        nxt = ev.next_generation(r, pool, fit, c, 3, 4, lo, hi)
        assert nxt[:2] == [pool[order[0]], pool[order[1]]]
        for d, rules in nxt:
            assert 0 <= d < 4 and 1 <= len(rules) <= c["max_rules"]
            for cls, conds in rules:
                assert 0 <= cls < 4 and 1 <= len(conds) <= c["max_conds"]
                for k in conds:
                    assert 0 <= k["f"] < 3 and 0 <= k["op"] < 4
                    if k["kind"] == 1:
                        assert k["g"] != k["f"] and k["theta"] == 0
                    else:
                        assert lo[k["f"]] <= k["theta"] <= hi[k["f"]] and k["coef2"] == 0
        pool = nxt
