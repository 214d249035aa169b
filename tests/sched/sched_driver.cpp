// Host test of the serving loop's admission policy (serve_sched.h) with a
// simulated executor.  Requests arrive on a simulated clock; a launch takes
// the FIFO prefix admit_prefix chooses, occupies one of K slots and an arena
// range for a time that grows with its size, then frees both.  After every
// step the driver checks what the serving loop relies on:
//   * ranges of launches in flight never overlap, lie inside the arena, and
//     the allocator's used bytes equal their sum;
//   * free ranges are sorted, disjoint, coalesced, and free + used = arena;
//   * requests launch in arrival order (a later request never overtakes
//     the head), at most max_batch per launch, at most K launches in flight;
//   * when the head does not fit the largest free range nothing launches
//     (back-pressure), and a prefix stops only where the next request
//     breaks one of the admission limits;
//   * every request completes, and the arena is whole again at the end.
// ArenaAlloc's first-fit choices are also compared with a brute-force model
// of the arena, one flag per 256-byte unit.  Prints "ok" and the run's
// launch statistics; exits non-zero at the first violation.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <vector>

#include "serve_sched.h"

using namespace aerl;

static unsigned g_seed = 0;
#define CHECK(c)                                                                       \
  do {                                                                                 \
    if (!(c)) {                                                                        \
      std::fprintf(stderr, "FAILED: %s (line %d, seed %u)\n", #c, __LINE__, g_seed); \
      std::exit(1);                                                                    \
    }                                                                                  \
  } while (0)

constexpr size_t kUnit = 256;

static void check_free_list(const ArenaAlloc &a, size_t arena) {
  size_t free_total = 0, end = 0;
  bool first = true;
  for (const auto &kv : a.free_ranges()) {
    CHECK(kv.second > 0);
    CHECK(first || kv.first > end);  // disjoint and coalesced (a gap before it)
    CHECK(kv.first + kv.second <= arena);
    end = kv.first + kv.second;
    free_total += kv.second;
    first = false;
  }
  CHECK(free_total + a.used() == arena);
}

// First-fit against a brute-force model of the arena (one flag per unit).
static void allocator_against_model(unsigned seed, size_t units, int steps) {
  g_seed = seed;
  std::mt19937_64 rng(seed);
  ArenaAlloc a;
  a.reset(units * kUnit);
  std::vector<char> busy(units, 0);
  std::vector<std::pair<size_t, size_t>> live;  // (offset, bytes)
  for (int i = 0; i < steps; ++i) {
    if (live.empty() || rng() % 3 != 0) {
      const size_t n = 1 + rng() % (units / 4 + 1);
      size_t model = SIZE_MAX;
      for (size_t u = 0, run = 0; u < units; ++u) {
        run = busy[u] ? 0 : run + 1;
        if (run == n) {
          model = u + 1 - n;
          break;
        }
      }
      size_t off = 0;
      const bool ok = a.alloc(n * kUnit, &off);
      CHECK(ok == (model != SIZE_MAX));
      if (ok) {
        CHECK(off == model * kUnit);
        for (size_t u = model; u < model + n; ++u) busy[u] = 1;
        live.push_back({off, n * kUnit});
      }
    } else {
      const size_t k = rng() % live.size();
      a.release(live[k].first, live[k].second);
      for (size_t u = live[k].first / kUnit; u < (live[k].first + live[k].second) / kUnit; ++u)
        busy[u] = 0;
      live[k] = live.back();
      live.pop_back();
    }
    check_free_list(a, units * kUnit);
    size_t largest = 0;
    for (size_t u = 0, run = 0; u < units; ++u) {
      run = busy[u] ? 0 : run + 1;
      largest = std::max(largest, run);
    }
    CHECK(a.largest() == largest * kUnit);
  }
}

struct Rq {
  double arrive;
  QueuedSize sz;
  bool launched = false, done = false;
};

struct Launch {
  size_t off, bytes;
  double end;
  std::vector<int> ids;
  int slot;
};

struct Stats {
  int launches = 0, max_inflight = 0;
  double mean_batch = 0;
  size_t peak_used = 0;
  int held_back = 0;  // steps where a free slot stayed idle because the head did not fit
};

// One simulated run.  slack plays the role of the per-launch table padding.
static Stats simulate(unsigned seed, size_t arena, int slots, int max_batch, int n_req,
                      double mean_gap_us, size_t cap0) {
  g_seed = seed;
  std::mt19937_64 rng(seed);
  const size_t slack = 16 * kUnit;
  std::vector<Rq> rq(n_req);
  double t = 0;
  std::exponential_distribution<double> gap(1.0 / mean_gap_us);
  for (int i = 0; i < n_req; ++i) {
    t += gap(rng);
    // log-uniform device footprint, every request fitting the arena alone
    const double lo = std::log(2.0 * kUnit), hi = std::log((double)(arena - slack));
    size_t dev = (size_t)std::exp(lo + (hi - lo) * std::uniform_real_distribution<double>(0, 1)(rng));
    dev = std::max<size_t>(kUnit, dev / kUnit * kUnit);
    if (dev + slack > arena) dev = arena - slack;
    const size_t in = dev / kUnit * (rng() % 8 + 1) / 10 * kUnit;
    const size_t out = dev - in;
    rq[i] = Rq{t, QueuedSize{dev, in, out}};
  }
  ArenaAlloc a;
  a.reset(arena);
  std::deque<int> pending;
  std::vector<Launch> inflight;
  std::vector<char> slot_busy(slots, 0);
  std::vector<size_t> in_cap(slots, cap0), out_cap(slots, cap0);
  Stats st;
  double now = 0;
  int next = 0, completed = 0, next_launch_id = 0;
  long long batched = 0;
  while (completed < n_req) {
    // completions
    for (size_t k = 0; k < inflight.size();) {
      if (inflight[k].end <= now) {
        a.release(inflight[k].off, inflight[k].bytes);
        for (int id : inflight[k].ids) {
          rq[id].done = true;
          ++completed;
        }
        slot_busy[inflight[k].slot] = 0;
        inflight[k] = inflight.back();
        inflight.pop_back();
      } else {
        ++k;
      }
    }
    // arrivals
    while (next < n_req && rq[next].arrive <= now) pending.push_back(next++);
    // admissions, one launch per free slot while the head fits
    for (int s = 0; s < slots && !pending.empty(); ++s) {
      if (slot_busy[s]) continue;
      size_t need = 0;
      const size_t room = a.largest();
      const int n = admit_prefix(pending, [&](int id) { return rq[id].sz; }, room, max_batch, slack,
                                 in_cap[s], out_cap[s], &need);
      if (n == 0) {
        // back-pressure: only a head that does not fit holds the queue
        CHECK(rq[pending.front()].sz.dev + slack > room);
        ++st.held_back;
        break;
      }
      CHECK(n <= max_batch && need <= room);
      size_t dev = slack, in = slack, out = 0;
      std::vector<int> ids;
      for (int i = 0; i < n; ++i) {
        const int id = pending.front();
        pending.pop_front();
        CHECK(id == next_launch_id);  // arrival order
        ++next_launch_id;
        CHECK(!rq[id].launched);
        rq[id].launched = true;
        dev += rq[id].sz.dev;
        in += rq[id].sz.in;
        out += rq[id].sz.out;
        ids.push_back(id);
      }
      CHECK(dev == need);
      CHECK(n == 1 || (in <= in_cap[s] && out <= out_cap[s]));
      // the prefix stops only where the next request breaks a limit
      if (!pending.empty() && n < max_batch) {
        const QueuedSize q = rq[pending.front()].sz;
        CHECK(dev + q.dev > room || in + q.in > in_cap[s] || out + q.out > out_cap[s]);
      }
      // pinned staging grows for a first request that needs more
      in_cap[s] = std::max(in_cap[s], in);
      out_cap[s] = std::max(out_cap[s], out);
      size_t off = 0;
      CHECK(a.alloc(need, &off));
      for (const Launch &l : inflight) CHECK(off + need <= l.off || l.off + l.bytes <= off);
      CHECK(off + need <= arena);
      const double service = 15.0 + 0.4 * n + (double)need / 4.0e4;
      inflight.push_back(Launch{off, need, now + service, ids, s});
      slot_busy[s] = 1;
      ++st.launches;
      batched += n;
    }
    // invariants
    size_t used = 0;
    for (const Launch &l : inflight) used += l.bytes;
    CHECK(used == a.used() && used <= arena);
    CHECK((int)inflight.size() <= slots);
    check_free_list(a, arena);
    st.max_inflight = std::max(st.max_inflight, (int)inflight.size());
    st.peak_used = std::max(st.peak_used, used);
    // next event; with nothing in flight the head fits the whole arena, so
    // a queue that cannot launch would be a deadlock
    double t_next = next < n_req ? rq[next].arrive : 1e300;
    for (const Launch &l : inflight) t_next = std::min(t_next, l.end);
    if (inflight.empty() && !pending.empty()) CHECK(false);
    if (t_next >= 1e300) CHECK(completed == n_req);
    now = std::max(now, t_next);
  }
  CHECK(a.used() == 0 && a.largest() == arena);
  for (const Rq &r : rq) CHECK(r.launched && r.done);
  st.mean_batch = (double)batched / std::max(st.launches, 1);
  return st;
}

int main() {
  for (unsigned s = 1; s <= 20; ++s) allocator_against_model(s, 64 + s * 7, 4000);
  struct Cfg {
    size_t arena;
    int slots, max_batch, n;
    double gap_us;
    size_t cap0;
  } cfgs[] = {
      {1 << 20, 4, 256, 3000, 5.0, 1 << 16},   // heavy load: batches grow, arena-bound
      {1 << 20, 4, 256, 3000, 200.0, 1 << 16}, // light load: mostly one request per launch
      {64 << 10, 2, 8, 2000, 2.0, 4096},       // tiny arena: constant back-pressure
      {8 << 20, 8, 1, 2000, 1.0, 1 << 20},     // one request per launch, all slots busy
      {1 << 20, 1, 64, 2000, 3.0, 1 << 12},    // one slot, small staging buffers
  };
  unsigned seed = 100;
  for (const Cfg &c : cfgs) {
    for (int rep = 0; rep < 4; ++rep, ++seed) {
      const Stats st = simulate(seed, c.arena, c.slots, c.max_batch, c.n, c.gap_us, c.cap0);
      if (rep == 0)
        std::printf("arena %zu slots %d max_batch %d: %d launches, mean batch %.2f, max in flight "
                    "%d, peak %zu bytes, held back %d times\n",
                    c.arena, c.slots, c.max_batch, st.launches, st.mean_batch, st.max_inflight,
                    st.peak_used, st.held_back);
    }
  }
  std::printf("ok\n");
  return 0;
}
