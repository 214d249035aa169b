// Host-side evolution loop that feeds the GPU evaluation (native runtime).
//
// Section 3: evolution runs on the CPU by tournament selection and
// offspring generation with randomized coefficients, candidates are loaded
// onto the GPU for evaluation, and back-propagation can refine each
// candidate's fitness every generation (the Baldwin effect: the tuned
// fitness steers selection, the offspring inherit the untuned rule sets).
// Section 4.1: a fixed pool of 100 candidate rule sets.  The operators are
// specified in include/aerl.h (aerl_evolve_cfg); every random draw comes
// from one SplitMix64 stream in a fixed order, so a run is reproducible from
// its seed and a checkpoint resumes it exactly.
#include <chrono>
#include <cmath>
#include <cstring>
#include <fstream>

#include "internal.h"

namespace aerl {

namespace {

// ------------------------------------------------------------ random stream
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014).
struct Rng {
  uint64_t s;
  uint64_t next() {
    s += 0x9e3779b97f4a7c15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }
  // integer in [0, n) by the multiply-shift of the high 32 bits
  int32_t below(int32_t n) { return (int32_t)(((next() >> 32) * (uint64_t)n) >> 32); }
  // float in [0, 1), 24 random bits (exact in fp32)
  float unit() { return (float)((double)(next() >> 40) * 0x1p-24); }
};

struct Cond {
  uint8_t op, kind;
  int32_t f, g;
  float coef, coef2, theta;
};

struct Ranges {
  int32_t nf, nc;
  const float *lo, *hi;
};

float range_theta(Rng &r, const Ranges &d, int32_t f) {
  const double u = (double)r.unit();
  return (float)((double)d.lo[f] + u * ((double)d.hi[f] - (double)d.lo[f]));
}

Cond random_cond(Rng &r, const aerl_evolve_cfg &c, const Ranges &d) {
  Cond k{};
  const bool ff = r.unit() < c.ff_frac && d.nf >= 2;
  k.f = r.below(d.nf);
  k.g = ff ? (k.f + 1 + r.below(d.nf - 1)) % d.nf : 0;
  k.op = (uint8_t)r.below(4);
  k.coef = r.unit();
  k.kind = ff ? 1 : 0;
  if (ff) {
    k.coef2 = r.unit();
    k.theta = 0.0f;
  } else {
    k.coef2 = 0.0f;
    k.theta = range_theta(r, d, k.f);
  }
  return k;
}

int32_t tournament(Rng &r, const int32_t *fit, int32_t n, int32_t k) {
  int32_t best = -1;
  for (int32_t t = 0; t < k; ++t) {
    const int32_t i = r.below(n);
    if (best < 0 || fit[i] > fit[best] || (fit[i] == fit[best] && i < best)) best = i;
  }
  return best;
}

// ------------------------------------------------------------ pools
// A pool in the flat form of aerl_population, owning its arrays; the fields
// a condition's kind does not use are 0 (g, coef2 of a threshold, theta of a
// feature-vs-feature condition).
struct Soa {
  std::vector<int32_t> set_rule_off, set_default, rule_cond_off, rule_class, f, g;
  std::vector<uint8_t> op, kind;
  std::vector<float> coef, coef2, theta;
  int32_t n_sets() const { return (int32_t)set_default.size(); }
  void clear() {
    set_rule_off.assign(1, 0);
    rule_cond_off.assign(1, 0);
    for (auto *v : {&set_default, &rule_class, &f, &g}) v->clear();
    op.clear();
    kind.clear();
    coef.clear();
    coef2.clear();
    theta.clear();
  }
  Cond cond(int32_t j) const { return Cond{op[j], kind[j], f[j], g[j], coef[j], coef2[j], theta[j]}; }
  void push_cond(const Cond &k) {
    op.push_back(k.op);
    kind.push_back(k.kind);
    f.push_back(k.f);
    g.push_back(k.g);
    coef.push_back(k.coef);
    coef2.push_back(k.coef2);
    theta.push_back(k.theta);
  }
  void end_rule(int32_t cls) {
    rule_class.push_back(cls);
    rule_cond_off.push_back((int32_t)op.size());
  }
  void end_set(int32_t dflt) {
    set_default.push_back(dflt);
    set_rule_off.push_back((int32_t)rule_class.size());
  }
  // rule set s of `from` appended unchanged
  void copy_set(const Soa &from, int32_t s) {
    for (int32_t r = from.set_rule_off[s]; r < from.set_rule_off[s + 1]; ++r) {
      for (int32_t j = from.rule_cond_off[r]; j < from.rule_cond_off[r + 1]; ++j) push_cond(from.cond(j));
      end_rule(from.rule_class[r]);
    }
    end_set(from.set_default[s]);
  }
  aerl_population view() const {
    aerl_population p{};
    p.n_sets = n_sets();
    p.set_rule_off = set_rule_off.data();
    p.set_default = set_default.data();
    p.rule_cond_off = rule_cond_off.data();
    p.rule_class = rule_class.data();
    p.op = op.data();
    p.kind = kind.data();
    p.f = f.data();
    p.g = g.data();
    p.coef = coef.data();
    p.coef2 = coef2.data();
    p.theta = theta.data();
    return p;
  }
};

// A validated caller pool of kinds 0 and 1 in flat form.
Soa from_view(const aerl_population &p) {
  Soa a;
  a.clear();
  for (int32_t s = 0; s < p.n_sets; ++s) {
    for (int32_t r = p.set_rule_off[s]; r < p.set_rule_off[s + 1]; ++r) {
      for (int32_t j = p.rule_cond_off[r]; j < p.rule_cond_off[r + 1]; ++j) {
        const bool ff = p.kind[j] != 0;
        a.push_cond(Cond{p.op[j], p.kind[j], p.f[j], ff ? p.g[j] : 0, p.coef[j],
                         ff ? p.coef2[j] : 0.0f, ff ? 0.0f : p.theta[j]});
      }
      a.end_rule(p.rule_class[r]);
    }
    a.end_set(p.set_default[s]);
  }
  return a;
}

// Whether every rule set has 1..max_rules rules of 1..max_conds conditions.
bool within_limits(const aerl_population &p, const aerl_evolve_cfg &c) {
  for (int32_t s = 0; s < p.n_sets; ++s) {
    const int32_t R = p.set_rule_off[s + 1] - p.set_rule_off[s];
    if (R < 1 || R > c.max_rules) return false;
    for (int32_t r = p.set_rule_off[s]; r < p.set_rule_off[s + 1]; ++r) {
      const int32_t K = p.rule_cond_off[r + 1] - p.rule_cond_off[r];
      if (K < 1 || K > c.max_conds) return false;
    }
  }
  return true;
}

// The child being bred: its rules in order, each a range of a condition
// buffer (rules added by a structural change put their condition at the
// end of the buffer, so the ranges need not follow the rule order).
struct Child {
  struct RuleRef {
    int32_t cls, start, count;
  };
  std::vector<RuleRef> rules;
  std::vector<Cond> conds;
  void add_rule(const Soa &p, int32_t r) {
    const int32_t start = (int32_t)conds.size();
    for (int32_t j = p.rule_cond_off[r]; j < p.rule_cond_off[r + 1]; ++j) conds.push_back(p.cond(j));
    rules.push_back({p.rule_class[r], start, p.rule_cond_off[r + 1] - p.rule_cond_off[r]});
  }
  // shift the ranges that start at or after `at` by d
  void shift_from(int32_t at, int32_t d) {
    for (RuleRef &u : rules)
      if (u.start >= at) u.start += d;
  }
};

// The next generation (the operators specified with aerl_evolve_cfg), into
// `out`; `ch` is scratch.  The random draws come in the same order as in
// the specification: the elite need none; each child draws its tournament,
// the crossover decision (and its second tournament and two cut points),
// one redraw decision per condition in rule order (and the redrawn values),
// the structural decision and its draws.
void breed(Rng &r, const Soa &pool, const int32_t *fit, const aerl_evolve_cfg &c, const Ranges &d,
           Soa &out, Child &ch) {
  const int32_t n = pool.n_sets();
  std::vector<int32_t> order(n);
  for (int32_t i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return fit[a] > fit[b]; });
  out.clear();
  for (int32_t i = 0; i < c.elite; ++i) out.copy_set(pool, order[i]);
  std::vector<std::pair<int32_t, int32_t>> refs;  // (rule set, rule) of the child's rules
  refs.reserve(2 * (size_t)c.max_rules + 1);
  for (int32_t i = c.elite; i < n; ++i) {
    const int32_t pa = tournament(r, fit, n, c.tournament);
    const int32_t a0 = pool.set_rule_off[pa], a1 = pool.set_rule_off[pa + 1];
    refs.clear();
    if (r.unit() < c.p_crossover) {
      const int32_t pb = tournament(r, fit, n, c.tournament);
      const int32_t b0 = pool.set_rule_off[pb], b1 = pool.set_rule_off[pb + 1];
      const int32_t ca = r.below(a1 - a0 + 1);
      const int32_t cb = r.below(b1 - b0 + 1);
      for (int32_t k = a0; k < a0 + ca; ++k) refs.push_back({pa, k});
      for (int32_t k = b0 + cb; k < b1; ++k) refs.push_back({pb, k});
      if (refs.empty()) refs.push_back({pa, a0});
      if ((int32_t)refs.size() > c.max_rules) refs.resize(c.max_rules);
    } else {
      for (int32_t k = a0; k < a1; ++k) refs.push_back({pa, k});
    }
    ch.rules.clear();
    ch.conds.clear();
    for (const auto &rf : refs) ch.add_rule(pool, rf.second);
    // the conditions of the rules in order: the buffer holds them so
    for (Cond &k : ch.conds) {
      if (r.unit() < c.p_coef) {
        k.coef = r.unit();
        if (k.kind == 1)
          k.coef2 = r.unit();
        else
          k.theta = range_theta(r, d, k.f);
      }
    }
    if (r.unit() < c.p_struct) {
      const int32_t t = r.below(4);
      const int32_t R = (int32_t)ch.rules.size();
      if (t == 0) {  // add a condition at the end of a rule
        const int32_t u = r.below(R);
        if (ch.rules[u].count < c.max_conds) {
          const int32_t at = ch.rules[u].start + ch.rules[u].count;
          const Cond k = random_cond(r, c, d);
          ch.shift_from(at, 1);
          ch.rules[u].count += 1;
          ch.conds.insert(ch.conds.begin() + at, k);
        }
      } else if (t == 1) {  // drop a condition of a rule that keeps one
        const int32_t u = r.below(R);
        if (ch.rules[u].count >= 2) {
          const int32_t at = ch.rules[u].start + r.below(ch.rules[u].count);
          ch.conds.erase(ch.conds.begin() + at);
          ch.rules[u].count -= 1;
          ch.shift_from(at + 1, -1);
        }
      } else if (t == 2) {  // a new one-condition rule at a random position
        if (R < c.max_rules) {
          const int32_t pos = r.below(R + 1);
          const int32_t cls = r.below(d.nc);
          ch.conds.push_back(random_cond(r, c, d));
          ch.rules.insert(ch.rules.begin() + pos, {cls, (int32_t)ch.conds.size() - 1, 1});
        }
      } else if (R >= 2) {  // drop a rule
        ch.rules.erase(ch.rules.begin() + r.below(R));
      }
    }
    for (const Child::RuleRef &u : ch.rules) {
      for (int32_t k = 0; k < u.count; ++k) out.push_cond(ch.conds[u.start + k]);
      out.end_rule(u.cls);
    }
    out.end_set(pool.set_default[pa]);
  }
}

Soa random_pool(Rng &r, const aerl_evolve_cfg &c, const Ranges &d) {
  Soa a;
  a.clear();
  for (int32_t s = 0; s < c.pool; ++s) {
    const int32_t R = 1 + r.below(c.max_rules);
    const int32_t dflt = r.below(d.nc);
    for (int32_t k = 0; k < R; ++k) {
      const int32_t K = 1 + r.below(c.max_conds);
      const int32_t cls = r.below(d.nc);
      for (int32_t j = 0; j < K; ++j) a.push_cond(random_cond(r, c, d));
      a.end_rule(cls);
    }
    a.end_set(dflt);
  }
  return a;
}

aerl_status write_out(const Soa &a, aerl_population_out *o) {
  if (!o || !o->set_rule_off || !o->set_default || !o->rule_cond_off || !o->rule_class || !o->op ||
      !o->kind || !o->f || !o->g || !o->coef || !o->coef2 || !o->theta)
    return AERL_EINVAL;
  // capacities: pool + 1, pool, pool * max_rules + 1, pool * max_rules * max_conds
  std::memcpy(o->set_rule_off, a.set_rule_off.data(), a.set_rule_off.size() * 4);
  std::memcpy(o->set_default, a.set_default.data(), a.set_default.size() * 4);
  std::memcpy(o->rule_cond_off, a.rule_cond_off.data(), a.rule_cond_off.size() * 4);
  std::memcpy(o->rule_class, a.rule_class.data(), a.rule_class.size() * 4);
  std::memcpy(o->op, a.op.data(), a.op.size());
  std::memcpy(o->kind, a.kind.data(), a.kind.size());
  std::memcpy(o->f, a.f.data(), a.f.size() * 4);
  std::memcpy(o->g, a.g.data(), a.g.size() * 4);
  std::memcpy(o->coef, a.coef.data(), a.coef.size() * 4);
  std::memcpy(o->coef2, a.coef2.data(), a.coef2.size() * 4);
  std::memcpy(o->theta, a.theta.data(), a.theta.size() * 4);
  o->n_sets = a.n_sets();
  o->n_rules = (int32_t)a.rule_class.size();
  o->n_conds = (int32_t)a.op.size();
  return AERL_OK;
}

// The loop breeds threshold and feature-vs-feature conditions only.
aerl_status check_kinds(aerl_ctx *ctx, const aerl_population &p, int32_t n_conds) {
  for (int32_t j = 0; j < n_conds; ++j)
    if (p.kind[j] > AERL_KIND_FEATURE)
      return fail(ctx, AERL_EINVAL, "condition %d: the evolution loop breeds kinds 0 and 1 only", j);
  return AERL_OK;
}

aerl_status check_cfg(aerl_ctx *ctx, const aerl_evolve_cfg *c, int32_t nf, int32_t nc, const float *lo,
                      const float *hi) {
  if (!c) return fail(ctx, AERL_EINVAL, "cfg is NULL");
  if (c->pool < 2 || c->tournament < 1 || c->elite < 0 || c->elite >= c->pool)
    return fail(ctx, AERL_EINVAL, "pool >= 2, tournament >= 1 and 0 <= elite < pool are required");
  if (c->max_rules < 1 || c->max_rules > kMaxEvolveRules || c->max_conds < 1 ||
      c->max_conds > AERL_MAX_RULE_CONDS ||
      (int64_t)c->max_rules * c->max_conds > kMaxSetRecords - 1)
    return fail(ctx, AERL_EINVAL, "max_rules in [1, %d], max_conds in [1, %d], product < %d", kMaxEvolveRules,
                AERL_MAX_RULE_CONDS, kMaxSetRecords - 1);
  if ((int64_t)c->pool * c->max_rules * c->max_conds > INT32_MAX)
    return fail(ctx, AERL_EINVAL, "pool x max_rules x max_conds exceeds 2^31 - 1");
  for (float p : {c->ff_frac, c->p_crossover, c->p_coef, c->p_struct})
    if (!(p >= 0.0f && p <= 1.0f)) return fail(ctx, AERL_EINVAL, "probabilities must lie in [0, 1]");
  if (c->tune_epochs < 0) return fail(ctx, AERL_EINVAL, "tune_epochs < 0");
  if (nf < 1 || nf > AERL_MAX_FEATURES || nc < 1 || nc > AERL_MAX_CLASSES)
    return fail(ctx, AERL_EINVAL, "feature or class count out of range");
  if (!lo || !hi) return fail(ctx, AERL_EINVAL, "feature ranges are NULL");
  for (int32_t f = 0; f < nf; ++f)
    if (!std::isfinite(lo[f]) || !std::isfinite(hi[f]) || lo[f] > hi[f])
      return fail(ctx, AERL_EINVAL, "feature %d: range [%g, %g] is not finite and ordered", f, lo[f], hi[f]);
  return AERL_OK;
}

}  // namespace

// ------------------------------------------------------------ the GPU loop
struct Evo {
  aerl_evolve_cfg cfg{};
  int32_t dataset_id = 0, nf = 0, nc = 0;
  std::vector<float> lo, hi;
  Rng rng{0};
  int32_t generation = 0;
  Soa pool;                      // the pool as last evaluated (state views point here)
  Soa next;                      // breeding output, swapped in
  Child scratch;
  std::vector<int32_t> fitness;
  std::vector<float> tuned[3];   // tuned coef, coef2, theta of that pool
  char *arena = nullptr;
  size_t arena_bytes = 0;
  EvolveArena layout{};
  void *staging = nullptr;       // pinned host image of a packed pool
  int32_t *fit_pinned = nullptr; // pinned landing place of the fitness counts
  double sec_eval = 0, sec_tune = 0, sec_breed = 0;
  ~Evo() {
    if (staging) (void)hipHostFree(staging);
    if (fit_pinned) (void)hipHostFree(fit_pinned);
  }
};

void destroy_evo(Evo *e) { delete e; }

EvolveArena evolve_arena(const DatasetRec &ds, const aerl_evolve_cfg &c) {
  EvolveArena A{};
  const int64_t rules = (int64_t)c.pool * c.max_rules, conds = rules * c.max_conds;
  const PackedLayout L = packed_layout(c.pool, (int32_t)rules, (int32_t)conds);
  auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
  size_t off = 0;
  A.pack_off = off;    off = al(off + L.total);
  A.pack_bytes = L.total;
  A.correct_off = off; off = al(off + (size_t)c.pool * 4);
  A.param_off = off;   off = al(off + 3 * (size_t)std::max<int64_t>(conds, 1) * 4);
  A.tune_off = off;
  if (c.tune_epochs > 0) {
    PopRec bound;
    bound.n_sets = c.pool;
    bound.n_rules = (int32_t)rules;
    bound.n_conds = (int32_t)conds;
    bound.max_rules = c.max_rules;
    bound.max_rule_conds = c.max_conds;
    bound.max_set_conds = c.max_rules * c.max_conds;
    bound.nf = ds.nf;
    bound.nc = ds.nc;
    A.tune_bytes = tune_layout(ds, bound).total;
    A.tune_ok = soft_backward_supported(ds, bound);
    off = al(off + A.tune_bytes);
  }
  A.total = off;
  A.staging_bytes = L.total;
  return A;
}

namespace {

// Evaluates e.pool: fitness (of the tuned rule sets when fine-tuning) into
// e.fitness, tuned parameters into e.tuned.  Synchronous.
aerl_status evaluate(aerl_ctx *ctx, Evo &e, hipStream_t st) {
  using clk = std::chrono::steady_clock;
  aerl_population view = e.pool.view();
  const size_t nconds = e.pool.op.size();
  char *pack = e.arena + e.layout.pack_off;
  int32_t *correct = reinterpret_cast<int32_t *>(e.arena + e.layout.correct_off);
  float *par = reinterpret_cast<float *>(e.arena + e.layout.param_off);
  int32_t pid = 0;
  aerl_status s = pack_staged(ctx, &view, e.nf, e.nc, pack, e.layout.pack_bytes, e.staging,
                              e.layout.staging_bytes, st, &pid);
  if (s) return s;
  for (auto &t : e.tuned) t.clear();
  if (e.cfg.tune_epochs > 0) {
    const auto t0 = clk::now();
    const float *src[3] = {e.pool.coef.data(), e.pool.coef2.data(), e.pool.theta.data()};
    for (int k = 0; k < 3; ++k)
      AERL_HIP(ctx, hipMemcpyAsync(par + k * nconds, src[k], nconds * 4, hipMemcpyHostToDevice, st));
    aerl_finetune_cfg tc = e.cfg.tune;
    tc.epochs = e.cfg.tune_epochs;
    s = aerl_finetune(ctx, e.dataset_id, pid, &tc, par, par + nconds, par + 2 * nconds, nullptr,
                      e.arena + e.layout.tune_off, e.layout.tune_bytes, st);
    if (s) {
      (void)aerl_release_population(ctx, pid);
      return s;
    }
    for (int k = 0; k < 3; ++k) {
      e.tuned[k].resize(nconds);
      AERL_HIP(ctx, hipMemcpyAsync(e.tuned[k].data(), par + k * nconds, nconds * 4,
                                   hipMemcpyDeviceToHost, st));
    }
    AERL_HIP(ctx, hipStreamSynchronize(st));
    (void)aerl_release_population(ctx, pid);
    view.coef = e.tuned[0].data();
    view.coef2 = e.tuned[1].data();
    view.theta = e.tuned[2].data();
    s = pack_staged(ctx, &view, e.nf, e.nc, pack, e.layout.pack_bytes, e.staging,
                    e.layout.staging_bytes, st, &pid);
    if (s) return s;
    e.sec_tune += std::chrono::duration<double>(clk::now() - t0).count();
  }
  const auto t1 = clk::now();
  s = aerl_eval_population(ctx, e.dataset_id, pid, correct, nullptr, st);
  if (s == AERL_OK) {
    const int32_t n = e.pool.n_sets();
    hipError_t h = hipMemcpyAsync(e.fit_pinned, correct, (size_t)n * 4, hipMemcpyDeviceToHost, st);
    if (h == hipSuccess) h = hipStreamSynchronize(st);
    if (h != hipSuccess) s = fail(ctx, AERL_EDEVICE, "fitness copy failed: %s", hipGetErrorString(h));
    else e.fitness.assign(e.fit_pinned, e.fit_pinned + n);
  }
  (void)aerl_release_population(ctx, pid);
  e.sec_eval += std::chrono::duration<double>(clk::now() - t1).count();
  return s;
}

aerl_status attach(aerl_ctx *ctx, Evo &e, int32_t dataset_id, void *arena, size_t arena_bytes) {
  auto di = ctx->datasets.find(dataset_id);
  if (di == ctx->datasets.end()) return fail(ctx, AERL_ENOENT, "unknown dataset %d", dataset_id);
  if (di->second.nf != e.nf || di->second.nc != e.nc)
    return fail(ctx, AERL_EINVAL, "dataset has %d features / %d classes, the run %d / %d", di->second.nf,
                di->second.nc, e.nf, e.nc);
  e.dataset_id = dataset_id;
  e.layout = evolve_arena(di->second, e.cfg);
  if (e.cfg.tune_epochs > 0 && !e.layout.tune_ok)
    return fail(ctx, AERL_EINVAL, "rule sets of %d rules are too long to fine-tune", e.cfg.max_rules);
  if (!arena || ((uintptr_t)arena & 255)) return fail(ctx, AERL_EINVAL, "arena is NULL or not 256-byte aligned");
  if (arena_bytes < e.layout.total)
    return fail(ctx, AERL_ENOMEM, "arena holds %zu bytes, %zu needed", arena_bytes, e.layout.total);
  e.arena = static_cast<char *>(arena);
  e.arena_bytes = arena_bytes;
  AERL_HIP(ctx, hipHostMalloc(&e.staging, e.layout.staging_bytes, hipHostMallocDefault));
  AERL_HIP(ctx, hipHostMalloc(reinterpret_cast<void **>(&e.fit_pinned),
                              (size_t)std::max(e.cfg.pool, 1) * 4, hipHostMallocDefault));
  return AERL_OK;
}

const uint64_t kCkptMagic = 0x314f5645'4c524541ull;  // "AERLEVO1"

template <class T>
void put(std::ofstream &o, const std::vector<T> &v) {
  const uint64_t n = v.size();
  o.write(reinterpret_cast<const char *>(&n), 8);
  if (n) o.write(reinterpret_cast<const char *>(v.data()), (std::streamsize)(n * sizeof(T)));
}
template <class T>
bool get(std::ifstream &i, std::vector<T> &v, uint64_t max_n) {
  uint64_t n = 0;
  if (!i.read(reinterpret_cast<char *>(&n), 8) || n > max_n) return false;
  v.resize(n);
  return n == 0 || (bool)i.read(reinterpret_cast<char *>(v.data()), (std::streamsize)(n * sizeof(T)));
}

}  // namespace
}  // namespace aerl

using namespace aerl;

extern "C" {

aerl_status aerl_random_pool(const aerl_evolve_cfg *cfg, int32_t nf, int32_t nc, const float *lo,
                             const float *hi, uint64_t *rng_state, aerl_population_out *out) {
  aerl_status s = check_cfg(nullptr, cfg, nf, nc, lo, hi);
  if (s) return s;
  if (!rng_state) return AERL_EINVAL;
  Rng r{*rng_state};
  s = write_out(random_pool(r, *cfg, Ranges{nf, nc, lo, hi}), out);
  if (s == AERL_OK) *rng_state = r.s;
  return s;
}

aerl_status aerl_breed(const aerl_population *pool, const int32_t *fitness, const aerl_evolve_cfg *cfg,
                       int32_t nf, int32_t nc, const float *lo, const float *hi, uint64_t *rng_state,
                       aerl_population_out *out) {
  aerl_status s = check_cfg(nullptr, cfg, nf, nc, lo, hi);
  if (s) return s;
  if (!rng_state || !fitness) return AERL_EINVAL;
  int32_t nr = 0, nk = 0;
  s = validate_population(nullptr, pool, nf, nc, &nr, &nk);
  if (s) return s;
  if (pool->n_sets != cfg->pool || check_kinds(nullptr, *pool, nk) || !within_limits(*pool, *cfg))
    return AERL_EINVAL;
  const Soa in = from_view(*pool);
  Rng r{*rng_state};
  Soa next;
  Child scratch;
  breed(r, in, fitness, *cfg, Ranges{nf, nc, lo, hi}, next, scratch);
  s = write_out(next, out);
  if (s == AERL_OK) *rng_state = r.s;
  return s;
}

aerl_status aerl_evolve_arena_bytes(aerl_ctx *ctx, int32_t dataset_id, const aerl_evolve_cfg *cfg,
                                    size_t *bytes) {
  if (!ctx || !bytes || !cfg) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  auto di = ctx->datasets.find(dataset_id);
  if (di == ctx->datasets.end()) return fail(ctx, AERL_ENOENT, "unknown dataset %d", dataset_id);
  *bytes = evolve_arena(di->second, *cfg).total;
  return AERL_OK;
}

aerl_status aerl_evolve_create(aerl_ctx *ctx, int32_t dataset_id, const aerl_evolve_cfg *cfg,
                               const float *lo, const float *hi, const aerl_population *initial,
                               void *arena, size_t arena_bytes, hipStream_t stream, int32_t *evo_id) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->err.clear();
  if (!evo_id) return fail(ctx, AERL_EINVAL, "evo_id is NULL");
  auto di = ctx->datasets.find(dataset_id);
  if (di == ctx->datasets.end()) return fail(ctx, AERL_ENOENT, "unknown dataset %d", dataset_id);
  const int32_t nf = di->second.nf, nc = di->second.nc;
  aerl_status s = check_cfg(ctx, cfg, nf, nc, lo, hi);
  if (s) return s;
  std::unique_ptr<Evo, EvoDeleter> e(new Evo());
  e->cfg = *cfg;
  e->nf = nf;
  e->nc = nc;
  e->lo.assign(lo, lo + nf);
  e->hi.assign(hi, hi + nf);
  e->rng.s = cfg->seed;
  if (initial) {
    int32_t nr = 0, nk = 0;
    s = validate_population(ctx, initial, nf, nc, &nr, &nk);
    if (s) return s;
    s = check_kinds(ctx, *initial, nk);
    if (s) return s;
    if (initial->n_sets != cfg->pool)
      return fail(ctx, AERL_EINVAL, "initial population has %d rule sets, the pool %d", initial->n_sets, cfg->pool);
    if (!within_limits(*initial, *cfg))
      return fail(ctx, AERL_EINVAL,
                  "initial rule sets need 1..max_rules rules of 1..max_conds conditions");
    e->pool = from_view(*initial);
  } else {
    e->pool = random_pool(e->rng, *cfg, Ranges{nf, nc, e->lo.data(), e->hi.data()});
  }
  s = attach(ctx, *e, dataset_id, arena, arena_bytes);
  if (s) return s;
  AERL_HIP(ctx, hipSetDevice(ctx->device));
  s = evaluate(ctx, *e, stream);
  if (s) return s;
  const int32_t id = ctx->next_id++;
  ctx->evos[id] = std::move(e);
  *evo_id = id;
  return AERL_OK;
}

aerl_status aerl_evolve_run(aerl_ctx *ctx, int32_t evo_id, int32_t generations, hipStream_t stream) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->err.clear();
  auto it = ctx->evos.find(evo_id);
  if (it == ctx->evos.end()) return fail(ctx, AERL_ENOENT, "unknown run %d", evo_id);
  if (generations < 0) return fail(ctx, AERL_EINVAL, "generations < 0");
  Evo &e = *it->second;
  if (!ctx->datasets.count(e.dataset_id)) return fail(ctx, AERL_ENOENT, "the run's dataset was released");
  AERL_HIP(ctx, hipSetDevice(ctx->device));
  for (int32_t g = 0; g < generations; ++g) {
    const auto t0 = std::chrono::steady_clock::now();
    breed(e.rng, e.pool, e.fitness.data(), e.cfg, Ranges{e.nf, e.nc, e.lo.data(), e.hi.data()}, e.next,
          e.scratch);
    std::swap(e.pool, e.next);
    e.sec_breed += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    aerl_status s = evaluate(ctx, e, stream);
    if (s) return s;
    ++e.generation;
  }
  return AERL_OK;
}

aerl_status aerl_evolve_state(aerl_ctx *ctx, int32_t evo_id, aerl_evolve_info *out) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  auto it = ctx->evos.find(evo_id);
  if (it == ctx->evos.end()) return fail(ctx, AERL_ENOENT, "unknown run %d", evo_id);
  if (!out) return fail(ctx, AERL_EINVAL, "out is NULL");
  const Evo &e = *it->second;
  std::memset(out, 0, sizeof *out);
  out->generation = e.generation;
  out->pool = e.pool.view();
  out->fitness = e.fitness.data();
  const bool tuned = e.cfg.tune_epochs > 0;
  out->tuned_coef = tuned ? e.tuned[0].data() : nullptr;
  out->tuned_coef2 = tuned ? e.tuned[1].data() : nullptr;
  out->tuned_theta = tuned ? e.tuned[2].data() : nullptr;
  out->rng_state = e.rng.s;
  out->seconds_eval = e.sec_eval;
  out->seconds_tune = e.sec_tune;
  out->seconds_breed = e.sec_breed;
  return AERL_OK;
}

aerl_status aerl_evolve_save(aerl_ctx *ctx, int32_t evo_id, const char *path) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  auto it = ctx->evos.find(evo_id);
  if (it == ctx->evos.end()) return fail(ctx, AERL_ENOENT, "unknown run %d", evo_id);
  if (!path) return fail(ctx, AERL_EINVAL, "path is NULL");
  const Evo &e = *it->second;
  std::ofstream o(path, std::ios::binary | std::ios::trunc);
  if (!o) return fail(ctx, AERL_EINVAL, "cannot open %s", path);
  o.write(reinterpret_cast<const char *>(&kCkptMagic), 8);
  o.write(reinterpret_cast<const char *>(&e.cfg), sizeof e.cfg);
  const int32_t head[3] = {e.nf, e.nc, e.generation};
  o.write(reinterpret_cast<const char *>(head), sizeof head);
  o.write(reinterpret_cast<const char *>(&e.rng.s), 8);
  put(o, e.lo);
  put(o, e.hi);
  const Soa &a = e.pool;
  put(o, a.set_rule_off); put(o, a.set_default); put(o, a.rule_cond_off); put(o, a.rule_class);
  put(o, a.op); put(o, a.kind); put(o, a.f); put(o, a.g);
  put(o, a.coef); put(o, a.coef2); put(o, a.theta);
  put(o, e.fitness);
  for (const auto &t : e.tuned) put(o, t);
  if (!o) return fail(ctx, AERL_EINVAL, "writing %s failed", path);
  return AERL_OK;
}

aerl_status aerl_evolve_load(aerl_ctx *ctx, int32_t dataset_id, const char *path, void *arena,
                             size_t arena_bytes, int32_t *evo_id) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->err.clear();
  if (!path || !evo_id) return fail(ctx, AERL_EINVAL, "path or evo_id is NULL");
  std::ifstream i(path, std::ios::binary);
  if (!i) return fail(ctx, AERL_ENOENT, "cannot open %s", path);
  uint64_t magic = 0;
  std::unique_ptr<Evo, EvoDeleter> e(new Evo());
  int32_t head[3] = {};
  if (!i.read(reinterpret_cast<char *>(&magic), 8) || magic != kCkptMagic ||
      !i.read(reinterpret_cast<char *>(&e->cfg), sizeof e->cfg) ||
      !i.read(reinterpret_cast<char *>(head), sizeof head) ||
      !i.read(reinterpret_cast<char *>(&e->rng.s), 8))
    return fail(ctx, AERL_EINVAL, "%s is not an evolution checkpoint", path);
  e->nf = head[0];
  e->nc = head[1];
  e->generation = head[2];
  const uint64_t cap = 1ull << 31;
  Soa a;
  bool ok = get(i, e->lo, AERL_MAX_FEATURES) && get(i, e->hi, AERL_MAX_FEATURES) &&
            get(i, a.set_rule_off, cap) && get(i, a.set_default, cap) && get(i, a.rule_cond_off, cap) &&
            get(i, a.rule_class, cap) && get(i, a.op, cap) && get(i, a.kind, cap) && get(i, a.f, cap) &&
            get(i, a.g, cap) && get(i, a.coef, cap) && get(i, a.coef2, cap) && get(i, a.theta, cap) &&
            get(i, e->fitness, cap);
  for (auto &t : e->tuned) ok = ok && get(i, t, cap);
  if (!ok || (int32_t)e->lo.size() != e->nf || (int32_t)e->hi.size() != e->nf)
    return fail(ctx, AERL_EINVAL, "%s is truncated or inconsistent", path);
  aerl_status s = check_cfg(ctx, &e->cfg, e->nf, e->nc, e->lo.data(), e->hi.data());
  if (s) return s;
  const aerl_population v = a.view();
  const size_t n_sets = a.set_default.size();
  int32_t nr = 0, nk = 0;
  if (n_sets != (size_t)e->cfg.pool || a.set_rule_off.size() != n_sets + 1 ||
      a.rule_cond_off.size() != a.rule_class.size() + 1 || e->fitness.size() != n_sets ||
      a.f.size() != a.op.size() || a.g.size() != a.op.size() || a.kind.size() != a.op.size() ||
      a.coef.size() != a.op.size() || a.coef2.size() != a.op.size() || a.theta.size() != a.op.size() ||
      validate_population(ctx, &v, e->nf, e->nc, &nr, &nk) != AERL_OK ||
      (size_t)nr != a.rule_class.size() || (size_t)nk != a.op.size() ||
      check_kinds(ctx, v, nk) != AERL_OK || !within_limits(v, e->cfg))
    return fail(ctx, AERL_EINVAL, "%s holds an invalid pool", path);
  e->pool = from_view(v);
  s = attach(ctx, *e, dataset_id, arena, arena_bytes);
  if (s) return s;
  const int32_t id = ctx->next_id++;
  ctx->evos[id] = std::move(e);
  *evo_id = id;
  return AERL_OK;
}

aerl_status aerl_evolve_release(aerl_ctx *ctx, int32_t evo_id) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (!ctx->evos.erase(evo_id)) return fail(ctx, AERL_ENOENT, "unknown run %d", evo_id);
  return AERL_OK;
}

}  // extern "C"
