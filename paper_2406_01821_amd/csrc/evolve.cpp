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
struct Rule {
  int32_t cls;
  std::vector<Cond> conds;
};
struct Set {
  int32_t dflt;
  std::vector<Rule> rules;
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

Rule random_rule(Rng &r, const aerl_evolve_cfg &c, const Ranges &d) {
  Rule u;
  u.cls = r.below(d.nc);
  u.conds.push_back(random_cond(r, c, d));
  return u;
}

int32_t tournament(Rng &r, const int32_t *fit, int32_t n, int32_t k) {
  int32_t best = -1;
  for (int32_t t = 0; t < k; ++t) {
    const int32_t i = r.below(n);
    if (best < 0 || fit[i] > fit[best] || (fit[i] == fit[best] && i < best)) best = i;
  }
  return best;
}

std::vector<Set> breed(Rng &r, const std::vector<Set> &pool, const int32_t *fit,
                       const aerl_evolve_cfg &c, const Ranges &d) {
  const int32_t n = (int32_t)pool.size();
  std::vector<int32_t> order(n);
  for (int32_t i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return fit[a] > fit[b]; });
  std::vector<Set> out;
  out.reserve(n);
  for (int32_t i = 0; i < c.elite; ++i) out.push_back(pool[order[i]]);
  for (int32_t i = c.elite; i < n; ++i) {
    Set child = pool[tournament(r, fit, n, c.tournament)];
    if (r.unit() < c.p_crossover) {
      const Set &b = pool[tournament(r, fit, n, c.tournament)];
      const int32_t ca = r.below((int32_t)child.rules.size() + 1);
      const int32_t cb = r.below((int32_t)b.rules.size() + 1);
      std::vector<Rule> merged(child.rules.begin(), child.rules.begin() + ca);
      merged.insert(merged.end(), b.rules.begin() + cb, b.rules.end());
      if (merged.empty()) merged.push_back(child.rules.front());
      if ((int32_t)merged.size() > c.max_rules) merged.resize(c.max_rules);
      child.rules = std::move(merged);
    }
    for (Rule &u : child.rules) {
      for (Cond &k : u.conds) {
        if (r.unit() < c.p_coef) {
          k.coef = r.unit();
          if (k.kind == 1)
            k.coef2 = r.unit();
          else
            k.theta = range_theta(r, d, k.f);
        }
      }
    }
    if (r.unit() < c.p_struct) {
      const int32_t t = r.below(4);
      const int32_t R = (int32_t)child.rules.size();
      if (t == 0) {
        Rule &u = child.rules[r.below(R)];
        if ((int32_t)u.conds.size() < c.max_conds) u.conds.push_back(random_cond(r, c, d));
      } else if (t == 1) {
        Rule &u = child.rules[r.below(R)];
        if (u.conds.size() >= 2) u.conds.erase(u.conds.begin() + r.below((int32_t)u.conds.size()));
      } else if (t == 2) {
        if (R < c.max_rules) {
          const int32_t pos = r.below(R + 1);
          Rule u = random_rule(r, c, d);
          child.rules.insert(child.rules.begin() + pos, std::move(u));
        }
      } else if (R >= 2) {
        child.rules.erase(child.rules.begin() + r.below(R));
      }
    }
    out.push_back(std::move(child));
  }
  return out;
}

std::vector<Set> random_pool(Rng &r, const aerl_evolve_cfg &c, const Ranges &d) {
  std::vector<Set> pool(c.pool);
  for (Set &s : pool) {
    const int32_t R = 1 + r.below(c.max_rules);
    s.dflt = r.below(d.nc);
    for (int32_t k = 0; k < R; ++k) {
      Rule u;
      const int32_t K = 1 + r.below(c.max_conds);
      u.cls = r.below(d.nc);
      for (int32_t j = 0; j < K; ++j) u.conds.push_back(random_cond(r, c, d));
      s.rules.push_back(std::move(u));
    }
  }
  return pool;
}

// ------------------------------------------------------------ SoA forms
struct Soa {
  std::vector<int32_t> set_rule_off, set_default, rule_cond_off, rule_class, f, g;
  std::vector<uint8_t> op, kind;
  std::vector<float> coef, coef2, theta;
  aerl_population view() const {
    aerl_population p{};
    p.n_sets = (int32_t)set_default.size();
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

Soa to_soa(const std::vector<Set> &pool) {
  Soa a;
  a.set_rule_off.push_back(0);
  a.rule_cond_off.push_back(0);
  for (const Set &s : pool) {
    a.set_default.push_back(s.dflt);
    for (const Rule &u : s.rules) {
      a.rule_class.push_back(u.cls);
      for (const Cond &k : u.conds) {
        a.op.push_back(k.op);
        a.kind.push_back(k.kind);
        a.f.push_back(k.f);
        a.g.push_back(k.g);
        a.coef.push_back(k.coef);
        a.coef2.push_back(k.coef2);
        a.theta.push_back(k.theta);
      }
      a.rule_cond_off.push_back((int32_t)a.op.size());
    }
    a.set_rule_off.push_back((int32_t)a.rule_class.size());
  }
  return a;
}

std::vector<Set> from_view(const aerl_population &p) {
  std::vector<Set> pool(p.n_sets);
  for (int32_t s = 0; s < p.n_sets; ++s) {
    pool[s].dflt = p.set_default[s];
    for (int32_t r = p.set_rule_off[s]; r < p.set_rule_off[s + 1]; ++r) {
      Rule u;
      u.cls = p.rule_class[r];
      for (int32_t j = p.rule_cond_off[r]; j < p.rule_cond_off[r + 1]; ++j) {
        Cond k{};
        k.op = p.op[j];
        k.kind = p.kind[j];
        k.f = p.f[j];
        k.g = k.kind ? p.g[j] : 0;
        k.coef = p.coef[j];
        k.coef2 = k.kind ? p.coef2[j] : 0.0f;
        k.theta = k.kind ? 0.0f : p.theta[j];
        u.conds.push_back(k);
      }
      pool[s].rules.push_back(std::move(u));
    }
  }
  return pool;
}

aerl_status write_out(const std::vector<Set> &pool, const aerl_evolve_cfg &c, aerl_population_out *o) {
  if (!o || !o->set_rule_off || !o->set_default || !o->rule_cond_off || !o->rule_class || !o->op ||
      !o->kind || !o->f || !o->g || !o->coef || !o->coef2 || !o->theta)
    return AERL_EINVAL;
  const Soa a = to_soa(pool);
  (void)c;  // capacities: pool + 1, pool, pool * max_rules + 1, pool * max_rules * max_conds
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
  o->n_sets = (int32_t)pool.size();
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
  std::vector<Set> pool;
  std::vector<int32_t> fitness;
  Soa soa;                       // the pool as last evaluated (state views point here)
  std::vector<float> tuned[3];   // tuned coef, coef2, theta of that pool
  char *arena = nullptr;
  size_t arena_bytes = 0;
  EvolveArena layout{};
  void *staging = nullptr;       // pinned host image of a packed pool
  double sec_eval = 0, sec_tune = 0, sec_breed = 0;
  ~Evo() {
    if (staging) (void)hipHostFree(staging);
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
  e.soa = to_soa(e.pool);
  aerl_population view = e.soa.view();
  const size_t nconds = e.soa.op.size();
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
    const float *src[3] = {e.soa.coef.data(), e.soa.coef2.data(), e.soa.theta.data()};
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
    e.fitness.resize(e.pool.size());
    hipError_t h = hipMemcpyAsync(e.fitness.data(), correct, e.pool.size() * 4, hipMemcpyDeviceToHost, st);
    if (h == hipSuccess) h = hipStreamSynchronize(st);
    if (h != hipSuccess) s = fail(ctx, AERL_EDEVICE, "fitness copy failed: %s", hipGetErrorString(h));
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
  const std::vector<Set> pool = random_pool(r, *cfg, Ranges{nf, nc, lo, hi});
  s = write_out(pool, *cfg, out);
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
  if (pool->n_sets != cfg->pool || check_kinds(nullptr, *pool, nk)) return AERL_EINVAL;
  const std::vector<Set> in = from_view(*pool);
  for (const Set &st : in) {
    if (st.rules.empty() || (int32_t)st.rules.size() > cfg->max_rules) return AERL_EINVAL;
    for (const Rule &u : st.rules)
      if (u.conds.empty() || (int32_t)u.conds.size() > cfg->max_conds) return AERL_EINVAL;
  }
  Rng r{*rng_state};
  const std::vector<Set> next = breed(r, in, fitness, *cfg, Ranges{nf, nc, lo, hi});
  s = write_out(next, *cfg, out);
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
    e->pool = from_view(*initial);
    for (const Set &st : e->pool) {
      if (st.rules.empty() || (int32_t)st.rules.size() > cfg->max_rules)
        return fail(ctx, AERL_EINVAL, "initial rule sets need 1..max_rules rules");
      for (const Rule &u : st.rules)
        if (u.conds.empty() || (int32_t)u.conds.size() > cfg->max_conds)
          return fail(ctx, AERL_EINVAL, "initial rules need 1..max_conds conditions");
    }
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
    e.pool = breed(e.rng, e.pool, e.fitness.data(), e.cfg, Ranges{e.nf, e.nc, e.lo.data(), e.hi.data()});
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
  out->pool = e.soa.view();
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
  const Soa &a = e.soa;
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
      (size_t)nr != a.rule_class.size() || (size_t)nk != a.op.size())
    return fail(ctx, AERL_EINVAL, "%s holds an invalid pool", path);
  e->pool = from_view(v);
  e->soa = std::move(a);
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
