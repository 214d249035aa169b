// Host-only exercise of libaerl's CPU code (validation, multi-threaded
// packing, launch planning, the evolution loop's breeding) for sanitizer
// builds: built with AddressSanitizer + UndefinedBehaviorSanitizer or with
// ThreadSanitizer against a library whose host code carries the same
// instrumentation.  No GPU is touched.  Exits non-zero on any unexpected
// status; the sanitizers abort on any finding.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "aerl.h"

namespace {

struct Pop {
  std::vector<int32_t> set_rule_off{0}, set_default, rule_cond_off{0}, rule_class, f, g;
  std::vector<uint8_t> op, kind;
  std::vector<float> coef, coef2, theta;
  std::vector<uint64_t> mask;
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
    p.cat_mask = mask.data();
    return p;
  }
};

// Random population: rules 0..max_rules (empty rule sets and empty rules
// included), every kind, special coefficient values.
Pop random_pop(std::mt19937_64 &rng, int n_sets, int max_rules, int max_conds, int nf, int nc) {
  Pop p;
  auto u = [&](int n) { return (int)(rng() % (uint64_t)n); };
  const float specials[] = {0.0f, -0.0f, 1.0f, -1.0f, 1e-45f, 3e38f, 0.5f, -2.5f};
  for (int s = 0; s < n_sets; ++s) {
    p.set_default.push_back(u(nc));
    const int R = u(max_rules + 1);
    for (int r = 0; r < R; ++r) {
      p.rule_class.push_back(u(nc));
      const int K = u(max_conds + 1);
      for (int k = 0; k < K; ++k) {
        const int kind = nf >= 2 ? u(3) : (u(2) ? 2 : 0);
        const int f = u(nf);
        p.kind.push_back((uint8_t)kind);
        p.op.push_back((uint8_t)u(4));
        p.f.push_back(f);
        p.g.push_back(kind == 1 ? (f + 1 + u(nf - 1)) % nf : 0);
        p.coef.push_back(u(4) ? (float)(rng() % 1000) / 500.0f - 1.0f : specials[u(8)]);
        p.coef2.push_back((float)(rng() % 1000) / 700.0f);
        p.theta.push_back(u(8) ? (float)(rng() % 1000) / 100.0f : (u(2) ? INFINITY : -INFINITY));
        p.mask.push_back(rng());
      }
      p.rule_cond_off.push_back((int32_t)p.op.size());
    }
    p.set_rule_off.push_back((int32_t)p.rule_class.size());
  }
  return p;
}

int failures = 0;
void expect(bool ok, const char *what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what);
    ++failures;
  }
}

void pack_checks(std::mt19937_64 &rng) {
  // small and large populations (the large ones pack on several threads)
  for (int n_sets : {0, 1, 7, 300, 40000}) {
    const Pop p = random_pop(rng, n_sets, 6, 5, 9, 3);
    const aerl_population v = p.view();
    size_t bytes = 0;
    expect(aerl_population_bytes(&v, 9, 3, &bytes) == AERL_OK, "population_bytes");
    std::vector<unsigned char> img(bytes + 64, 0xcd);
    expect(aerl_pack_population_host(&v, 9, 3, img.data(), bytes) == AERL_OK, "pack");
    for (size_t i = bytes; i < img.size(); ++i) expect(img[i] == 0xcd, "pack wrote past its image");
    expect(aerl_pack_population_host(&v, 9, 3, img.data(), bytes - 1) == AERL_ENOMEM,
           "pack into a short buffer");
  }
  // invalid populations are refused, never read out of bounds
  Pop bad = random_pop(rng, 5, 3, 3, 4, 2);
  bad.op.push_back(9);  // stray entries past the offsets are never read
  aerl_population v = bad.view();
  v.rule_class = nullptr;
  size_t bytes = 0;
  expect(aerl_population_bytes(&v, 4, 2, &bytes) == AERL_EINVAL || bad.rule_class.empty(),
         "NULL rule_class refused");
  Pop f_out = random_pop(rng, 3, 2, 2, 4, 2);
  if (!f_out.f.empty()) {
    f_out.f[0] = 4;
    aerl_population w = f_out.view();
    expect(aerl_population_bytes(&w, 4, 2, &bytes) == AERL_EINVAL, "feature index refused");
  }
}

void plan_checks() {
  size_t b = 0;
  for (int nc : {1, 2, 64}) {
    const int64_t m = aerl_max_samples(nc);
    expect(aerl_dataset_bytes(m, 3, nc, &b) == AERL_OK, "dataset_bytes at the limit");
    expect(aerl_dataset_bytes(m + 1, 3, nc, &b) == AERL_EINVAL, "dataset_bytes past the limit");
  }
  const int64_t counts[4] = {(int64_t)1 << 24, 5, 1 << 20, 0};
  aerl_eval_launch L{};
  expect(aerl_eval_plan(counts, 4, 64, 4096, 256, &L) == AERL_OK, "eval_plan");
  expect(L.workgroups > 0 && L.tiles_per_group >= 1, "eval_plan output");
}

void breed_checks() {
  aerl_evolve_cfg c{};
  c.pool = 60;
  c.tournament = 3;
  c.elite = 2;
  c.max_rules = 7;
  c.max_conds = 4;
  c.ff_frac = 0.3f;
  c.p_crossover = 0.6f;
  c.p_coef = 0.3f;
  c.p_struct = 0.8f;
  const int nf = 6, nc = 3;
  std::vector<float> lo(nf, -1.0f), hi(nf, 2.0f);
  const size_t R = (size_t)c.pool * c.max_rules, K = R * c.max_conds;
  std::vector<int32_t> a(c.pool + 1), b(c.pool), d(R + 1), e(R), f(K), g(K);
  std::vector<uint8_t> op(K), kind(K);
  std::vector<float> c1(K), c2(K), th(K);
  aerl_population_out out{0, 0, 0, a.data(), b.data(), d.data(), e.data(), op.data(), kind.data(),
                          f.data(), g.data(), c1.data(), c2.data(), th.data()};
  uint64_t st = 42;
  expect(aerl_random_pool(&c, nf, nc, lo.data(), hi.data(), &st, &out) == AERL_OK, "random_pool");
  std::mt19937_64 rng(7);
  for (int gen = 0; gen < 50; ++gen) {
    aerl_population in{};
    in.n_sets = out.n_sets;
    std::vector<int32_t> a2(a.begin(), a.begin() + out.n_sets + 1), b2(b.begin(), b.begin() + out.n_sets),
        d2(d.begin(), d.begin() + out.n_rules + 1), e2(e.begin(), e.begin() + out.n_rules),
        f2(f.begin(), f.begin() + out.n_conds), g2(g.begin(), g.begin() + out.n_conds);
    std::vector<uint8_t> op2(op.begin(), op.begin() + out.n_conds), k2(kind.begin(), kind.begin() + out.n_conds);
    std::vector<float> c12(c1.begin(), c1.begin() + out.n_conds), c22(c2.begin(), c2.begin() + out.n_conds),
        th2(th.begin(), th.begin() + out.n_conds);
    in.set_rule_off = a2.data();
    in.set_default = b2.data();
    in.rule_cond_off = d2.data();
    in.rule_class = e2.data();
    in.op = op2.data();
    in.kind = k2.data();
    in.f = f2.data();
    in.g = g2.data();
    in.coef = c12.data();
    in.coef2 = c22.data();
    in.theta = th2.data();
    std::vector<int32_t> fit(c.pool);
    for (auto &x : fit) x = (int32_t)(rng() % 500);
    expect(aerl_breed(&in, fit.data(), &c, nf, nc, lo.data(), hi.data(), &st, &out) == AERL_OK, "breed");
  }
}

}  // namespace

int main() {
  std::mt19937_64 rng(2024);
  pack_checks(rng);
  plan_checks();
  breed_checks();
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("host driver: all checks passed\n");
  return 0;
}
