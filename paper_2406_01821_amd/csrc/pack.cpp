// Population validation and packing (host side).
//
// The caller hands over rule sets in the paper's tensorized form, stored
// sparsely: each condition is a rule-tensor row with one weight and a bias
// (threshold) or two weights and zero bias (feature-vs-feature), Section 3
// and Fig. 1a.  The packed form regroups each rule's conditions (a rule is an
// AND, so their order never changes a result) and rewrites every condition
// exactly into one of three comparison forms the kernels evaluate:
//
//   threshold   a*x[f] > b        from  c*x op t:
//       >   a = c,  b = t
//       <   a = -c, b = -t                    (-fl(c*x) == fl(-c*x))
//       >=  a = c,  b = next_down(t)          (no float lies strictly between)
//       <=  a = -c, b = -next_up(t)
//       >= -inf and <= +inf always hold and become 0*x > -1.
//   feature     a*x[f] > b*x[g]   (> as is, < with both weights negated)
//               a*x[f] >= b*x[g]  (>= as is, <= with both weights negated)
//
// Products and comparisons are IEEE fp32 and never NaN for finite inputs, so
// each rewrite gives the caller's result bit for bit.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <thread>
#include <vector>

#include "internal.h"

namespace aerl {

namespace {

struct HostPacked {
  std::vector<int4> sets;
  std::vector<int4> rules;
  std::vector<uint4> hconds;
  std::vector<uint32_t> sconds;
};

uint32_t fbits(float v) {
  uint32_t u;
  std::memcpy(&u, &v, 4);
  return u;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Position of a non-NaN float in the order -inf < ... < -0 < +0 < ... < +inf.
int64_t fkey(float v) {
  const uint32_t u = fbits(v);
  return (u >> 31) ? -(int64_t)(u & 0x7fffffffu) - 1 : (int64_t)u;
}

float fkey_float(int64_t k) {
  const uint32_t u = k >= 0 ? (uint32_t)k : (0x80000000u | (uint32_t)(-(k + 1)));
  float v;
  std::memcpy(&v, &u, 4);
  return v;
}

// The product a*x (one fp32 rounding) against b.
bool passes(float a, float x, float b, bool strict) {
  const float p = a * x;
  return strict ? p > b : p >= b;
}

// Threshold folding.  For a > 0 and b not NaN, x -> fl(a*x) is monotone
// non-decreasing over the floats (rounding is monotone; -0 and +0 give equal
// products), so the x that pass form an upper interval of the order above.
// Returns its least element (NaN when no x passes), which turns the test
// into the single compare x >= t, exact for every x including +-inf and NaN.
// The least element is found next to b/a in almost every case (a few
// products, each answer checked against its neighbour below); otherwise by
// bisection over the order.
float fold_least(float a, float b, bool strict) {
  const float q = (float)((double)b / (double)a);
  if (std::isfinite(q)) {
    int64_t k = fkey(q);
    bool pk = passes(a, q, b, strict);
    for (int step = 0; step < 4; ++step) {
      if (pk) {  // k passes: the answer unless k-1 passes too
        if (!passes(a, fkey_float(k - 1), b, strict)) return fkey_float(k);
        --k;
      } else {  // k fails: the answer is k+1 if it passes
        ++k;
        pk = passes(a, fkey_float(k), b, strict);
        if (pk) return fkey_float(k);
      }
    }
  }
  if (!passes(a, INFINITY, b, strict)) return NAN;
  if (passes(a, -INFINITY, b, strict)) return -INFINITY;
  int64_t lo = fkey(-INFINITY), hi = fkey(INFINITY);  // lo fails, hi passes
  while (hi - lo > 1) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (passes(a, fkey_float(mid), b, strict)) hi = mid;
    else lo = mid;
  }
  return fkey_float(hi);
}

// Threshold record for coef*x[f] op theta: (y, z, flags).
void threshold_record(float c, float t, int op, float *y, float *z, uint32_t *flags) {
  // c*x > t, c*x >= t as they are; c*x < t as (-c)*x > -t (negation is exact)
  const bool strict = op == AERL_OP_GT || op == AERL_OP_LT;
  const bool neg = op == AERL_OP_LT || op == AERL_OP_LE;
  const float a = neg ? -c : c, b = neg ? -t : t;
  if (a > 0.0f) {
    *y = fold_least(a, b, strict);
    *z = b;
    *flags = 0;
  } else if (a < 0.0f) {
    // a*x = (-a)*(-x) exactly: the passing x form a lower interval
    *y = -fold_least(-a, b, strict);
    *z = b;
    *flags = kRecLE;
  } else {
    // zero coefficient: the product is +-0 for finite x and NaN otherwise;
    // >= b on those values is > the float below b (> -max for b = -inf)
    *y = a;
    *z = strict ? b : (b == -INFINITY ? -FLT_MAX : std::nextafter(b, -INFINITY));
    *flags = kRecMul;
  }
}

}  // namespace

PackedLayout packed_layout(int32_t n_sets, int32_t n_rules, int32_t n_conds) {
  // The hard stream holds one record per condition, one per empty rule and
  // one closing record per set; n_conds + n_rules + n_sets bounds it.  One
  // spare record keeps a read-ahead of the record after the last one inside
  // the buffer.
  PackedLayout L{};
  size_t off = 0;
  L.sets_off = off;
  off = align256(off + sizeof(int4) * (size_t)(n_sets > 0 ? n_sets : 1));
  L.ssets_off = off;
  off = align256(off + sizeof(int4) * (size_t)(n_sets > 0 ? n_sets : 1));
  L.rules_off = off;
  off = align256(off + sizeof(int4) * (size_t)(n_rules > 0 ? n_rules : 1));
  L.hconds_off = off;
  off = align256(off + sizeof(uint4) * ((size_t)n_conds + (size_t)n_rules + (size_t)std::max(n_sets, 0) + 1));
  L.sconds_off = off;
  off = align256(off + sizeof(uint32_t) * (size_t)(n_conds > 0 ? n_conds : 1));
  L.heads_off = off;
  off = align256(off + sizeof(uint4) * ((size_t)n_conds + (size_t)n_rules + (size_t)std::max(n_sets, 0) + 1));
  L.cmask_off = off;
  off = align256(off + sizeof(uint2) * (size_t)(n_conds > 0 ? n_conds : 1));
  L.total = off;
  return L;
}

// Host threads available (read once: the query reads a system file).
unsigned host_threads() {
  static const unsigned n = std::max(1u, std::thread::hardware_concurrency());
  return n;
}

// Runs fn(i) for i in [0, n) on up to n host threads (i = 0 on the caller).
template <class F>
void run_parts(int n, const F &fn) {
  std::vector<std::thread> th;
  th.reserve(n > 1 ? n - 1 : 0);
  for (int i = 1; i < n; ++i) {
    try {
      th.emplace_back(fn, i);
    } catch (...) {  // no thread to be had: this part runs here
      fn(i);
    }
  }
  fn(0);
  for (auto &t : th) t.join();
}

// Whether every condition in [j0, j1) is valid, without a message: the
// checks of the detailed pass below, branch-light, for the common case of
// a valid population.  Needs the op, kind, f, coef, g, coef2 and theta
// arrays (the caller checks them); cat_mask only where a condition is
// categorical.
bool conds_valid(const aerl_population *p, int32_t j0, int32_t j1, int32_t nf) {
  bool ok = true;
  for (int32_t j = j0; j < j1; ++j) {
    const uint32_t op = p->op[j], kind = p->kind[j], f = (uint32_t)p->f[j];
    bool c = op <= 3u && kind <= 2u && f < (uint32_t)nf;
    if (kind == AERL_KIND_FEATURE) {
      const uint32_t g = (uint32_t)p->g[j];
      c = c && g < (uint32_t)nf && g != f && std::isfinite(p->coef[j]) &&
          std::isfinite(p->coef2[j]);
    } else if (kind == AERL_KIND_CATEGORICAL) {
      c = c && p->cat_mask != nullptr;
    } else {
      c = c && std::isfinite(p->coef[j]) && !std::isnan(p->theta[j]);
    }
    ok = ok && c;
  }
  return ok;
}

// Validates pop; on success fills the counts.  Returns AERL_OK or AERL_EINVAL
// with the message in ctx (ctx may be null: then only the code is returned).
aerl_status validate_population(aerl_ctx *ctx, const aerl_population *p, int32_t nf, int32_t nc,
                                int32_t *n_rules_out, int32_t *n_conds_out) {
  if (!p) return fail(ctx, AERL_EINVAL, "population is NULL");
  if (nf < 1 || nf > AERL_MAX_FEATURES)
    return fail(ctx, AERL_EINVAL, "n_features %d outside [1, %d]", nf, AERL_MAX_FEATURES);
  if (nc < 1 || nc > AERL_MAX_CLASSES)
    return fail(ctx, AERL_EINVAL, "n_classes %d outside [1, %d]", nc, AERL_MAX_CLASSES);
  if (p->n_sets < 0) return fail(ctx, AERL_EINVAL, "n_sets %d < 0", p->n_sets);
  if (!p->set_rule_off) return fail(ctx, AERL_EINVAL, "set_rule_off is NULL");
  if (p->set_rule_off[0] != 0) return fail(ctx, AERL_EINVAL, "set_rule_off[0] != 0");
  if (p->n_sets > 0 && !p->set_default) return fail(ctx, AERL_EINVAL, "set_default is NULL");
  for (int32_t s = 0; s < p->n_sets; ++s) {
    if (p->set_rule_off[s + 1] < p->set_rule_off[s])
      return fail(ctx, AERL_EINVAL, "set_rule_off decreases at set %d", s);
    if (p->set_default[s] < 0 || p->set_default[s] >= nc)
      return fail(ctx, AERL_EINVAL, "set_default[%d] = %d outside [0, %d)", s, p->set_default[s], nc);
  }
  const int32_t n_rules = p->set_rule_off[p->n_sets];
  if (n_rules > 0 && (!p->rule_cond_off || !p->rule_class))
    return fail(ctx, AERL_EINVAL, "rule arrays are NULL");
  if (n_rules > 0 && p->rule_cond_off[0] != 0) return fail(ctx, AERL_EINVAL, "rule_cond_off[0] != 0");
  for (int32_t r = 0; r < n_rules; ++r) {
    const int32_t k = p->rule_cond_off[r + 1] - p->rule_cond_off[r];
    if (k < 0) return fail(ctx, AERL_EINVAL, "rule_cond_off decreases at rule %d", r);
    if (k > AERL_MAX_RULE_CONDS)
      return fail(ctx, AERL_EINVAL, "rule %d has %d conditions (max %d)", r, k, AERL_MAX_RULE_CONDS);
    if (p->rule_class[r] < 0 || p->rule_class[r] >= nc)
      return fail(ctx, AERL_EINVAL, "rule_class[%d] = %d outside [0, %d)", r, p->rule_class[r], nc);
  }
  const int32_t n_conds = n_rules > 0 ? p->rule_cond_off[n_rules] : 0;
  if (n_conds > 0 && (!p->op || !p->kind || !p->f || !p->coef))
    return fail(ctx, AERL_EINVAL, "condition arrays are NULL");
  // the conditions in parallel parts first; the detailed pass (the first
  // offending index and its message) only when some part finds a fault
  bool fast_ok = false;
  if (n_conds > 0 && p->g && p->coef2 && p->theta) {
    const unsigned hw = host_threads();
    const int parts = (int)std::min<int64_t>(std::min(hw, 8u), (int64_t)n_conds / 32768 + 1);
    std::vector<char> part_ok(parts, 0);
    run_parts(parts, [&](int i) {
      part_ok[i] = conds_valid(p, (int32_t)((int64_t)n_conds * i / parts),
                               (int32_t)((int64_t)n_conds * (i + 1) / parts), nf);
    });
    fast_ok = std::all_of(part_ok.begin(), part_ok.end(), [](char v) { return v != 0; });
  }
  for (int32_t j = 0; j < (fast_ok ? 0 : n_conds); ++j) {
    if (p->op[j] > 3) return fail(ctx, AERL_EINVAL, "op[%d] = %d is not an operator", j, p->op[j]);
    if (p->kind[j] > 2) return fail(ctx, AERL_EINVAL, "kind[%d] = %d is not a kind", j, p->kind[j]);
    if (p->f[j] < 0 || p->f[j] >= nf)
      return fail(ctx, AERL_EINVAL, "f[%d] = %d outside [0, %d)", j, p->f[j], nf);
    if (p->kind[j] == AERL_KIND_CATEGORICAL) {
      if (!p->cat_mask) return fail(ctx, AERL_EINVAL, "cat_mask is NULL with a categorical condition");
      continue;
    }
    if (!std::isfinite(p->coef[j])) return fail(ctx, AERL_EINVAL, "coef[%d] is not finite", j);
    if (p->kind[j] == AERL_KIND_FEATURE) {
      if (!p->g || !p->coef2) return fail(ctx, AERL_EINVAL, "g/coef2 arrays are NULL");
      if (p->g[j] < 0 || p->g[j] >= nf)
        return fail(ctx, AERL_EINVAL, "g[%d] = %d outside [0, %d)", j, p->g[j], nf);
      if (p->g[j] == p->f[j]) return fail(ctx, AERL_EINVAL, "g[%d] == f[%d]", j, j);
      if (!std::isfinite(p->coef2[j])) return fail(ctx, AERL_EINVAL, "coef2[%d] is not finite", j);
    } else {
      if (!p->theta) return fail(ctx, AERL_EINVAL, "theta array is NULL");
      if (std::isnan(p->theta[j])) return fail(ctx, AERL_EINVAL, "theta[%d] is NaN", j);
    }
  }
  for (int32_t s = 0; s < p->n_sets; ++s) {
    int32_t recs = 0;
    for (int32_t r = p->set_rule_off[s]; r < p->set_rule_off[s + 1]; ++r)
      recs += std::max(p->rule_cond_off[r + 1] - p->rule_cond_off[r], 1);
    if (recs + 1 > kMaxSetRecords)
      return fail(ctx, AERL_EINVAL, "rule set %d has %d conditions (+1 per empty rule); max %d", s,
                  recs, kMaxSetRecords - 1);
  }
  if (n_rules_out) *n_rules_out = n_rules;
  if (n_conds_out) *n_conds_out = n_conds;
  return AERL_OK;
}

namespace {

// Summary counts of a range of rule sets.
struct PackStats {
  int32_t max_rules = 0, max_rule_conds = 0, max_set_conds = 0;
  int64_t nominal = 0;
};

// Hard stream, head table and set records of rule sets [s0, s1), whose
// first records start at index first[s] (sets do not share records, so
// ranges of sets are packed independently).  For each rule set its rules in
// order, then a closing always-true record of the default class; inside a
// rule the folded >= thresholds first, then <=, zero coefficients,
// feature >, feature >= (an AND: the order changes no result).  An empty
// rule (always fires) becomes one always-true record.
void pack_sets(const aerl_population *p, const int32_t *first_of, int32_t s0, int32_t s1,
               int4 *sets, int4 *ssets, uint4 *hc, uint4 *heads, PackStats *st) {
  const uint32_t no_test = fbits(-INFINITY);
  int32_t max_rules = 0, max_rule_conds = 0;
  int64_t nominal = 0;
  for (int32_t s = s0; s < s1; ++s) {
    const int32_t r0 = p->set_rule_off[s], r1 = p->set_rule_off[s + 1];
    const int32_t nominal_s = r1 > r0 ? p->rule_cond_off[r1] - p->rule_cond_off[r0] : 0;
    const int32_t first = first_of[s];
    int32_t out = first;
    for (int32_t r = r0; r < r1; ++r) {
      const int32_t j0 = p->rule_cond_off[r], j1 = p->rule_cond_off[r + 1];
      const int32_t k = j1 - j0;
      if (k > max_rule_conds) max_rule_conds = k;
      const uint32_t cls = (uint32_t)p->rule_class[r] << kRecClsShift;
      const uint32_t next = (uint32_t)(out - first + std::max(k, 1)) * 16u << kRecNextShift;
      // the rule's head entry: its start, and the tile tests of its first
      // two records when they are folded thresholds (filled in below)
      uint4 &head = heads[first + (r - r0)];
      head = make_uint4((uint32_t)(out - first) * 16u, no_test, 0u, no_test);
      if (k == 0) {
        hc[out++] = make_uint4(0u, 0u, 0u, kRecAlways | kRecLast | cls | next);
        continue;
      }
      // groups: folded >=, folded <=, zero coefficient, feature >, feature >=,
      // categorical (the sign of the rewritten coefficient decides a
      // threshold's group); a stable counting sort puts the rule's conditions
      // in group order
      uint8_t grp_of[256], order[256];  // at most AERL_MAX_RULE_CONDS conditions
      int32_t start[7] = {0, 0, 0, 0, 0, 0, 0};
      for (int32_t j = j0; j < j1; ++j) {
        const int op = p->op[j];
        int g;
        if (p->kind[j] == AERL_KIND_CATEGORICAL) {
          g = 5;
        } else if (p->kind[j] == AERL_KIND_FEATURE) {
          g = (op == AERL_OP_GT || op == AERL_OP_LT) ? 3 : 4;
        } else {
          const float a0 = (op == AERL_OP_LT || op == AERL_OP_LE) ? -p->coef[j] : p->coef[j];
          g = a0 > 0.0f ? 0 : a0 < 0.0f ? 1 : 2;
        }
        grp_of[j - j0] = (uint8_t)g;
        ++start[g + 1];
      }
      for (int g = 0; g < 6; ++g) start[g + 1] += start[g];
      for (int32_t i = 0; i < k; ++i) order[start[grp_of[i]]++] = (uint8_t)i;
      int prev_grp = -1;
      for (int32_t pos = 0; pos < k; ++pos) {
        const int32_t j = j0 + order[pos];
        const int grp = grp_of[order[pos]];
        const int op = p->op[j];
        float a, b;
        uint32_t w = cls | next;
        uint32_t ya = 0, zb = 0;  // raw operand bits of a categorical record
        if (grp == 5) {
          const uint64_t mk = p->cat_mask[j];
          ya = (uint32_t)mk;
          zb = (uint32_t)(mk >> 32);
          a = b = 0.0f;
          w |= kRecCat;
        } else if (grp < 3) {
          uint32_t flags;
          threshold_record(p->coef[j], p->theta[j], op, &a, &b, &flags);
          if (grp == 1 && prev_grp != 1) flags |= kRecDirChg;
          w |= flags;
        } else {
          const bool neg = op == AERL_OP_LT || op == AERL_OP_LE;
          a = neg ? -p->coef[j] : p->coef[j];
          b = neg ? -p->coef2[j] : p->coef2[j];
          w |= (uint32_t)p->g[j] | kRecFF | (grp == 4 ? kRecGE : 0u);
        }
        prev_grp = grp;
        if (pos == k - 1) w |= kRecLast;
        if (pos < 2 && grp < 2) {
          const uint32_t e = 8u * (uint32_t)p->f[j] + (grp == 1 ? 4u : 0u);
          const uint32_t tt = fbits(grp == 1 ? -a : a);
          if (pos == 0) {
            head.x |= e << kHeadExtShift;
            head.y = tt;
          } else {
            head.z = e;
            head.w = tt;
          }
        }
        hc[out++] = make_uint4((uint32_t)p->f[j] * 1024u, grp == 5 ? ya : fbits(a),
                               grp == 5 ? zb : fbits(b), w);
      }
    }
    const uint32_t end = (uint32_t)(out - first + 1) * 16u << kRecNextShift;
    heads[first + (r1 - r0)] = make_uint4((uint32_t)(out - first) * 16u, no_test, 0u, no_test);
    // entries past the head count are never read; zero keeps the image exact
    for (int32_t e = first + (r1 - r0) + 1; e <= out; ++e) heads[e] = make_uint4(0u, 0u, 0u, 0u);
    hc[out++] = make_uint4(0u, 0u, 0u,
                           kRecAlways | kRecLast | (uint32_t)p->set_default[s] << kRecClsShift | end);
    sets[s] = make_int4(first, (out - first) | (r1 - r0 + 1) << 16, p->set_default[s], nominal_s);
    ssets[s] = make_int4(r0, r1 - r0, r1 > r0 ? p->rule_cond_off[r0] : 0, nominal_s);
    if (nominal_s > st->max_set_conds) st->max_set_conds = nominal_s;
    nominal += nominal_s;
    if (r1 - r0 > max_rules) max_rules = r1 - r0;
  }
  st->max_rules = std::max(st->max_rules, max_rules);
  st->max_rule_conds = std::max(st->max_rule_conds, max_rule_conds);
  st->nominal += nominal;
}

// Soft-path rule records and condition words of rules [q0, q1); counts the
// feature-vs-feature conditions among their conditions.
void pack_rules(const aerl_population *p, int32_t q0, int32_t q1, int4 *rules, uint32_t *sc,
                uint2 *cm, int32_t *n_ff, int32_t *n_cat) {
  int32_t ff = 0, cat = 0;
  for (int32_t r = q0; r < q1; ++r) {
    const int32_t j0 = p->rule_cond_off[r], j1 = p->rule_cond_off[r + 1];
    rules[r] = make_int4(j0, j1 - j0, p->rule_class[r], 0);
    for (int32_t j = j0; j < j1; ++j) {
      const bool is_ff = p->kind[j] == AERL_KIND_FEATURE;
      const bool is_cat = p->kind[j] == AERL_KIND_CATEGORICAL;
      const uint32_t g = is_ff ? (uint32_t)p->g[j] : 0u;
      sc[j] = (uint32_t)p->f[j] | (g << 12) | (is_ff ? kSoftFF : 0u) |
              ((uint32_t)(p->op[j] >= AERL_OP_GT) << 25) | (is_cat ? kSoftCat : 0u);
      const uint64_t mk = is_cat ? p->cat_mask[j] : 0u;
      cm[j] = make_uint2((uint32_t)mk, (uint32_t)(mk >> 32));
      ff += is_ff;
      cat += is_cat;
    }
  }
  *n_ff = ff;
  *n_cat = cat;
}


}  // namespace

// Writes the packed image of a validated population into `dst` (host memory
// of PackedLayout::total bytes) and fills the summary fields of `rec`.
// Large populations are packed by several host threads, each a range of
// rule sets (and of rules); the image does not depend on their number.
void pack_population_image(const aerl_population *p, int32_t nf, int32_t nc, int32_t n_rules,
                           int32_t n_conds, void *dst, PopRec *rec) {
  const PackedLayout L = packed_layout(p->n_sets, n_rules, n_conds);
  char *base = static_cast<char *>(dst);
  int4 *sets = reinterpret_cast<int4 *>(base + L.sets_off);
  int4 *ssets = reinterpret_cast<int4 *>(base + L.ssets_off);
  int4 *rules = reinterpret_cast<int4 *>(base + L.rules_off);
  uint4 *hc = reinterpret_cast<uint4 *>(base + L.hconds_off);
  uint32_t *sc = reinterpret_cast<uint32_t *>(base + L.sconds_off);
  uint4 *heads = reinterpret_cast<uint4 *>(base + L.heads_off);
  uint2 *cm = reinterpret_cast<uint2 *>(base + L.cmask_off);
  // first record of every rule set: one per condition, one per empty rule,
  // one closing record
  std::vector<int32_t> first(p->n_sets + 1);
  first[0] = 0;
  for (int32_t s = 0; s < p->n_sets; ++s) {
    int32_t recs = 1;
    for (int32_t r = p->set_rule_off[s]; r < p->set_rule_off[s + 1]; ++r)
      recs += std::max(p->rule_cond_off[r + 1] - p->rule_cond_off[r], 1);
    first[s + 1] = first[s] + recs;
  }
  const int32_t n_rec = first[p->n_sets];
  // bytes no part writes: the read-ahead pad record, the unused tails of the
  // regions and the alignment gaps between them
  const auto zero_tail = [&](size_t used_end, size_t region_end) {
    if (region_end > used_end) std::memset(base + used_end, 0, region_end - used_end);
  };
  zero_tail(L.sets_off + sizeof(int4) * (size_t)p->n_sets, L.ssets_off);
  zero_tail(L.ssets_off + sizeof(int4) * (size_t)p->n_sets, L.rules_off);
  zero_tail(L.rules_off + sizeof(int4) * (size_t)n_rules, L.hconds_off);
  zero_tail(L.hconds_off + sizeof(uint4) * (size_t)n_rec, L.sconds_off);
  zero_tail(L.sconds_off + sizeof(uint32_t) * (size_t)n_conds, L.heads_off);
  zero_tail(L.heads_off + sizeof(uint4) * (size_t)n_rec, L.cmask_off);
  zero_tail(L.cmask_off + sizeof(uint2) * (size_t)n_conds, L.total);
  // about 16k conditions per thread, at most 8 threads
  const unsigned hw = host_threads();
  const int parts = (int)std::max<int64_t>(
      1, std::min<int64_t>({(int64_t)std::min(hw, 8u), (int64_t)n_conds / 16384 + 1,
                            (int64_t)std::max(p->n_sets, 1)}));
  std::vector<PackStats> stats(parts);
  std::vector<int32_t> ffs(parts, 0), cats(parts, 0);
  run_parts(parts, [&](int i) {
    // sets split by records, rules by index
    const int64_t lo_rec = (int64_t)n_rec * i / parts, hi_rec = (int64_t)n_rec * (i + 1) / parts;
    const int32_t s0 = (int32_t)(std::lower_bound(first.begin(), first.end() - 1, (int32_t)lo_rec) - first.begin());
    const int32_t s1 = i + 1 == parts ? p->n_sets
        : (int32_t)(std::lower_bound(first.begin(), first.end() - 1, (int32_t)hi_rec) - first.begin());
    pack_sets(p, first.data(), s0, s1, sets, ssets, hc, heads, &stats[i]);
    const int32_t q0 = (int32_t)((int64_t)n_rules * i / parts);
    const int32_t q1 = (int32_t)((int64_t)n_rules * (i + 1) / parts);
    pack_rules(p, q0, q1, rules, sc, cm, &ffs[i], &cats[i]);
  });
  PackStats all;
  int32_t n_ff = 0, n_cat = 0;
  for (int i = 0; i < parts; ++i) {
    n_cat += cats[i];
    all.max_rules = std::max(all.max_rules, stats[i].max_rules);
    all.max_rule_conds = std::max(all.max_rule_conds, stats[i].max_rule_conds);
    all.max_set_conds = std::max(all.max_set_conds, stats[i].max_set_conds);
    all.nominal += stats[i].nominal;
    n_ff += ffs[i];
  }
  (void)nf;
  (void)nc;
  rec->max_set_conds = all.max_set_conds;
  rec->n_ff = n_ff;
  rec->n_cat = n_cat;
  rec->n_sets = p->n_sets;
  rec->n_rules = n_rules;
  rec->n_conds = n_conds;
  rec->nf = nf;
  rec->nc = nc;
  rec->max_rules = all.max_rules;
  rec->max_rule_conds = all.max_rule_conds;
  rec->nominal_conds = all.nominal;
}

}  // namespace aerl
