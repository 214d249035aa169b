// Soft (sigmoid-relaxed) forward pass and its adjoint.
//
// Section 3: a differentiable activation (a sigmoid) replaces the step so that
// rule coefficients and thresholds can be tuned by back-propagation.  The
// relaxation evaluated here (one sample, label y, rules k = 0..R-1):
//   z_j  = s_j * (coef_j * x[f_j] - rhs_j) / tau[f_j],  rhs = theta or coef2*x[g]
//   a_k  = sum_j log sigmoid(z_j)             (log of the rule's soft truth r_k)
//   b_k  = log(1 - r_k)
//   l_k  = a_k + sum_{m<k} b_m                (log P(rule k fires first))
//   log P_y = LSE({l_k : class_k = y} u {sum_m b_m if default = y})
//   L = min(-log P_y, 100),  loss = mean over samples.
// Everything is carried in log space in fp32 with accurate log1p / expm1 /
// log1mexp built from the hardware exp2/log2 (both within ~1 ulp, also near 1).
//
// Adjoint (derivation in the oracle): with V_k = P(class y | rules 0..k did not
// fire) = exp(U_k), U_{R-1} = [default = y] ? 0 : -inf,
// U_{k-1} = LSE([class_k = y] a_k, b_k + U_k):
//   dL/da_k = exp(l_k + U_k - log P_y)                      if class_k != y
//           = -exp(l_k - log P_y) * (1 - V_k)               if class_k == y
//   dL/dz_j = dL/da_k * sigmoid(-z_j),  formed as one exponent (bounded by 1).
// The backward kernel re-evaluates every condition: a forward sweep keeps only
// a_k and the survival prefix per rule and sample (in LDS), then a reverse
// sweep rebuilds U_k and recomputes each sigmoid to form its gradient.
//
// Work decomposition matches the hard path: block (chunk of rule sets, group
// of label-uniform tiles).  Per-(set, tile) wave sums go into LDS with one
// writer per entry; per-block partials go to the caller's workspace and a
// second kernel reduces them over groups in a fixed order, so every result is
// bit-identical from run to run.
#include "eval_core.h"
#include "internal.h"

namespace aerl {

namespace {

// Log-domain quantities inside the kernels are in bits (base-2 logs): the
// hardware computes 2^x (v_exp_f32) and log2(x) (v_log_f32) directly, so the
// inner loops carry no scaling multiplies.  A condition value is evaluated as
// z2 = z * log2(e); the loss is converted back to nats at the end.
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr float kNegInf = -__builtin_huge_valf();
constexpr float kLossCap = 100.0f;  // nats

__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float flog2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// log2(1 + u) for u in [0, 1]: w = 1 + u is rounded; (w - 1) - u is that
// rounding error exactly, which corrects log2(w) to first order.
__device__ __forceinline__ float log2_1p_unit(float u) {
  const float w = 1.0f + u;
  return fmaf(-((w - 1.0f) - u), kLog2e, flog2(w));
}

// Per-rule accumulator of the soft truth: a = log2 r = sum_j log2 sigmoid(z_j),
// and us = sum_j 2^(kShift2 - |z2_j|).  When every condition holds strongly,
// a is so close to 0 that fp32 cannot carry -a (it underflows near 2^-126),
// yet log(1 - r) ~ log(sum_j e^-z_j) still matters down to the loss clamp
// (e^-100); the shifted sum keeps it (normal floats down to z ~ 150).  The
// shift is a power of two, so unscaling it is exact.
constexpr float kShift2 = 92.0f;
constexpr float kExp2NegShift = 0x1p-92f;
struct RuleAcc {
  float a = 0.0f, us = 0.0f;
  // Adds condition value z2; returns log2(1 + 2^-|z2|), from which
  // -log2 sigmoid(+-z) = max(-+z2, 0) + that.
  __device__ __forceinline__ float add(float z2) {
    const float e_s = fexp2(kShift2 - fabsf(z2));
    const float lp = log2_1p_unit(e_s * kExp2NegShift);
    a -= fmaxf(-z2, 0.0f) + lp;
    us += e_s;
    return lp;
  }
  // add's return value for z2, without adding the condition
  __device__ static __forceinline__ float term(float z2) {
    return log2_1p_unit(fexp2(kShift2 - fabsf(z2)) * kExp2NegShift);
  }
};

// 1 - 2^a for a <= 0 (bits).  Near 0 uses Kahan's form of expm1,
// 2^a - 1 = (u - 1) * a / log2(u) with u = 2^a, which cancels the rounding
// of u.
__device__ __forceinline__ float one_minus_exp2(float a) {
  const float u = fexp2(a);
  if (a > -1.0f) {
    const float lu = flog2(u);
    const float em1 = (u == 1.0f) ? a * kLn2 : (u - 1.0f) * (a * frcp(lu));
    return -em1;
  }
  return 1.0f - u;
}

// log2(1 - 2^a) for a <= 0 (a = 0 gives -inf).
__device__ __forceinline__ float log1mexp2(float a) { return flog2(one_minus_exp2(a)); }

// log2(1 - r) of a rule: from a while fp32 represents -a well, otherwise from
// the shifted sum (there 1 - r = sum_j e^-z_j to within a relative 1e-30).
__device__ __forceinline__ float rule_log_miss(const RuleAcc &r) {
  return r.a > -1e-30f ? flog2(r.us) - kShift2 : log1mexp2(r.a);
}

// log2(2^p + 2^q), -inf safe.
__device__ __forceinline__ float lse(float p, float q) {
  float m;  // fmaxf(p, q); p and q are never NaN, so no canonicalizing copies
  asm("v_max_f32 %0, %1, %2" : "=v"(m) : "v"(p), "v"(q));
  if (m == kNegInf) return kNegInf;
  return m + log2_1p_unit(fexp2(-fabsf(p - q)));
}

// Interface shared by the two accumulators below:
//   add(z2)                 adds a condition, returns a per-condition value t
//   sig_neg(pre, z2, t)     2^pre * sigmoid(-z) for that condition
//   finish(a2, b2)          a2 = log2 r, b2 = log2(1 - r) of the rule
__device__ __forceinline__ void acc_finish(const RuleAcc &r, float &a2, float &b2) {
  a2 = r.a;
  b2 = rule_log_miss(r);
}
__device__ __forceinline__ float acc_log_r(const RuleAcc &r) { return r.a; }
__device__ __forceinline__ float acc_sig_neg(const RuleAcc &, float pre, float z2, float lp) {
  return fexp2(pre - (fmaxf(z2, 0.0f) + lp));
}

// log2(1 + p) for any p >= 0 (first-order correction of the rounding of
// w = 1 + p, as in log2_1p_unit).
__device__ __forceinline__ float log2_1p(float p) {
  const float w = 1.0f + p;
  return fmaf(-((w - 1.0f) - p) * frcp(w), kLog2e, flog2(w));
}

// Product form of a rule's soft truth, for rules of at most kProdMaxConds
// conditions.  With u_j = e^-|z_j| and M = sum_j max(-z_j, 0),
//   r = e^-M / prod_j (1 + u_j),  p = prod_j (1 + u_j) - 1 >= 0,
//   log r = -M - log1p(p),  1 - r = (p + (1 - e^-M)) / (1 + p),
// and p is built by p <- p (1 + u) + u from non-negative terms (1 + u
// rounded once), so it keeps full relative accuracy (also when r is within
// e^-100 of 1) with one exponential per condition; the logarithms are taken
// once per rule.  p is
// kept scaled by 2^64 (pt), so that u down to 2^-190 stays a normal float;
// with at most 60 conditions pt < 2^124.
constexpr int kProdMaxConds = 60;
// min(v, 0) in one v_min_f32.  fminf on a value the compiler cannot prove
// canonical (here a product carried across the wave reductions' branches)
// gets a canonicalizing copy first; no signaling NaN reaches this point, so
// the copy changes nothing and is left out.
__device__ __forceinline__ float min0(float v) {
  float r;
  asm("v_min_f32 %0, 0, %1" : "=v"(r) : "v"(v));
  return r;
}

struct RuleProd {
  float m = 0.0f, pt = 0.0f;  // m = M in bits, pt = p * 2^64
  // returns 1 + u, rounded once
  __device__ __forceinline__ float add(float z2) {
    const float ut = fexp2(64.0f - fabsf(z2));  // u * 2^64
    const float w = fmaf(ut, 0x1p-64f, 1.0f);
    // p' = p (1 + u) + u: rounding 1 + u first moves the product by at most
    // one rounding of it (a term of p' that is at least p), so p' keeps the
    // accuracy of two roundings while sharing 1 + u with the sigmoid
    pt = fmaf(pt, w, ut);
    m -= min0(z2);  // m += max(-z2, 0), the same value bit for bit
    return w;
  }
  // add's return value for z2, without adding the condition
  __device__ static __forceinline__ float term(float z2) {
    return fmaf(fexp2(64.0f - fabsf(z2)), 0x1p-64f, 1.0f);
  }
};
// log2(x * 2^-64) for x >= 0, from the exact exponent and the mantissa, so
// that a result near -64 carries no rounding of 64.
__device__ __forceinline__ float log2_scaled64(float x) {
  const float mant = __builtin_amdgcn_frexp_mantf(x);  // [0.5, 1), or 0
  const int e = __builtin_amdgcn_frexp_expf(x);
  return flog2(mant) + (float)(e - 64);
}

// a2 = log2 r = -M - log2(1 + p) is accurate in every regime.  b2 = log2(1 - r)
// follows from a2 while r is not within 2^-60 of 1; closer than that, from
// 1 - r = (p + (1 - e^-M)) / (1 + p) with p kept scaled (p may be far below
// the normal range there).
__device__ __forceinline__ void acc_finish(const RuleProd &r, float &a2, float &b2) {
  const float l1p = log2_1p(r.pt * 0x1p-64f);
  a2 = -r.m - l1p;
  b2 = a2 > -0x1p-60f ? log2_scaled64(fmaf(one_minus_exp2(-r.m), 0x1p64f, r.pt)) - l1p
                       : log1mexp2(a2);
}
// a2 alone, the same value as acc_finish's
__device__ __forceinline__ float acc_log_r(const RuleProd &r) {
  return -r.m - log2_1p(r.pt * 0x1p-64f);
}
__device__ __forceinline__ float acc_sig_neg(const RuleProd &, float pre, float z2, float w) {
  return fexp2(pre - fmaxf(z2, 0.0f)) * frcp(w);
}

// Loss of one sample in nats from log2 P_y.
__device__ __forceinline__ float sample_loss(float logpy2) { return fminf(-logpy2 * kLn2, kLossCap); }

// Sum of v over the wave, left in lane 63: an inclusive scan inside each
// 16-lane row (row_shr 1, 2, 4, 8), then the row totals carried forward
// with row_bcast 15 and 31.  A fixed order, so bit-identical from run to run.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v) {
  return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, true));
}
__device__ __forceinline__ float wave_total_last(float v) {
  v = dpp_add<0x111, 0xf>(v);
  v = dpp_add<0x112, 0xf>(v);
  v = dpp_add<0x114, 0xf>(v);
  v = dpp_add<0x118, 0xf>(v);
  v = dpp_add<0x142, 0xa>(v);
  v = dpp_add<0x143, 0xc>(v);
  return v;
}

// Wave totals of four values at once, each ending in lane 15 of one row:
// row 0 the total of a0, row 1 of b0, row 2 of a1, row 3 of b1.  The
// half-wave swaps pair lane l with l + 32 (a0 with a1, b0 with b1 in the two
// halves), then rows with the row 16 lanes on; an inclusive scan in each
// row finishes.  A fixed order, so bit-identical from run to run.
__device__ __forceinline__ float wave_totals4(float a0, float a1, float b0, float b1) {
  const auto sa = __builtin_amdgcn_permlane32_swap(__float_as_uint(a0), __float_as_uint(a1), false, false);
  const auto sb = __builtin_amdgcn_permlane32_swap(__float_as_uint(b0), __float_as_uint(b1), false, false);
  // lanes 0-31: a0 (b0) over lanes l and l + 32; lanes 32-63: a1 (b1)
  const float pa = __uint_as_float(sa[0]) + __uint_as_float(sa[1]);
  const float pb = __uint_as_float(sb[0]) + __uint_as_float(sb[1]);
  const auto sr = __builtin_amdgcn_permlane16_swap(__float_as_uint(pa), __float_as_uint(pb), false, false);
  // rows 0 and 2: pa over a row and the next; rows 1 and 3: pb
  float v = __uint_as_float(sr[0]) + __uint_as_float(sr[1]);
  v = dpp_add<0x111, 0xf>(v);
  v = dpp_add<0x112, 0xf>(v);
  v = dpp_add<0x114, 0xf>(v);
  v = dpp_add<0x118, 0xf>(v);
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

struct SoftArgs {
  const float *x_fm;
  int64_t n_pad;
  int32_t nf, nc;
  const int32_t *tile_info;
  const float *inv_tau;
  const int4 *sets;   // hard set records (default class in .z)
  const int4 *ssets;  // {first rule, #rules, first condition, #conditions}
  const int4 *rules;  // {first condition, #conditions, class, 0}
  const uint32_t *sconds;
  const float *coef, *coef2, *theta;
  // per condition {sconds, coef, theta or coef2, +-log2(e)/tau_f}, gathered
  // once per launch so that a condition is one scalar load
  const uint4 *crec;
  int32_t n_sets;
  int32_t sets_per_chunk, tiles_per_group, n_groups;
  int32_t max_rules, max_set_conds;
  double *part_loss;  // [n_groups][n_sets]
  float *part_grad;   // [n_groups][n_conds][2]
  int32_t n_conds;
  int32_t region_tile0[AERL_MAX_CLASSES];
  int32_t region_tiles[AERL_MAX_CLASSES];
};

// Class region and tile range of block group g (uniform).
__device__ __forceinline__ void group_range(const SoftArgs &a, int g, int &label, int &lo, int &hi) {
  label = 0; lo = 0; hi = 0;
  for (int c = 0; c < a.nc; ++c) {
    const int ng = (a.region_tiles[c] + a.tiles_per_group - 1) / a.tiles_per_group;
    if (g < ng) {
      label = c;
      lo = a.region_tile0[c] + g * a.tiles_per_group;
      hi = min(lo + a.tiles_per_group, a.region_tile0[c] + a.region_tiles[c]);
      return;
    }
    g -= ng;
  }
}

// A categorical condition has no parameter to relax: its soft truth is its
// truth, z = +inf (x[f] is a code k in 0..63 with bit k of the mask {lo, hi}
// set) or -inf.
__device__ __forceinline__ float cat_z(float v, uint32_t lo, uint32_t hi) {
  const bool ok = v >= 0.0f && v <= 63.0f && v == truncf(v);  // NaN fails
  const int code = ok ? (int)v : 0;
  const uint32_t word = code < 32 ? lo : hi;
  const bool in = ok && ((word >> (code & 31)) & 1u) != 0u;
  return in ? __builtin_huge_valf() : -__builtin_huge_valf();
}

// z2 = z*log2(e) of condition j for S values of x[f], with x[f] and the
// right-hand factor xg: x[g] for feature conditions, 1 for threshold ones (so
// dz*xg is their theta term).  Branch-free on the kind (the row of g is read
// for threshold conditions too; g is 0 there), which keeps every array in
// registers.
template <int S>
__device__ __forceinline__ void cond_z(const SoftArgs &a, const float *xs, int lane, int j,
                                       float (&z)[S], float (&xf)[S], float (&xg)[S], bool &ff) {
  const uint4 r = ldc(a.crec, j);
  const uint32_t sc = r.x;
  const uint32_t f = sc & 0xfffu, g = (sc >> 12) & 0xfffu;
  ff = (sc & kSoftFF) != 0;
  const float c = __uint_as_float(r.y), rv = __uint_as_float(r.z), sinv = __uint_as_float(r.w);
  load_row<S>(xs, f * 1024u, lane, xf);
  load_row<S>(xs, g * 1024u, lane, xg);
  if (sc & kSoftCat) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      z[s] = cat_z(xf[s], r.y, r.z);
      xg[s] = 1.0f;
    }
    return;
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const float rhs = ff ? rv * xg[s] : rv;
    xg[s] = ff ? xg[s] : 1.0f;
    z[s] = fmaf(c, xf[s], -rhs) * sinv;
  }
}

// Threshold-only populations: z2 and x[f] (xg is 1).
template <int S>
__device__ __forceinline__ void cond_z_t(const SoftArgs &a, const float *xs, int lane, int j,
                                         float (&z)[S], float (&xf)[S], float (&xg)[S]) {
  const uint4 r = ldc(a.crec, j);
  const uint32_t f = r.x & 0xfffu;
  const float c = __uint_as_float(r.y), th = __uint_as_float(r.z), sinv = __uint_as_float(r.w);
  load_row<S>(xs, f * 1024u, lane, xf);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    z[s] = fmaf(c, xf[s], -th) * sinv;
    xg[s] = 1.0f;
  }
}

// z2 only (forward pass): nothing but z leaves the branch on the kind.
template <int S>
__device__ __forceinline__ void cond_z_only(const SoftArgs &a, const float *xs, int lane, int j,
                                            float (&z)[S]) {
  const uint4 r = ldc(a.crec, j);
  const uint32_t sc = r.x;
  const uint32_t f = sc & 0xfffu, g = (sc >> 12) & 0xfffu;
  const float c = __uint_as_float(r.y), rv = __uint_as_float(r.z), sinv = __uint_as_float(r.w);
  float xf[S];
  load_row<S>(xs, f * 1024u, lane, xf);
  if (sc & kSoftFF) {
    float xg[S];
    load_row<S>(xs, g * 1024u, lane, xg);
#pragma unroll
    for (int s = 0; s < S; ++s) z[s] = fmaf(c, xf[s], -(rv * xg[s])) * sinv;
  } else if (sc & kSoftCat) {
#pragma unroll
    for (int s = 0; s < S; ++s) z[s] = cat_z(xf[s], r.y, r.z);
  } else {
#pragma unroll
    for (int s = 0; s < S; ++s) z[s] = fmaf(c, xf[s], -rv) * sinv;
  }
}

// z2 of conditions j .. j+3 (forward pass): the four records in one 64-byte
// scalar load and the four x[f] rows requested together, so that their
// latencies overlap; the same arithmetic as cond_z_only.  TONLY: threshold
// conditions only.
template <int S, bool TONLY>
__device__ __forceinline__ void cond_z4(const SoftArgs &a, const float *xs, int lane, int j,
                                        float (&z)[4][S]) {
  typedef uint32_t v16u __attribute__((ext_vector_type(16)));
  typedef const __attribute__((address_space(4))) v16u *cptr;
  const v16u r = *(cptr)(a.crec + j);
  float xf[4][S];
#pragma unroll
  for (int k = 0; k < 4; ++k) load_row<S>(xs, (r[4 * k] & 0xfffu) * 1024u, lane, xf[k]);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t sc = r[4 * k];
    const float c = __uint_as_float(r[4 * k + 1]), rv = __uint_as_float(r[4 * k + 2]);
    const float sinv = __uint_as_float(r[4 * k + 3]);
    if (!TONLY && (sc & kSoftFF)) {
      float xg[S];
      load_row<S>(xs, ((sc >> 12) & 0xfffu) * 1024u, lane, xg);
#pragma unroll
      for (int s = 0; s < S; ++s) z[k][s] = fmaf(c, xf[k][s], -(rv * xg[s])) * sinv;
    } else if (!TONLY && (sc & kSoftCat)) {
#pragma unroll
      for (int s = 0; s < S; ++s) z[k][s] = cat_z(xf[k][s], r[4 * k + 1], r[4 * k + 2]);
    } else {
#pragma unroll
      for (int s = 0; s < S; ++s) z[k][s] = fmaf(c, xf[k][s], -rv) * sinv;
    }
  }
}

// Gathers the per-condition record read by the kernels above: the operand of
// the right-hand side is theta for a threshold and coef2 for a
// feature-vs-feature condition; sinv = +-log2(e)/tau_f by direction.
__global__ void k_soft_prep(const uint32_t *__restrict__ sconds, const float *__restrict__ inv_tau,
                            const float *__restrict__ coef, const float *__restrict__ coef2,
                            const float *__restrict__ theta, const uint2 *__restrict__ cmask,
                            int32_t n_conds, uint4 *__restrict__ crec) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_conds) return;
  const uint32_t sc = sconds[j];
  if (sc & kSoftCat) {  // the code set replaces the parameters
    const uint2 m = cmask[j];
    crec[j] = make_uint4(sc, m.x, m.y, 0u);
    return;
  }
  const float inv = inv_tau[sc & 0xfffu] * kLog2e;
  const float sinv = ((sc >> 25) & 1u) ? inv : -inv;
  const float rv = ((sc >> 24) & 1u) ? coef2[j] : theta[j];
  crec[j] = make_uint4(sc, __float_as_uint(coef[j]), __float_as_uint(rv), __float_as_uint(sinv));
}

constexpr int kSoftBlock = 512;

// ------------------------------------------------------------------ forward
template <int S, class Acc, bool TONLY>
__global__ __launch_bounds__(kSoftBlock) void k_soft_fwd(const SoftArgs a) {
  constexpr int TS = 64 * S, WPT = AERL_TILE / TS;
  extern __shared__ __align__(16) float smem[];
  float *xs = smem;
  double *acc = reinterpret_cast<double *>(smem + (size_t)a.nf * TS);  // [Q]
  __shared__ int32_t next_q;
  const int lane = threadIdx.x & 63;
  int label, tile_lo, tile_hi;
  group_range(a, blockIdx.y, label, tile_lo, tile_hi);
  const int q0 = blockIdx.x * a.sets_per_chunk;
  const int Q = min(a.sets_per_chunk, a.n_sets - q0);
  for (int i = threadIdx.x; i < Q; i += blockDim.x) acc[i] = 0.0;
  const int n4 = a.nf * (TS / 4);
  const float4 *src = reinterpret_cast<const float4 *>(a.x_fm);
  float4 *dst = reinterpret_cast<float4 *>(xs);
  const int64_t row4 = a.n_pad / 4;
  for (int64_t wt = (int64_t)tile_lo * WPT; wt < (int64_t)tile_hi * WPT; ++wt) {
    __syncthreads();
    const int64_t base4 = wt * (TS / 4);
    for (int i = threadIdx.x; i < n4; i += blockDim.x) {
      const int f = i / (TS / 4), k = i % (TS / 4);
      dst[i] = src[(int64_t)f * row4 + base4 + k];
    }
    if (threadIdx.x == 0) next_q = 0;
    __syncthreads();
    const int info = ldc(a.tile_info, wt / WPT);
    const int valid = min(max((info >> 8) - (int)(wt % WPT) * TS, 0), TS);
    bool live[S];
#pragma unroll
    for (int s = 0; s < S; ++s) live[s] = lane * S + s < valid;
    for (;;) {
      const int q = next_item(&next_q);
      if (q >= Q) break;
      const int4 ss = ldc(a.ssets, q0 + q);
      const int dflt = ldc(a.sets, q0 + q).z;
      float logpy[S], surv[S];
#pragma unroll
      for (int s = 0; s < S; ++s) { logpy[s] = kNegInf; surv[s] = 0.0f; }
      // each rule's record is requested one rule ahead (the last one twice)
      int4 r_next = ldc(a.rules, ss.x);
      for (int k = 0; k < ss.y; ++k) {
        const int4 r = r_next;
        r_next = ldc(a.rules, ss.x + min(k + 1, ss.y - 1));
        Acc ra[S];
        // conditions four at a time, then one at a time (same order)
        int j = r.x;
        const int je = r.x + r.y;
        for (; j + 4 <= je; j += 4) {
          float z[4][S];
          cond_z4<S, TONLY>(a, xs, lane, j, z);
#pragma unroll
          for (int c4 = 0; c4 < 4; ++c4) {
#pragma unroll
            for (int s = 0; s < S; ++s) (void)ra[s].add(z[c4][s]);
          }
        }
        for (; j < je; ++j) {
          float z[S];
          cond_z_only<S>(a, xs, lane, j, z);
#pragma unroll
          for (int s = 0; s < S; ++s) (void)ra[s].add(z[s]);
        }
        const bool hit = r.z == label;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          float a2, b2;
          acc_finish(ra[s], a2, b2);
          if (hit) logpy[s] = lse(logpy[s], a2 + surv[s]);
          surv[s] += b2;
        }
      }
      float part = 0.0f;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const float lp = dflt == label ? lse(logpy[s], surv[s]) : logpy[s];
        part += live[s] ? sample_loss(lp) : 0.0f;
      }
      part = wave_sum(part);
      if (lane == 0) acc[q] += (double)part;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < Q; i += blockDim.x)
    a.part_loss[(int64_t)blockIdx.y * a.n_sets + q0 + i] = acc[i];
}

// Mean loss per rule set from the per-group partial sums: block b takes
// sets 64b .. 64b+63 (lane: set, so a wave reads 512 contiguous bytes per
// group), wave w the groups w, w+16, ...; the 16 wave sums are then added
// in wave order (a fixed order: the result does not depend on timing).
constexpr int kFwdFinalWaves = 16;
__global__ __launch_bounds__(kFwdFinalWaves * 64) void k_soft_fwd_final(
    const double *__restrict__ part, int32_t n_groups, int32_t n_sets, int64_t n,
    float *__restrict__ loss) {
  __shared__ double acc[kFwdFinalWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int p = blockIdx.x * 64 + lane;
  double s = 0.0;
  if (p < n_sets)
    for (int g = w; g < n_groups; g += kFwdFinalWaves) s += part[(int64_t)g * n_sets + p];
  acc[w][lane] = s;
  __syncthreads();
  if (w == 0 && p < n_sets) {
    double t = 0.0;
    for (int k = 0; k < kFwdFinalWaves; ++k) t += acc[k][lane];
    loss[p] = n > 0 ? (float)(t / (double)n) : 0.0f;
  }
}

// ----------------------------------------------------------------- backward
// Waves per block of the LDS-state adjoint kernels: up to kBwdWaves, fewer
// for rule sets whose per-wave state ([R][2][64] floats) would not fit.
constexpr int kBwdWaves = 8;

__global__ __launch_bounds__(kBwdWaves * 64) void k_soft_bwd(const SoftArgs a) {
  constexpr int TS = 64, WPT = AERL_TILE / TS;
  extern __shared__ __align__(16) float smem[];
  float *xs = smem;                                     // [nf][64]
  float *acc = xs + (size_t)a.nf * TS;                  // [Q][max_set_conds][2]
  float *store = acc + (size_t)a.sets_per_chunk * a.max_set_conds * 2;  // [wave][R][2][64]
  __shared__ int32_t next_q;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float *my = store + (size_t)wave * a.max_rules * 128;
  int label, tile_lo, tile_hi;
  group_range(a, blockIdx.y, label, tile_lo, tile_hi);
  const int q0 = blockIdx.x * a.sets_per_chunk;
  const int Q = min(a.sets_per_chunk, a.n_sets - q0);
  for (int i = threadIdx.x; i < Q * a.max_set_conds * 2; i += blockDim.x) acc[i] = 0.0f;
  const int n4 = a.nf * (TS / 4);
  const float4 *src = reinterpret_cast<const float4 *>(a.x_fm);
  float4 *dst = reinterpret_cast<float4 *>(xs);
  const int64_t row4 = a.n_pad / 4;
  for (int64_t wt = (int64_t)tile_lo * WPT; wt < (int64_t)tile_hi * WPT; ++wt) {
    __syncthreads();
    const int64_t base4 = wt * (TS / 4);
    for (int i = threadIdx.x; i < n4; i += blockDim.x) {
      const int f = i / (TS / 4), k = i % (TS / 4);
      dst[i] = src[(int64_t)f * row4 + base4 + k];
    }
    if (threadIdx.x == 0) next_q = 0;
    __syncthreads();
    const int info = ldc(a.tile_info, wt / WPT);
    const int valid = min(max((info >> 8) - (int)(wt % WPT) * TS, 0), TS);
    const bool live = lane < valid;
    for (;;) {
      const int q = next_item(&next_q);
      if (q >= Q) break;
      const int4 ss = ldc(a.ssets, q0 + q);
      const int dflt = ldc(a.sets, q0 + q).z;
      // forward sweep: keep a_k and the survival prefix before rule k
      float logpy = kNegInf, surv = 0.0f;
      for (int k = 0; k < ss.y; ++k) {
        const int4 r = ldc(a.rules, ss.x + k);
        RuleAcc ra;
        for (int j = r.x; j < r.x + r.y; ++j) {
          float z[1];
          cond_z_only<1>(a, xs, lane, j, z);
          ra.add(z[0]);
        }
        my[k * 128 + lane] = ra.a;
        my[k * 128 + 64 + lane] = surv;
        if (r.z == label) logpy = lse(logpy, ra.a + surv);
        surv += rule_log_miss(ra);
      }
      if (dflt == label) logpy = lse(logpy, surv);
      // samples whose loss is clamped (or padding) get no gradient; their
      // log P_y is replaced by 0 so that every exponent below stays finite
      const bool on = live && -logpy * kLn2 <= kLossCap;
      const float gate = on ? 1.0f : 0.0f;
      const float lpy = on ? logpy : 0.0f;
      // reverse sweep
      float U = dflt == label ? 0.0f : kNegInf;
      for (int k = ss.y - 1; k >= 0; --k) {
        const int4 r = ldc(a.rules, ss.x + k);
        const float ak = my[k * 128 + lane];
        const float lk = ak + my[k * 128 + 64 + lane];
        const bool hit = r.z == label;
        float pre, mul;
        if (hit) {
          pre = lk - lpy;
          mul = -one_minus_exp2(U) * gate;
        } else {
          pre = lk + U - lpy;
          mul = gate;
        }
        RuleAcc ra;
        for (int j = r.x; j < r.x + r.y; ++j) {
          float z[1], xf[1], xg[1];
          bool ff;
          cond_z<1>(a, xs, lane, j, z, xf, xg, ff);
          const float lp = ra.add(z[0]);
          // dL/dz = dL/da_k * sigmoid(-z), one exponent in bits
          const float dz = mul * fexp2(pre - (fmaxf(z[0], 0.0f) + lp));
          const float g0 = wave_sum(dz * xg[0]);
          const float g1 = wave_sum(dz * xf[0]);
          if (lane == 0) {
            float *ap = acc + ((size_t)q * a.max_set_conds + (j - ss.z)) * 2;
            ap[0] += g0;
            ap[1] += g1;
          }
        }
        U = lse(hit ? ak : kNegInf, rule_log_miss(ra) + U);
      }
    }
  }
  __syncthreads();
  for (int q = 0; q < Q; ++q) {
    const int4 ss = ldc(a.ssets, q0 + q);
    for (int i = threadIdx.x; i < ss.w * 2; i += blockDim.x)
      a.part_grad[((int64_t)blockIdx.y * a.n_conds + ss.z) * 2 + i] =
          acc[(size_t)q * a.max_set_conds * 2 + i];
  }
}

// Adjoint for rule sets of at most RMAX rules with S samples per lane: the
// per-rule state kept between the two sweeps is l_k = a_k + (survival
// before k) and log2(1 - r_k), two RMAX x S arrays of floats per lane, read
// and written through a uniform branch chain on k; at the 64-VGPR budget of
// eight waves per SIMD the compiler keeps them in per-lane private memory
// (scratch, served by the vector caches) for RMAX = 16 with four samples per
// lane.  The reverse sweep recomputes every condition once for its
// sigmoid(-z); only a rule of the label adds its conditions up again, for
// the a_k of the U recurrence (the other rules' step of it needs
// log2(1 - r_k) alone).  Per condition the S slots are summed in the lane; two
// conditions' sums go over the wave in one reduction (wave_totals4), and the
// lane that ends each adds it to the block's LDS accumulators (one writer per
// rule set and tile).
// The reverse sweep over one rule's conditions, two at a time: their four
// sums over the wave in one reduction (wave_totals4), added (negated when
// neg) to the rule set's block accumulators accq by the lane that holds each
// (one writer per rule set and tile: the order of these adds is fixed).
// pre: log2 |dL/da_k| per slot (with MUL, log2 r_k, and mul holds
// dL/dr_k).  UPD: also adds every condition to ra, for the rule's log2 r
// afterwards.
template <int S, class Acc, bool TONLY, bool UPD, bool MUL = false>
__device__ __forceinline__ void bwd_rule_conds(const SoftArgs &a, const float *xs, int lane,
                                               int4 r, int cz, float *accq, const float (&pre)[S],
                                               const float (&mul)[S], bool neg, Acc (&ra)[S]) {
  for (int j0 = r.x; j0 < r.x + r.y; j0 += 2) {
    // sums start at -0, so that the first term is added exactly as is
    float g0[2] = {-0.0f, -0.0f}, g1[2] = {-0.0f, -0.0f};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int j = j0 + c;
      if (j >= r.x + r.y) break;
      float z[S], xf[S], xg[S];
      if constexpr (TONLY) {
        cond_z_t<S>(a, xs, lane, j, z, xf, xg);
      } else {
        bool ff;
        cond_z<S>(a, xs, lane, j, z, xf, xg, ff);
      }
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const float t = UPD ? ra[s].add(z[s]) : Acc::term(z[s]);
        // |dL/dz| = |dL/da_k| * sigmoid(-z), or dL/dz = dL/dr_k * r_k * sigmoid(-z)
        const float sg = acc_sig_neg(ra[s], pre[s], z[s], t);
        const float dz = MUL ? mul[s] * sg : sg;
        g0[c] = fmaf(dz, xg[s], g0[c]);
        g1[c] = fmaf(dz, xf[s], g1[c]);
      }
    }
    const float tot = wave_totals4(g0[0], g0[1], g1[0], g1[1]);
    const int row = lane >> 4, c = row >> 1;
    if ((lane & 15) == 15 && j0 + c < r.x + r.y) {
      float *ap = accq + (j0 + c - cz) * 2 + (row & 1);
      *ap += neg ? -tot : tot;
    }
  }
}

template <int K, int RMAX, int S>
__device__ __forceinline__ void l_get(const float (&L)[RMAX][S], int k, float (&out)[S]) {
  if constexpr (K < RMAX) {
    if (k == K) {
#pragma unroll
      for (int s = 0; s < S; ++s) out[s] = L[K][s];
    } else {
      l_get<K + 1, RMAX, S>(L, k, out);
    }
  }
}
template <int K, int RMAX, int S>
__device__ __forceinline__ void l_set(float (&L)[RMAX][S], int k, const float (&v)[S]) {
  if constexpr (K < RMAX) {
    if (k == K) {
#pragma unroll
      for (int s = 0; s < S; ++s) L[K][s] = v[s];
    } else {
      l_set<K + 1, RMAX, S>(L, k, v);
    }
  }
}

// 16 waves share a block's tile and accumulators in LDS, so the LDS limit
// still leaves 32 waves per CU.
constexpr int kBwdRegBlock = 1024;

// Eight waves per SIMD (two blocks per CU) need at most 64 VGPRs and 80
// SGPRs per wave (the SGPR bound measured on gfx950): k_soft_bwd_reg is held
// to that; the variants that keep two samples per lane over 16 or 32 rules
// would spill VGPRs at that size and run as k_soft_bwd_reg_wide, one block
// per CU.
#define AERL_BWD_SGPR_CAP __attribute__((amdgpu_num_sgpr(80)))

// TONLY: the population has threshold conditions only (no x[g] rows).
template <int S, int RMAX, class Acc, bool TONLY>
__device__ __forceinline__ void soft_bwd_reg(const SoftArgs &a) {
  constexpr int TS = 64 * S, WPT = AERL_TILE / TS;
  extern __shared__ __align__(16) float smem[];
  float *xs = smem;                       // [nf][TS]
  float *acc = xs + (size_t)a.nf * TS;    // [Q][max_set_conds][2]
  __shared__ int32_t next_q;
  const int lane = threadIdx.x & 63;
  int label, tile_lo, tile_hi;
  group_range(a, blockIdx.y, label, tile_lo, tile_hi);
  const int q0 = blockIdx.x * a.sets_per_chunk;
  const int Q = min(a.sets_per_chunk, a.n_sets - q0);
  for (int i = threadIdx.x; i < Q * a.max_set_conds * 2; i += blockDim.x) acc[i] = 0.0f;
  const int n4 = a.nf * (TS / 4);
  const float4 *src = reinterpret_cast<const float4 *>(a.x_fm);
  float4 *dst = reinterpret_cast<float4 *>(xs);
  const int64_t row4 = a.n_pad / 4;
  for (int64_t wt = (int64_t)tile_lo * WPT; wt < (int64_t)tile_hi * WPT; ++wt) {
    __syncthreads();
    const int64_t base4 = wt * (TS / 4);
    for (int i = threadIdx.x; i < n4; i += blockDim.x) {
      const int f = i / (TS / 4), k = i % (TS / 4);
      dst[i] = src[(int64_t)f * row4 + base4 + k];
    }
    if (threadIdx.x == 0) next_q = 0;
    __syncthreads();
    const int info = ldc(a.tile_info, wt / WPT);
    const int valid = min(max((info >> 8) - (int)(wt % WPT) * TS, 0), TS);
    bool live[S];
#pragma unroll
    for (int s = 0; s < S; ++s) live[s] = lane * S + s < valid;
    for (;;) {
      const int q = next_item(&next_q);
      if (q >= Q) break;
      const int4 ss = ldc(a.ssets, q0 + q);
      const int dflt = ldc(a.sets, q0 + q).z;
      float L[RMAX][S], B[RMAX][S];
      float logpy[S], surv[S];
#pragma unroll
      for (int s = 0; s < S; ++s) { logpy[s] = kNegInf; surv[s] = 0.0f; }
      // forward sweep
      for (int k = 0; k < ss.y; ++k) {
        const int4 r = ldc(a.rules, ss.x + k);
        Acc ra[S];
        // conditions four at a time, then one at a time (same order)
        int j = r.x;
        const int je = r.x + r.y;
        for (; j + 4 <= je; j += 4) {
          float z[4][S];
          cond_z4<S, TONLY>(a, xs, lane, j, z);
#pragma unroll
          for (int c4 = 0; c4 < 4; ++c4) {
#pragma unroll
            for (int s = 0; s < S; ++s) (void)ra[s].add(z[c4][s]);
          }
        }
        for (; j < je; ++j) {
          float z[S];
          cond_z_only<S>(a, xs, lane, j, z);
#pragma unroll
          for (int s = 0; s < S; ++s) (void)ra[s].add(z[s]);
        }
        const bool hit = r.z == label;
        float lk[S], bk[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
          float a2, b2;
          acc_finish(ra[s], a2, b2);
          lk[s] = a2 + surv[s];
          bk[s] = b2;
          if (hit) logpy[s] = lse(logpy[s], lk[s]);
          surv[s] += b2;
        }
        l_set<0, RMAX, S>(L, k, lk);
        l_set<0, RMAX, S>(B, k, bk);
      }
      float gate[S], U[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        if (dflt == label) logpy[s] = lse(logpy[s], surv[s]);
        // samples whose loss is clamped (or padding) get no gradient; their
        // log P_y is replaced by 0 so that every exponent below stays finite
        const bool on = live[s] && -logpy[s] * kLn2 <= kLossCap;
        gate[s] = on ? 1.0f : 0.0f;
        logpy[s] = on ? logpy[s] : 0.0f;
        U[s] = dflt == label ? 0.0f : kNegInf;
      }
      // reverse sweep
      for (int k = ss.y - 1; k >= 0; --k) {
        const int4 r = ldc(a.rules, ss.x + k);
        const bool hit = r.z == label;
        // dL/da_k = -(1 - 2^U) 2^pre for a rule of the label, +2^pre for
        // another: log2 of its size goes into pre (-inf for a sample with no
        // gradient) and its sign, the same for the whole wave, onto the sums.
        // U, the log2 of a probability, can round to just above 0: 1 - 2^U
        // is then taken as 0.
        float lk[S], bk[S], pre[S];
        l_get<0, RMAX, S>(L, k, lk);
        l_get<0, RMAX, S>(B, k, bk);
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const float lm = hit ? log1mexp2(fminf(U[s], 0.0f)) : U[s];
          pre[s] = gate[s] != 0.0f ? lk[s] + lm - logpy[s] : kNegInf;
        }
        float *accq = acc + (size_t)q * a.max_set_conds * 2;
        Acc ra[S];
        if (hit) {
          // U takes the rule's own log2 r: the conditions are added again
          bwd_rule_conds<S, Acc, TONLY, true>(a, xs, lane, r, ss.z, accq, pre, pre, true, ra);
#pragma unroll
          for (int s = 0; s < S; ++s) U[s] = lse(acc_log_r(ra[s]), bk[s] + U[s]);
        } else {
          // U_k = log2(1 - r_k) + U_k+1, from the forward sweep's log2(1 - r_k)
          bwd_rule_conds<S, Acc, TONLY, false>(a, xs, lane, r, ss.z, accq, pre, pre, false, ra);
#pragma unroll
          for (int s = 0; s < S; ++s) U[s] = bk[s] + U[s];
        }
      }
    }
  }
  __syncthreads();
  for (int q = 0; q < Q; ++q) {
    const int4 ss = ldc(a.ssets, q0 + q);
    for (int i = threadIdx.x; i < ss.w * 2; i += blockDim.x)
      a.part_grad[((int64_t)blockIdx.y * a.n_conds + ss.z) * 2 + i] =
          acc[(size_t)q * a.max_set_conds * 2 + i];
  }
}

template <int S, int RMAX, class Acc, bool TONLY>
__global__ __launch_bounds__(kBwdRegBlock, 8) AERL_BWD_SGPR_CAP void k_soft_bwd_reg(
    const SoftArgs a) {
  soft_bwd_reg<S, RMAX, Acc, TONLY>(a);
}

template <int S, int RMAX, class Acc, bool TONLY>
__global__ __launch_bounds__(kBwdRegBlock) void k_soft_bwd_reg_wide(const SoftArgs a) {
  soft_bwd_reg<S, RMAX, Acc, TONLY>(a);
}

// One block per rule set: sums the group partials of its conditions in a
// fixed order and applies dz/dparam = +-x/tau, -+1/tau and dloss/N.
__global__ void k_soft_bwd_final(const float *__restrict__ part, int32_t n_groups,
                                 int32_t n_conds, const int4 *__restrict__ ssets,
                                 const uint32_t *__restrict__ sconds,
                                 const float *__restrict__ inv_tau,
                                 const float *__restrict__ dloss, int64_t n,
                                 float *__restrict__ dcoef, float *__restrict__ dcoef2,
                                 float *__restrict__ dtheta) {
  const int p = blockIdx.x;
  const int4 ss = ssets[p];
  const double scale = n > 0 ? (double)dloss[p] / (double)n : 0.0;
  for (int i = threadIdx.x; i < ss.w; i += blockDim.x) {
    const int j = ss.z + i;
    // groups in order, eight loads in flight at a time
    double g0 = 0.0, g1 = 0.0;
    int g = 0;
    for (; g + 8 <= n_groups; g += 8) {
      float2 v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k)
        v[k] = *reinterpret_cast<const float2 *>(part + ((int64_t)(g + k) * n_conds + j) * 2);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        g0 += (double)v[k].x;
        g1 += (double)v[k].y;
      }
    }
    for (; g < n_groups; ++g) {
      const float *pp = part + ((int64_t)g * n_conds + j) * 2;
      g0 += (double)pp[0];
      g1 += (double)pp[1];
    }
    const uint32_t sc = sconds[j];
    const bool ff = ((sc >> 24) & 1u) != 0;
    const double sinv = (((sc >> 25) & 1u) ? 1.0 : -1.0) * (double)inv_tau[sc & 0xfffu];
    dcoef[j] = (float)(sinv * g1 * scale);
    dcoef2[j] = ff ? (float)(-sinv * g0 * scale) : 0.0f;
    dtheta[j] = ff ? 0.0f : (float)(-sinv * g0 * scale);
  }
}

struct SoftPlan {
  int S, Q, TG, n_groups;
  int rmax;  // backward: rule bound of the register-resident kernel, 0 = general kernel
  int waves; // LDS-state kernels: waves per block
  size_t lds;
};

// Waves and rule-set chunk of an LDS-state adjoint kernel (tile xs bytes,
// per_set accumulator bytes, per_wave state bytes): the most waves (at most
// max_waves) that fit with one rule set per chunk, then the largest chunk
// (at most max_q sets) that fits.
void lds_state_plan(SoftPlan &p, size_t xs, size_t per_set, size_t per_wave, int max_waves,
                    int max_q, int n_sets) {
  p.waves = max_waves;
  while (p.waves > 1 && xs + per_set + p.waves * per_wave > kDynLdsMax) p.waves >>= 1;
  p.Q = std::max(1, std::min(n_sets, max_q));
  while (p.Q > 1 && xs + p.Q * per_set + p.waves * per_wave > kDynLdsMax) p.Q >>= 1;
  p.lds = xs + (size_t)p.Q * per_set + p.waves * per_wave;
}

int64_t count_groups(const DatasetRec &ds, int tg) {
  int64_t g = 0;
  for (int c = 0; c < ds.nc; ++c) g += (ds.region_tiles[c] + tg - 1) / tg;
  return g;
}

// Tiles per block group.  A launch has (set chunks) x (tile groups) blocks;
// the fewest groups that still give about `target` blocks (measured on the
// 262,144 x 32, 1024-set workload: a forward grid of one wave of blocks,
// 64 groups, runs 10.9 ms, 1024 groups 6.9 ms, as its blocks no longer stage
// their tiles in step; the adjoint runs 22.8 ms at 64 groups and 20.8 ms at
// 256), then fewer while the per-group partial sums (bytes_per_group each)
// exceed max_bytes.
int tiles_per_group(const DatasetRec &ds, int64_t chunks, int64_t target, size_t bytes_per_group,
                    size_t max_bytes) {
  int32_t widest = 1;
  for (int c = 0; c < ds.nc; ++c) widest = std::max(widest, ds.region_tiles[c]);
  const int64_t need = (target + std::max<int64_t>(chunks, 1) - 1) / std::max<int64_t>(chunks, 1);
  int tg = 1;
  while (tg < widest && count_groups(ds, 2 * tg) >= need) tg *= 2;
  while (tg < widest && (size_t)count_groups(ds, tg) * bytes_per_group > max_bytes) tg *= 2;
  return tg;
}
// Forward: 16 blocks per block slot (four 512-thread blocks per CU on 256
// CUs), fp64 partials of at most 8 MiB (half the no-allocation scratch).
constexpr int64_t kFwdTargetBlocks = 16384;
constexpr size_t kFwdPartMax = (size_t)8 << 20;
// Backward: 8 blocks per slot (two 1024-thread blocks per CU), partial
// gradients of at most 1 GiB.
constexpr int64_t kBwdTargetBlocks = 4096;
constexpr size_t kBwdPartMax = (size_t)1 << 30;

// Rule sets per block: 64, or fewer, down to one per wave (min_q), while
// the grid (set chunks x `groups` tile groups) stays under `target` blocks,
// so that a small workload spreads over more CUs instead of walking several
// rule sets per wave on a few of them.
int sets_per_block(int n_sets, int64_t groups, int64_t target, int min_q) {
  int q = std::max(1, std::min(n_sets, 64));
  while (q / 2 >= min_q && (int64_t)((n_sets + q - 1) / q) * groups < target) q /= 2;
  return q;
}

SoftPlan plan_forward(const DatasetRec &ds, const PopRec &pop) {
  SoftPlan p{};
  p.S = 4;
  while (p.S > 1 && (size_t)ds.nf * 256 * p.S > 64 * 1024) p.S >>= 1;
  p.Q = sets_per_block(pop.n_sets, count_groups(ds, 1), kFwdTargetBlocks, kSoftBlock / 64);
  p.TG = tiles_per_group(ds, (pop.n_sets + p.Q - 1) / p.Q, kFwdTargetBlocks,
                         (size_t)std::max(pop.n_sets, 1) * sizeof(double), kFwdPartMax);
  p.n_groups = (int)count_groups(ds, p.TG);
  p.lds = (size_t)ds.nf * 64 * p.S * 4 + (size_t)p.Q * 8;
  return p;
}

// Backward: the register-resident kernel when the longest rule set has at
// most 32 rules (bound 8 or 16: four samples per lane; 32: two), else the
// general kernel with per-rule state in LDS (one sample per lane).
SoftPlan plan_backward(const DatasetRec &ds, const PopRec &pop) {
  SoftPlan p{};
  const int R = std::max(pop.max_rules, 1);
  const size_t per_set = (size_t)std::max(pop.max_set_conds, 1) * 2 * 4;
  p.TG = tiles_per_group(ds, (pop.n_sets + 63) / 64, kBwdTargetBlocks,
                         (size_t)std::max(pop.n_conds, 1) * 2 * sizeof(float), kBwdPartMax);
  p.n_groups = (int)count_groups(ds, p.TG);
  p.rmax = R <= 8 ? 8 : R <= 16 ? 16 : R <= 32 ? 32 : 0;
  if (p.rmax > 0) {
    p.S = p.rmax <= 16 ? 4 : 2;
    while (p.S > 1 && (size_t)ds.nf * 256 * p.S > 64 * 1024) p.S >>= 1;
    const size_t xs = (size_t)ds.nf * 64 * p.S * 4;
    p.Q = sets_per_block(pop.n_sets, p.n_groups, kBwdTargetBlocks, kBwdRegBlock / 64);
    while (p.Q > 1 && xs + p.Q * per_set > kLdsPerCu / 2 - kStaticLds) p.Q >>= 1;  // two blocks per CU
    p.lds = xs + (size_t)p.Q * per_set;
    if (p.lds <= kDynLdsMax) return p;
  }
  p.rmax = 0;
  p.S = 1;
  lds_state_plan(p, (size_t)ds.nf * 64 * 4, per_set, (size_t)R * 128 * 4, kBwdWaves, 16, pop.n_sets);
  return p;
}

void fill_args(SoftArgs &a, const SoftLaunch &l, const SoftPlan &p) {
  const DatasetRec &ds = *l.ds;
  const PopRec &pop = *l.pop;
  a = SoftArgs{};
  a.x_fm = ds.x_fm;
  a.n_pad = ds.n_pad;
  a.nf = ds.nf;
  a.nc = ds.nc;
  a.tile_info = ds.tile_info;
  a.inv_tau = ds.inv_tau;
  a.sets = pop.sets;
  a.ssets = pop.ssets;
  a.rules = pop.rules;
  a.sconds = pop.sconds;
  a.coef = l.coef;
  a.coef2 = l.coef2;
  a.theta = l.theta;
  a.n_sets = pop.n_sets;
  a.n_conds = pop.n_conds;
  a.sets_per_chunk = p.Q;
  a.tiles_per_group = p.TG;
  a.n_groups = p.n_groups;
  a.max_rules = std::max(pop.max_rules, 1);
  a.max_set_conds = std::max(pop.max_set_conds, 1);
  for (int c = 0; c < ds.nc; ++c) {
    a.region_tile0[c] = ds.region_tile0[c];
    a.region_tiles[c] = ds.region_tiles[c];
  }
}

template <class Acc, bool TONLY>
void launch_fwd(const SoftPlan &p, dim3 grid, hipStream_t st, const SoftArgs &a) {
  switch (p.S) {
    case 4: hipLaunchKernelGGL((k_soft_fwd<4, Acc, TONLY>), grid, dim3(kSoftBlock), p.lds, st, a); break;
    case 2: hipLaunchKernelGGL((k_soft_fwd<2, Acc, TONLY>), grid, dim3(kSoftBlock), p.lds, st, a); break;
    default: hipLaunchKernelGGL((k_soft_fwd<1, Acc, TONLY>), grid, dim3(kSoftBlock), p.lds, st, a); break;
  }
}

template <class Acc, bool TONLY>
void launch_bwd_reg(const SoftPlan &p, dim3 grid, hipStream_t st, const SoftArgs &a) {
  const dim3 rb(kBwdRegBlock);
  if (p.rmax == 8 && p.S == 4) {
    hipLaunchKernelGGL((k_soft_bwd_reg<4, 8, Acc, TONLY>), grid, rb, p.lds, st, a);
  } else if (p.rmax == 8 && p.S == 2) {
    hipLaunchKernelGGL((k_soft_bwd_reg<2, 8, Acc, TONLY>), grid, rb, p.lds, st, a);
  } else if (p.rmax == 16 && p.S == 4) {
    hipLaunchKernelGGL((k_soft_bwd_reg<4, 16, Acc, TONLY>), grid, rb, p.lds, st, a);
  } else if (p.rmax == 16 && p.S == 2) {
    hipLaunchKernelGGL((k_soft_bwd_reg_wide<2, 16, Acc, TONLY>), grid, rb, p.lds, st, a);
  } else if (p.rmax == 32 && p.S == 2) {
    hipLaunchKernelGGL((k_soft_bwd_reg_wide<2, 32, Acc, TONLY>), grid, rb, p.lds, st, a);
  } else if (p.rmax == 8) {  // one sample per lane (wide datasets)
    hipLaunchKernelGGL((k_soft_bwd_reg<1, 8, Acc, TONLY>), grid, rb, p.lds, st, a);
  } else if (p.rmax == 16) {
    hipLaunchKernelGGL((k_soft_bwd_reg<1, 16, Acc, TONLY>), grid, rb, p.lds, st, a);
  } else {
    hipLaunchKernelGGL((k_soft_bwd_reg<1, 32, Acc, TONLY>), grid, rb, p.lds, st, a);
  }
}

}  // namespace

bool soft_backward_supported(const DatasetRec &ds, const PopRec &pop) {
  return plan_backward(ds, pop).lds <= kDynLdsMax;
}

namespace {

// Workspace: the partial sums, then (256-byte aligned) the condition records.
size_t soft_part_bytes(const DatasetRec &ds, const PopRec &pop, bool backward) {
  size_t b;
  if (backward) {
    const SoftPlan p = plan_backward(ds, pop);
    b = (size_t)p.n_groups * (size_t)std::max(pop.n_conds, 1) * 2 * sizeof(float);
  } else {
    const SoftPlan p = plan_forward(ds, pop);
    b = (size_t)p.n_groups * (size_t)std::max(pop.n_sets, 1) * sizeof(double);
  }
  return (b + 255) & ~size_t(255);
}

hipError_t launch_prep(const SoftLaunch &l, const SoftArgs &a, uint4 *crec, hipStream_t st) {
  const int n = l.pop->n_conds;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_soft_prep, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a.sconds,
                     a.inv_tau, a.coef, a.coef2, a.theta, l.pop->cmask, n, crec);
  return hipGetLastError();
}

}  // namespace

size_t soft_ws_bytes(const DatasetRec &ds, const PopRec &pop, bool backward) {
  return soft_part_bytes(ds, pop, backward) + (size_t)std::max(pop.n_conds, 1) * sizeof(uint4);
}

hipError_t launch_soft_forward(const SoftLaunch &l, hipStream_t st) {
  const PopRec &pop = *l.pop;
  if (pop.n_sets == 0) return hipSuccess;
  const SoftPlan p = plan_forward(*l.ds, pop);
  SoftArgs a;
  fill_args(a, l, p);
  a.part_loss = static_cast<double *>(l.ws);
  uint4 *crec = reinterpret_cast<uint4 *>(static_cast<char *>(l.ws) + soft_part_bytes(*l.ds, pop, false));
  a.crec = crec;
  hipError_t e0 = launch_prep(l, a, crec, st);
  if (e0 != hipSuccess) return e0;
  if (p.n_groups > 0) {
    const dim3 grid((unsigned)((pop.n_sets + p.Q - 1) / p.Q), (unsigned)p.n_groups);
    const bool prod = pop.max_rule_conds <= kProdMaxConds, tonly = pop.n_ff == 0 && pop.n_cat == 0;
    if (prod && tonly) {
      launch_fwd<RuleProd, true>(p, grid, st, a);
    } else if (prod) {
      launch_fwd<RuleProd, false>(p, grid, st, a);
    } else if (tonly) {
      launch_fwd<RuleAcc, true>(p, grid, st, a);
    } else {
      launch_fwd<RuleAcc, false>(p, grid, st, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_soft_fwd_final, dim3((unsigned)((pop.n_sets + 63) / 64)),
                     dim3(kFwdFinalWaves * 64), 0, st,
                     a.part_loss, p.n_groups, pop.n_sets, l.ds->n, l.loss);
  return hipGetLastError();
}

// ------------------------------------------------------------ softmax head
// Section 5: probabilistic outputs through a softmax.  Each rule votes for
// its class with its soft truth r_k, the default class takes the probability
// that no rule fires, D = prod_k (1 - r_k):
//   v_c = sum_{k: class_k = c} r_k + [c = default] D,  P = softmax(beta v),
// L = min(-log P_y, 100).  Adjoint: dL/dv_c = beta (P_c - [c = y]),
// dL/dr_k = dL/dv_{class_k} - dL/dv_default * prod_{i != k} (1 - r_i), the
// product being 2^(S_k + T_k) with the prefix S_k and suffix T_k sums of
// log2(1 - r_i); dL/dz = dL/dr_k * r_k * sigmoid(-z).  Classes are padded to
// NC (a power of two up to kSmaxMaxClasses) in registers; rule classes are
// wave-uniform, so a vote is NC selects.
namespace {

template <int NC>
__device__ __forceinline__ void add_vote(float (&v)[NC], int cls, float r) {
#pragma unroll
  for (int c = 0; c < NC; ++c) v[c] += (c == cls) ? r : 0.0f;
}

template <int NC>
__device__ __forceinline__ float pick(const float (&v)[NC], int cls) {
  float out = 0.0f;
#pragma unroll
  for (int c = 0; c < NC; ++c) out = (c == cls) ? v[c] : out;
  return out;
}

// log2 P_y from the votes, and P (every class) into p.  beta2 = beta*log2(e).
template <int NC>
__device__ __forceinline__ float smax_log2py(const float (&v)[NC], int nc, float beta2, int y,
                                             float (&p)[NC]) {
  float m = kNegInf;
#pragma unroll
  for (int c = 0; c < NC; ++c)
    if (c < nc) m = fmaxf(m, beta2 * v[c]);
  float sum = 0.0f;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    p[c] = c < nc ? fexp2(beta2 * v[c] - m) : 0.0f;
    sum += p[c];
  }
  const float inv = 1.0f / sum;
  float ty = 0.0f;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    ty = (c == y) ? beta2 * v[c] : ty;
    p[c] *= inv;
  }
  return ty - m - flog2(sum);
}

constexpr int kSmaxFwdS = 2;
constexpr int kSmaxBwdWaves = 4;

template <int NC, class Acc, bool TONLY>
__global__ __launch_bounds__(kSoftBlock) void k_smax_fwd(const SoftArgs a, float beta2) {
  constexpr int S = kSmaxFwdS, TS = 64 * S, WPT = AERL_TILE / TS;
  extern __shared__ __align__(16) float smem[];
  float *xs = smem;
  double *acc = reinterpret_cast<double *>(smem + (size_t)a.nf * TS);  // [Q]
  __shared__ int32_t next_q;
  const int lane = threadIdx.x & 63;
  int label, tile_lo, tile_hi;
  group_range(a, blockIdx.y, label, tile_lo, tile_hi);
  const int q0 = blockIdx.x * a.sets_per_chunk;
  const int Q = min(a.sets_per_chunk, a.n_sets - q0);
  for (int i = threadIdx.x; i < Q; i += blockDim.x) acc[i] = 0.0;
  const int n4 = a.nf * (TS / 4);
  const float4 *src = reinterpret_cast<const float4 *>(a.x_fm);
  float4 *dst = reinterpret_cast<float4 *>(xs);
  const int64_t row4 = a.n_pad / 4;
  for (int64_t wt = (int64_t)tile_lo * WPT; wt < (int64_t)tile_hi * WPT; ++wt) {
    __syncthreads();
    const int64_t base4 = wt * (TS / 4);
    for (int i = threadIdx.x; i < n4; i += blockDim.x) {
      const int f = i / (TS / 4), k = i % (TS / 4);
      dst[i] = src[(int64_t)f * row4 + base4 + k];
    }
    if (threadIdx.x == 0) next_q = 0;
    __syncthreads();
    const int info = ldc(a.tile_info, wt / WPT);
    const int valid = min(max((info >> 8) - (int)(wt % WPT) * TS, 0), TS);
    for (;;) {
      const int q = next_item(&next_q);
      if (q >= Q) break;
      const int4 ss = ldc(a.ssets, q0 + q);
      const int dflt = ldc(a.sets, q0 + q).z;
      float v[S][NC], surv[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        surv[s] = 0.0f;
#pragma unroll
        for (int c = 0; c < NC; ++c) v[s][c] = 0.0f;
      }
      for (int k = 0; k < ss.y; ++k) {
        const int4 r = ldc(a.rules, ss.x + k);
        Acc ra[S];
        int j = r.x;
        const int je = r.x + r.y;
        for (; j + 4 <= je; j += 4) {
          float z[4][S];
          cond_z4<S, TONLY>(a, xs, lane, j, z);
#pragma unroll
          for (int c4 = 0; c4 < 4; ++c4) {
#pragma unroll
            for (int s = 0; s < S; ++s) (void)ra[s].add(z[c4][s]);
          }
        }
        for (; j < je; ++j) {
          float z[S];
          cond_z_only<S>(a, xs, lane, j, z);
#pragma unroll
          for (int s = 0; s < S; ++s) (void)ra[s].add(z[s]);
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
          float a2, b2;
          acc_finish(ra[s], a2, b2);
          add_vote(v[s], r.z, fexp2(a2));
          surv[s] += b2;
        }
      }
      float part = 0.0f;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        add_vote(v[s], dflt, fexp2(surv[s]));
        float p[NC];
        const float l2 = smax_log2py(v[s], a.nc, beta2, label, p);
        part += lane * S + s < valid ? sample_loss(l2) : 0.0f;
      }
      part = wave_sum(part);
      if (lane == 0) acc[q] += (double)part;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < Q; i += blockDim.x)
    a.part_loss[(int64_t)blockIdx.y * a.n_sets + q0 + i] = acc[i];
}

template <int NC, class Acc, bool TONLY>
__global__ __launch_bounds__(kSmaxBwdWaves * 64) void k_smax_bwd(const SoftArgs a, float beta,
                                                                 float beta2) {
  constexpr int TS = 64, WPT = AERL_TILE / TS;
  extern __shared__ __align__(16) float smem[];
  float *xs = smem;                                                     // [nf][64]
  float *acc = xs + (size_t)a.nf * TS;                                  // [Q][max_set_conds][2]
  float *store = acc + (size_t)a.sets_per_chunk * a.max_set_conds * 2;  // [wave][R][2][64]
  __shared__ int32_t next_q;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float *my = store + (size_t)wave * a.max_rules * 128;
  int label, tile_lo, tile_hi;
  group_range(a, blockIdx.y, label, tile_lo, tile_hi);
  const int q0 = blockIdx.x * a.sets_per_chunk;
  const int Q = min(a.sets_per_chunk, a.n_sets - q0);
  for (int i = threadIdx.x; i < Q * a.max_set_conds * 2; i += blockDim.x) acc[i] = 0.0f;
  const int n4 = a.nf * (TS / 4);
  const float4 *src = reinterpret_cast<const float4 *>(a.x_fm);
  float4 *dst = reinterpret_cast<float4 *>(xs);
  const int64_t row4 = a.n_pad / 4;
  for (int64_t wt = (int64_t)tile_lo * WPT; wt < (int64_t)tile_hi * WPT; ++wt) {
    __syncthreads();
    const int64_t base4 = wt * (TS / 4);
    for (int i = threadIdx.x; i < n4; i += blockDim.x) {
      const int f = i / (TS / 4), k = i % (TS / 4);
      dst[i] = src[(int64_t)f * row4 + base4 + k];
    }
    if (threadIdx.x == 0) next_q = 0;
    __syncthreads();
    const int info = ldc(a.tile_info, wt / WPT);
    const int valid = min(max((info >> 8) - (int)(wt % WPT) * TS, 0), TS);
    const bool live = lane < valid;
    for (;;) {
      const int q = next_item(&next_q);
      if (q >= Q) break;
      const int4 ss = ldc(a.ssets, q0 + q);
      const int dflt = ldc(a.sets, q0 + q).z;
      // forward sweep: log2 r_k and the prefix of log2(1 - r_i) before k
      float v[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) v[c] = 0.0f;
      float surv = 0.0f;
      for (int k = 0; k < ss.y; ++k) {
        const int4 r = ldc(a.rules, ss.x + k);
        Acc ra;
        for (int j = r.x; j < r.x + r.y; ++j) {
          float z[1];
          cond_z_only<1>(a, xs, lane, j, z);
          (void)ra.add(z[0]);
        }
        float a2, b2;
        acc_finish(ra, a2, b2);
        my[k * 128 + lane] = a2;
        my[k * 128 + 64 + lane] = surv;
        add_vote(v, r.z, fexp2(a2));
        surv += b2;
      }
      add_vote(v, dflt, fexp2(surv));
      float p[NC];
      const float l2 = smax_log2py(v, a.nc, beta2, label, p);
      // clamped samples (and padding) get no gradient
      const bool on = live && -l2 * kLn2 <= kLossCap;
      // dL/dv_c = beta (P_c - [c = y]); for the label, -beta times the sum of
      // the other classes' probabilities (P_y - 1 would cancel when P_y ~ 1)
      float others = 0.0f;
#pragma unroll
      for (int c = 0; c < NC; ++c) others += c == label ? 0.0f : p[c];
      float gv[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) gv[c] = on ? beta * (c == label ? -others : p[c]) : 0.0f;
      const float gd = pick(gv, dflt);
      // reverse sweep with the suffix of log2(1 - r_i) after k
      float tail = 0.0f;
      const bool few = ss.w <= 64;
      int tot0 = 0, tot1 = 0;
      for (int k = ss.y - 1; k >= 0; --k) {
        const int4 r = ldc(a.rules, ss.x + k);
        const float a2k = my[k * 128 + lane];
        const float others = my[k * 128 + 64 + lane] + tail;  // log2 prod_{i != k} (1 - r_i)
        // a rule of the default class: g_d (1 - prod), with 1 - prod formed
        // directly (the difference of the two terms would cancel)
        const float drk = r.z == dflt ? gd * one_minus_exp2(others)
                                      : pick(gv, r.z) - gd * fexp2(others);
        Acc ra;
        for (int j = r.x; j < r.x + r.y; ++j) {
          float z[1], xf[1], xg[1];
          if constexpr (TONLY) {
            cond_z_t<1>(a, xs, lane, j, z, xf, xg);
          } else {
            bool ff;
            cond_z<1>(a, xs, lane, j, z, xf, xg, ff);
          }
          const float t = ra.add(z[0]);
          // dL/dz = dL/dr_k * r_k * sigmoid(-z)
          const float dz = drk * acc_sig_neg(ra, a2k, z[0], t);
          const float g0 = wave_total_last(dz * xg[0]);
          const float g1 = wave_total_last(dz * xf[0]);
          if (few) {
            // lane i keeps the walk's totals of condition i of the set
            const int v0 = __builtin_amdgcn_readlane(__float_as_int(g0), 63);
            const int v1 = __builtin_amdgcn_readlane(__float_as_int(g1), 63);
            const bool mine = lane == j - ss.z;
            tot0 = mine ? v0 : tot0;
            tot1 = mine ? v1 : tot1;
          } else if (lane == 63) {
            // one writer per (rule set, tile): the order of these adds is fixed
            float *ap = acc + ((size_t)q * a.max_set_conds + (j - ss.z)) * 2;
            ap[0] += g0;
            ap[1] += g1;
          }
        }
        float a2, b2;
        acc_finish(ra, a2, b2);
        tail += b2;
      }
      if (few && lane < ss.w) {
        float *ap = acc + ((size_t)q * a.max_set_conds + lane) * 2;
        ap[0] += __int_as_float(tot0);
        ap[1] += __int_as_float(tot1);
      }
    }
  }
  __syncthreads();
  for (int q = 0; q < Q; ++q) {
    const int4 ss = ldc(a.ssets, q0 + q);
    for (int i = threadIdx.x; i < ss.w * 2; i += blockDim.x)
      a.part_grad[((int64_t)blockIdx.y * a.n_conds + ss.z) * 2 + i] =
          acc[(size_t)q * a.max_set_conds * 2 + i];
  }
}

// Adjoint of the softmax head for rule sets of at most 16 rules and at most
// four classes, four samples per lane, 16 waves per block: the per-rule
// state between the two sweeps (log2 r_k, the prefix sum of log2(1 - r_i)
// before k and log2(1 - r_k), for each of the lane's samples) is a
// 16 x 4 x 3 array per lane, read and written through a uniform branch chain
// on k (the compiler keeps it in per-lane private memory at the 64-VGPR
// budget of two blocks per CU).  The reverse sweep needs each condition's
// sigmoid(-z) alone, so it adds no condition up again; the conditions' sums
// go over the wave and to LDS as in the first-firing adjoint.  Same
// formulas as k_smax_bwd.
constexpr int kSmaxRegRules = 16;

template <int NC, class Acc, bool TONLY>
__global__ __launch_bounds__(kBwdRegBlock, 8) AERL_BWD_SGPR_CAP void k_smax_bwd_reg(
    const SoftArgs a, float beta, float beta2) {
  constexpr int S = 4, RMAX = kSmaxRegRules, TS = 64 * S, WPT = AERL_TILE / TS;
  extern __shared__ __align__(16) float smem[];
  float *xs = smem;                       // [nf][TS]
  float *acc = xs + (size_t)a.nf * TS;    // [Q][max_set_conds][2]
  __shared__ int32_t next_q;
  const int lane = threadIdx.x & 63;
  int label, tile_lo, tile_hi;
  group_range(a, blockIdx.y, label, tile_lo, tile_hi);
  const int q0 = blockIdx.x * a.sets_per_chunk;
  const int Q = min(a.sets_per_chunk, a.n_sets - q0);
  for (int i = threadIdx.x; i < Q * a.max_set_conds * 2; i += blockDim.x) acc[i] = 0.0f;
  const int n4 = a.nf * (TS / 4);
  const float4 *src = reinterpret_cast<const float4 *>(a.x_fm);
  float4 *dst = reinterpret_cast<float4 *>(xs);
  const int64_t row4 = a.n_pad / 4;
  for (int64_t wt = (int64_t)tile_lo * WPT; wt < (int64_t)tile_hi * WPT; ++wt) {
    __syncthreads();
    const int64_t base4 = wt * (TS / 4);
    for (int i = threadIdx.x; i < n4; i += blockDim.x) {
      const int f = i / (TS / 4), k = i % (TS / 4);
      dst[i] = src[(int64_t)f * row4 + base4 + k];
    }
    if (threadIdx.x == 0) next_q = 0;
    __syncthreads();
    const int info = ldc(a.tile_info, wt / WPT);
    const int valid = min(max((info >> 8) - (int)(wt % WPT) * TS, 0), TS);
    for (;;) {
      const int q = next_item(&next_q);
      if (q >= Q) break;
      const int4 ss = ldc(a.ssets, q0 + q);
      const int dflt = ldc(a.sets, q0 + q).z;
      float LA[RMAX][S], LP[RMAX][S], LB[RMAX][S];
      float v[S][NC], surv[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        surv[s] = 0.0f;
#pragma unroll
        for (int c = 0; c < NC; ++c) v[s][c] = 0.0f;
      }
      // forward sweep: log2 r_k and the prefix of log2(1 - r_i) before k
      for (int k = 0; k < ss.y; ++k) {
        const int4 r = ldc(a.rules, ss.x + k);
        Acc ra[S];
        // conditions four at a time, then one at a time (same order)
        int j = r.x;
        const int je = r.x + r.y;
        for (; j + 4 <= je; j += 4) {
          float z[4][S];
          cond_z4<S, TONLY>(a, xs, lane, j, z);
#pragma unroll
          for (int c4 = 0; c4 < 4; ++c4) {
#pragma unroll
            for (int s = 0; s < S; ++s) (void)ra[s].add(z[c4][s]);
          }
        }
        for (; j < je; ++j) {
          float z[S];
          cond_z_only<S>(a, xs, lane, j, z);
#pragma unroll
          for (int s = 0; s < S; ++s) (void)ra[s].add(z[s]);
        }
        float a2s[S], pre[S], b2s[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
          float a2, b2;
          acc_finish(ra[s], a2, b2);
          a2s[s] = a2;
          pre[s] = surv[s];
          b2s[s] = b2;
          add_vote(v[s], r.z, fexp2(a2));
          surv[s] += b2;
        }
        l_set<0, RMAX, S>(LA, k, a2s);
        l_set<0, RMAX, S>(LP, k, pre);
        l_set<0, RMAX, S>(LB, k, b2s);
      }
      // dL/dv per slot (clamped samples and padding get none); for the
      // label, -beta times the other classes' probabilities
      float gv[S][NC], gd[S], tail[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        add_vote(v[s], dflt, fexp2(surv[s]));
        float p[NC];
        const float l2 = smax_log2py(v[s], a.nc, beta2, label, p);
        const bool on = lane * S + s < valid && -l2 * kLn2 <= kLossCap;
        float others = 0.0f;
#pragma unroll
        for (int c = 0; c < NC; ++c) others += c == label ? 0.0f : p[c];
#pragma unroll
        for (int c = 0; c < NC; ++c) gv[s][c] = on ? beta * (c == label ? -others : p[c]) : 0.0f;
        gd[s] = pick(gv[s], dflt);
        tail[s] = 0.0f;
      }
      // reverse sweep with the suffix of log2(1 - r_i) after k
      for (int k = ss.y - 1; k >= 0; --k) {
        const int4 r = ldc(a.rules, ss.x + k);
        float la[S], lp[S], drk[S];
        l_get<0, RMAX, S>(LA, k, la);
        l_get<0, RMAX, S>(LP, k, lp);
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const float oth = lp[s] + tail[s];  // log2 prod_{i != k} (1 - r_i)
          drk[s] = r.z == dflt ? gd[s] * one_minus_exp2(oth)
                               : pick(gv[s], r.z) - gd[s] * fexp2(oth);
        }
        // the conditions' terms need no accumulator: log2(1 - r_k) comes
        // from the forward sweep
        Acc ra[S];
        bwd_rule_conds<S, Acc, TONLY, false, true>(a, xs, lane, r, ss.z,
                                                   acc + (size_t)q * a.max_set_conds * 2, la, drk,
                                                   false, ra);
        float lb[S];
        l_get<0, RMAX, S>(LB, k, lb);
#pragma unroll
        for (int s = 0; s < S; ++s) tail[s] += lb[s];
      }
    }
  }
  __syncthreads();
  for (int q = 0; q < Q; ++q) {
    const int4 ss = ldc(a.ssets, q0 + q);
    for (int i = threadIdx.x; i < ss.w * 2; i += blockDim.x)
      a.part_grad[((int64_t)blockIdx.y * a.n_conds + ss.z) * 2 + i] =
          acc[(size_t)q * a.max_set_conds * 2 + i];
  }
}

// Class probabilities of one rule set for row-major rows, one row per
// thread (the gathered condition records give z).
template <int NC>
__global__ __launch_bounds__(256) void k_smax_proba(const float *__restrict__ rows, int64_t n,
                                                    int32_t nf, int32_t nc, int32_t set,
                                                    const int4 *__restrict__ sets,
                                                    const int4 *__restrict__ ssets,
                                                    const int4 *__restrict__ rules,
                                                    const uint4 *__restrict__ crec, float beta2,
                                                    float *__restrict__ probs) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int4 ss = ssets[set];
  const int32_t dflt = sets[set].z;
  const float *x = rows + i * nf;
  float v[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) v[c] = 0.0f;
  float surv = 0.0f;
  for (int k = 0; k < ss.y; ++k) {
    const int4 r = rules[ss.x + k];
    RuleAcc ra;
    for (int j = r.x; j < r.x + r.y; ++j) {
      const uint4 c4 = crec[j];
      const uint32_t sc = c4.x;
      const float xf = x[sc & 0xfffu];
      if (sc & kSoftCat) {
        (void)ra.add(cat_z(xf, c4.y, c4.z));
        continue;
      }
      const float rv = __uint_as_float(c4.z);
      const float rhs = (sc & kSoftFF) ? rv * x[(sc >> 12) & 0xfffu] : rv;
      (void)ra.add(fmaf(__uint_as_float(c4.y), xf, -rhs) * __uint_as_float(c4.w));
    }
    float a2, b2;
    acc_finish(ra, a2, b2);
    add_vote(v, r.z, fexp2(a2));
    surv += b2;
  }
  add_vote(v, dflt, fexp2(surv));
  float p[NC];
  (void)smax_log2py(v, nc, beta2, 0, p);
  for (int c = 0; c < nc; ++c) probs[i * nc + c] = p[c];
}

int smax_nc(int nc) { return nc <= 2 ? 2 : nc <= 4 ? 4 : nc <= 8 ? 8 : 16; }

SoftPlan plan_smax_backward(const DatasetRec &ds, const PopRec &pop) {
  SoftPlan p{};
  const int R = std::max(pop.max_rules, 1);
  const size_t per_set = (size_t)std::max(pop.max_set_conds, 1) * 2 * 4;
  p.TG = tiles_per_group(ds, (pop.n_sets + 63) / 64, kBwdTargetBlocks,
                         (size_t)std::max(pop.n_conds, 1) * 2 * sizeof(float), kBwdPartMax);
  p.n_groups = (int)count_groups(ds, p.TG);
  // up to 16 rules and four classes on at most 64 features: four samples per
  // lane with the per-rule state in per-lane memory, two blocks per CU
  if (R <= kSmaxRegRules && smax_nc(ds.nc) <= 4 && (size_t)ds.nf * 256 * 4 <= 64 * 1024) {
    p.rmax = kSmaxRegRules;
    p.S = 4;
    const size_t xs = (size_t)ds.nf * 64 * p.S * 4;
    p.Q = sets_per_block(pop.n_sets, p.n_groups, kBwdTargetBlocks, kBwdRegBlock / 64);
    while (p.Q > 1 && xs + p.Q * per_set > kLdsPerCu / 2 - kStaticLds) p.Q >>= 1;
    p.lds = xs + (size_t)p.Q * per_set;
    if (p.lds <= kDynLdsMax) return p;
  }
  p.rmax = 0;
  p.S = 1;
  lds_state_plan(p, (size_t)ds.nf * 64 * 4, per_set, (size_t)R * 128 * 4, kSmaxBwdWaves, 16,
                 pop.n_sets);
  return p;
}

SoftPlan plan_smax_forward(const DatasetRec &ds, const PopRec &pop) {
  SoftPlan p = plan_forward(ds, pop);  // same groups (and so the same workspace)
  p.S = kSmaxFwdS;
  p.lds = (size_t)ds.nf * 64 * p.S * 4 + (size_t)p.Q * 8;
  return p;
}

template <int NC>
void launch_smax_fwd_nc(const SoftPlan &p, dim3 grid, hipStream_t st, const SoftArgs &a, bool prod,
                        bool tonly, float beta2) {
  if (prod && tonly)
    hipLaunchKernelGGL((k_smax_fwd<NC, RuleProd, true>), grid, dim3(kSoftBlock), p.lds, st, a, beta2);
  else if (prod)
    hipLaunchKernelGGL((k_smax_fwd<NC, RuleProd, false>), grid, dim3(kSoftBlock), p.lds, st, a, beta2);
  else if (tonly)
    hipLaunchKernelGGL((k_smax_fwd<NC, RuleAcc, true>), grid, dim3(kSoftBlock), p.lds, st, a, beta2);
  else
    hipLaunchKernelGGL((k_smax_fwd<NC, RuleAcc, false>), grid, dim3(kSoftBlock), p.lds, st, a, beta2);
}

template <int NC>
void launch_smax_bwd_nc(const SoftPlan &p, dim3 grid, hipStream_t st, const SoftArgs &a, bool prod,
                        bool tonly, float beta, float beta2) {
  if constexpr (NC <= 4) {
    if (p.rmax == kSmaxRegRules) {
      const dim3 rb(kBwdRegBlock);
      if (prod && tonly)
        hipLaunchKernelGGL((k_smax_bwd_reg<NC, RuleProd, true>), grid, rb, p.lds, st, a, beta, beta2);
      else if (prod)
        hipLaunchKernelGGL((k_smax_bwd_reg<NC, RuleProd, false>), grid, rb, p.lds, st, a, beta, beta2);
      else if (tonly)
        hipLaunchKernelGGL((k_smax_bwd_reg<NC, RuleAcc, true>), grid, rb, p.lds, st, a, beta, beta2);
      else
        hipLaunchKernelGGL((k_smax_bwd_reg<NC, RuleAcc, false>), grid, rb, p.lds, st, a, beta, beta2);
      return;
    }
  }
  const dim3 b(p.waves * 64);
  if (prod && tonly)
    hipLaunchKernelGGL((k_smax_bwd<NC, RuleProd, true>), grid, b, p.lds, st, a, beta, beta2);
  else if (prod)
    hipLaunchKernelGGL((k_smax_bwd<NC, RuleProd, false>), grid, b, p.lds, st, a, beta, beta2);
  else if (tonly)
    hipLaunchKernelGGL((k_smax_bwd<NC, RuleAcc, true>), grid, b, p.lds, st, a, beta, beta2);
  else
    hipLaunchKernelGGL((k_smax_bwd<NC, RuleAcc, false>), grid, b, p.lds, st, a, beta, beta2);
}

}  // namespace

bool smax_supported(const DatasetRec &ds, const PopRec &pop) {
  return ds.nc <= kSmaxMaxClasses && plan_smax_backward(ds, pop).lds <= kDynLdsMax &&
         plan_smax_forward(ds, pop).lds <= kDynLdsMax;
}

hipError_t launch_smax_forward(const SoftLaunch &l, float beta, hipStream_t st) {
  const PopRec &pop = *l.pop;
  if (pop.n_sets == 0) return hipSuccess;
  const SoftPlan p = plan_smax_forward(*l.ds, pop);
  SoftArgs a;
  fill_args(a, l, p);
  a.part_loss = static_cast<double *>(l.ws);
  uint4 *crec = reinterpret_cast<uint4 *>(static_cast<char *>(l.ws) + soft_part_bytes(*l.ds, pop, false));
  a.crec = crec;
  hipError_t e = launch_prep(l, a, crec, st);
  if (e != hipSuccess) return e;
  const float beta2 = beta * kLog2e;
  if (p.n_groups > 0) {
    const dim3 grid((unsigned)((pop.n_sets + p.Q - 1) / p.Q), (unsigned)p.n_groups);
    const bool prod = pop.max_rule_conds <= kProdMaxConds, tonly = pop.n_ff == 0 && pop.n_cat == 0;
    switch (smax_nc(l.ds->nc)) {
      case 2: launch_smax_fwd_nc<2>(p, grid, st, a, prod, tonly, beta2); break;
      case 4: launch_smax_fwd_nc<4>(p, grid, st, a, prod, tonly, beta2); break;
      case 8: launch_smax_fwd_nc<8>(p, grid, st, a, prod, tonly, beta2); break;
      default: launch_smax_fwd_nc<16>(p, grid, st, a, prod, tonly, beta2); break;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_soft_fwd_final, dim3((unsigned)((pop.n_sets + 63) / 64)),
                     dim3(kFwdFinalWaves * 64), 0, st,
                     a.part_loss, p.n_groups, pop.n_sets, l.ds->n, l.loss);
  return hipGetLastError();
}

hipError_t launch_smax_backward(const SoftLaunch &l, float beta, hipStream_t st) {
  const PopRec &pop = *l.pop;
  if (pop.n_sets == 0) return hipSuccess;
  const SoftPlan p = plan_smax_backward(*l.ds, pop);
  if (p.lds > kDynLdsMax) return hipErrorInvalidValue;
  SoftArgs a;
  fill_args(a, l, p);
  a.part_grad = static_cast<float *>(l.ws);
  uint4 *crec = reinterpret_cast<uint4 *>(static_cast<char *>(l.ws) + soft_part_bytes(*l.ds, pop, true));
  a.crec = crec;
  hipError_t e = launch_prep(l, a, crec, st);
  if (e != hipSuccess) return e;
  const float beta2 = beta * kLog2e;
  if (p.n_groups > 0) {
    const dim3 grid((unsigned)((pop.n_sets + p.Q - 1) / p.Q), (unsigned)p.n_groups);
    const bool prod = pop.max_rule_conds <= kProdMaxConds, tonly = pop.n_ff == 0 && pop.n_cat == 0;
    switch (smax_nc(l.ds->nc)) {
      case 2: launch_smax_bwd_nc<2>(p, grid, st, a, prod, tonly, beta, beta2); break;
      case 4: launch_smax_bwd_nc<4>(p, grid, st, a, prod, tonly, beta, beta2); break;
      case 8: launch_smax_bwd_nc<8>(p, grid, st, a, prod, tonly, beta, beta2); break;
      default: launch_smax_bwd_nc<16>(p, grid, st, a, prod, tonly, beta, beta2); break;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_soft_bwd_final, dim3((unsigned)pop.n_sets), dim3(64), 0, st, a.part_grad,
                     p.n_groups, pop.n_conds, pop.ssets, pop.sconds, l.ds->inv_tau, l.dloss,
                     l.ds->n, l.dcoef, l.dcoef2, l.dtheta);
  return hipGetLastError();
}

hipError_t launch_smax_proba(const SoftLaunch &l, int32_t set, float beta, const float *rows,
                             int64_t n, float *probs, hipStream_t st) {
  const PopRec &pop = *l.pop;
  if (n <= 0) return hipSuccess;
  SoftArgs a;
  fill_args(a, l, plan_forward(*l.ds, pop));
  uint4 *crec = reinterpret_cast<uint4 *>(static_cast<char *>(l.ws) + soft_part_bytes(*l.ds, pop, false));
  a.crec = crec;
  hipError_t e = launch_prep(l, a, crec, st);
  if (e != hipSuccess) return e;
  const float beta2 = beta * kLog2e;
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  const int nc = l.ds->nc;
  switch (smax_nc(nc)) {
    case 2:
      hipLaunchKernelGGL(k_smax_proba<2>, grid, block, 0, st, rows, n, pop.nf, nc, set, pop.sets,
                         pop.ssets, pop.rules, crec, beta2, probs);
      break;
    case 4:
      hipLaunchKernelGGL(k_smax_proba<4>, grid, block, 0, st, rows, n, pop.nf, nc, set, pop.sets,
                         pop.ssets, pop.rules, crec, beta2, probs);
      break;
    case 8:
      hipLaunchKernelGGL(k_smax_proba<8>, grid, block, 0, st, rows, n, pop.nf, nc, set, pop.sets,
                         pop.ssets, pop.rules, crec, beta2, probs);
      break;
    default:
      hipLaunchKernelGGL(k_smax_proba<16>, grid, block, 0, st, rows, n, pop.nf, nc, set, pop.sets,
                         pop.ssets, pop.rules, crec, beta2, probs);
      break;
  }
  return hipGetLastError();
}

namespace {
// Scratch of the no-allocation soft forward: one copy per GPU, loaded with the
// code object.  On the host this name is only a stand-in for the symbol;
// kernels receive the device address hipGetSymbolAddress gives for it.
static __device__ __align__(256) unsigned char scratch[AERL_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(int device, void **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (!g_scratch_ptr[device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

hipError_t launch_soft_backward(const SoftLaunch &l, hipStream_t st) {
  const PopRec &pop = *l.pop;
  if (pop.n_sets == 0) return hipSuccess;
  const SoftPlan p = plan_backward(*l.ds, pop);
  if (p.lds > kDynLdsMax) return hipErrorInvalidValue;
  SoftArgs a;
  fill_args(a, l, p);
  a.part_grad = static_cast<float *>(l.ws);
  uint4 *crec = reinterpret_cast<uint4 *>(static_cast<char *>(l.ws) + soft_part_bytes(*l.ds, pop, true));
  a.crec = crec;
  hipError_t e0 = launch_prep(l, a, crec, st);
  if (e0 != hipSuccess) return e0;
  if (p.n_groups > 0) {
    const dim3 grid((unsigned)((pop.n_sets + p.Q - 1) / p.Q), (unsigned)p.n_groups);
    const bool prod = pop.max_rule_conds <= kProdMaxConds, tonly = pop.n_ff == 0 && pop.n_cat == 0;
    if (p.rmax > 0 && prod && tonly) {
      launch_bwd_reg<RuleProd, true>(p, grid, st, a);
    } else if (p.rmax > 0 && prod) {
      launch_bwd_reg<RuleProd, false>(p, grid, st, a);
    } else if (p.rmax > 0 && tonly) {
      launch_bwd_reg<RuleAcc, true>(p, grid, st, a);
    } else if (p.rmax > 0) {
      launch_bwd_reg<RuleAcc, false>(p, grid, st, a);
    } else {
      hipLaunchKernelGGL(k_soft_bwd, grid, dim3(p.waves * 64), p.lds, st, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_soft_bwd_final, dim3((unsigned)pop.n_sets), dim3(64), 0, st, a.part_grad,
                     p.n_groups, pop.n_conds, pop.ssets, pop.sconds, l.ds->inv_tau, l.dloss,
                     l.ds->n, l.dcoef, l.dcoef2, l.dtheta);
  return hipGetLastError();
}

}  // namespace aerl
