// Device-side core of hard (step-activation) rule-set evaluation.
//
// One sample per wave64 lane (S samples per lane, S in {1, 2, 4}); the
// samples of the current tile sit feature-major in LDS, so the value of
// feature f for a lane's S samples is one ds_read of 4*S bytes.  Rule
// parameters are wave-uniform (scalar loads into SGPRs).  For every rule the
// wave keeps one 64-bit lane mask per sample slot ("fire"); a condition ANDs
// a ballot into it; the rule is abandoned as soon as no undecided lane can
// still fire it; lanes whose rule fired leave the "undecided" masks (first
// firing rule wins, Fig. 1b), and the rule set stops once every lane is
// decided.  Counts come from popcounts of the fire masks.
//
// Condition forms after packing (all exact rewrites of the caller's form):
//   threshold:        x[f] >= t  or  x[f] <= t  (t folded on the host from
//                     the fp32 product and the threshold), or a*x[f] > b
//                     when the coefficient is zero
//   feature (gt):     a*x[f] >  b*x[g]
//   feature (ge):     a*x[f] >= b*x[g]
//   always:           empty rules and the set's closing default rule
// Every product is one IEEE fp32 multiply (no contraction), compared as is.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace aerl {

// LDS tile row of S*64 samples for one feature: lane holds samples
// S*lane .. S*lane+S-1.  `off4` is the row's byte offset in a 256-sample
// (S = 4) tile, i.e. feature * 1024; smaller tiles scale it down.
template <int S>
__device__ __forceinline__ void load_row(const float *__restrict__ xs, uint32_t off4, int lane,
                                         float (&v)[S]) {
  constexpr uint32_t shift = S == 4 ? 0 : (S == 2 ? 1 : 2);
  const char *p = reinterpret_cast<const char *>(xs) + (off4 >> shift) + (uint32_t)lane * (4u * S);
  if constexpr (S == 4) {
    const float4 t = *reinterpret_cast<const float4 *>(p);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  } else if constexpr (S == 2) {
    const float2 t = *reinterpret_cast<const float2 *>(p);
    v[0] = t.x; v[1] = t.y;
  } else {
    v[0] = *reinterpret_cast<const float *>(p);
  }
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Next work item of a wave from an LDS counter.  Every lane of the (fully
// active) wave adds 1 and the first lane's old value / 64 is the item: no
// divergent region, so the surrounding loop stays a uniform loop.
__device__ __forceinline__ int next_item(int32_t *ctr) {
  return __builtin_amdgcn_readfirstlane(atomicAdd(ctr, 1)) >> 6;
}

// Wave-uniform read through the constant address space, so that the compiler
// issues a scalar load into SGPRs (read-only data: packed rule records).
// T is a 4- or 16-byte POD (int, int4, uint4).
template <class T>
__device__ __forceinline__ T ldc_at(const T *p, uint32_t byte_off) {
  typedef uint32_t v4u __attribute__((ext_vector_type(4)));
  typedef const __attribute__((address_space(4))) char *bptr;
  T out;
  if constexpr (sizeof(T) == 16) {
    typedef const __attribute__((address_space(4))) v4u *cptr;
    const v4u v = *(cptr)((bptr)(p) + byte_off);
    __builtin_memcpy(&out, &v, 16);
  } else {
    static_assert(sizeof(T) == 4, "ldc_at: 4- or 16-byte records");
    typedef const __attribute__((address_space(4))) uint32_t *cptr;
    const uint32_t v = *(cptr)((bptr)(p) + byte_off);
    __builtin_memcpy(&out, &v, 4);
  }
  return out;
}

template <class T>
__device__ __forceinline__ T ldc(const T *p, int64_t i) {
  return ldc_at(p + i, 0u);
}

// Evaluates rule set `set` = {first record, record count, default, -} of the
// hard stream for the S*64 samples of the tile.  vm[s]: lanes whose slot-s
// sample is real.  The set's closing record (always true, default class)
// decides every lane no rule fired for.
// COUNT mode (PRED = false): returns, in lane c, the number of the tile's
//   real samples predicted as class c.
// PRED mode: pred[s] receives the predicted class of each lane's samples.
// Portable form (any S, both modes); the 4-slot counting path below is the
// same walk written for the scalar unit by hand.
template <int S, bool PRED>
__device__ __forceinline__ int eval_set(const float *__restrict__ xs, int lane, int4 set,
                                        const uint4 *__restrict__ stream,
                                        const uint64_t (&vm)[S], int (&pred)[S]) {
  uint64_t und[S], fire[S];
#pragma unroll
  for (int s = 0; s < S; ++s) und[s] = fire[s] = vm[s];
  int acc = 0;
  const uint4 *base = stream + set.x;
  const uint32_t end = (uint32_t)set.y * 16u;
  uint32_t o = 0;
  while (o < end) {
    const uint4 r = ldc_at(base, o);
    const float ry = __uint_as_float(r.y), rz = __uint_as_float(r.z);
    uint64_t m[S];
    if (r.w & kRecFF) {
      float v1[S], v2[S];
      load_row<S>(xs, r.x, lane, v1);
      load_row<S>(xs, (r.w & kRecGMask) * 1024u, lane, v2);
      const bool ge = (r.w & kRecGE) != 0;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const float p = ry * v1[s], q = rz * v2[s];
        m[s] = ge ? ballot(p >= q) : ballot(p > q);
      }
    } else if (r.w & kRecAlways) {
#pragma unroll
      for (int s = 0; s < S; ++s) m[s] = ~0ull;
    } else {
      float v[S];
      load_row<S>(xs, r.x, lane, v);
      const bool mul = (r.w & kRecMul) != 0, le = (r.w & kRecLE) != 0;
#pragma unroll
      for (int s = 0; s < S; ++s)
        m[s] = mul ? ballot(ry * v[s] > rz) : le ? ballot(v[s] <= ry) : ballot(v[s] >= ry);
    }
    uint64_t any = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      fire[s] &= m[s];
      any |= fire[s];
    }
    uint32_t next = o + 16u;
    if (any == 0) {  // no undecided lane can fire this rule: next rule
      next = r.w >> kRecNextShift;
#pragma unroll
      for (int s = 0; s < S; ++s) fire[s] = und[s];
    } else if (r.w & kRecLast) {  // the rule fires: commit it
      const int cls = (int)((r.w >> kRecClsShift) & 63u);
      int nfire = 0;
      uint64_t left = 0;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        if constexpr (PRED) {
          if ((fire[s] >> lane) & 1ull) pred[s] = cls;
        }
        nfire += __builtin_popcountll(fire[s]);
        und[s] &= ~fire[s];
        left |= und[s];
        fire[s] = und[s];
      }
      if constexpr (!PRED) acc += (lane == cls) ? nfire : 0;
      if (left == 0) next = end;  // every lane decided
    }
    o = next;
  }
  return acc;
}

// 4-slot counting evaluation written for the scalar unit.  Same semantics as
// eval_set<4, false>.  Records are loaded two at a time (s_load_dwordx8 at
// byte offset o into quads A = s[64:67] and B = s[68:71]): a rule that goes
// on past an A record, or starts right after one, continues from B without
// another scalar load or wait.  The record after a rule set's last one lies
// inside the packed stream (the stream ends with a spare record).
//
// A non-last record with a folded threshold (x >= t or x <= t) takes the
// fast path: one flag test for the special kinds, one for the direction,
// four compares and four mask ANDs.  Special kinds (feature-vs-feature,
// zero coefficient, always true, a rule's last record) branch out to their
// own bodies.  Every walk ends in a commit of an always-true record or with
// no undecided lane left, so no end-of-stream test is needed.  Every load is
// waited on inside the asm block.  v[32:39] hold the feature values of the
// lane's four samples (two rows for feature-vs-feature records).
//   lds_lane: LDS byte address of the tile plus lane*16.

// Four compares of v32..v35 (or of the products in them) against T with
// opcode OP (T op x_i), ANDed into f_i = S_i & m_i.  The masks go through two
// temporaries (m and vcc), alternating, so that each AND waits only for its
// own compare; f0 is written last, so SCC = (f0 != 0).
#define AERL_CMP4(OP, T, S0, S1, S2, S3)                \
  "v_cmp_" OP "_f32_e64 %[m], " T ", v35\n"             \
  "v_cmp_" OP "_f32_e32 vcc, " T ", v34\n"              \
  "s_and_b64 %[f3], " S3 ", %[m]\n"                     \
  "v_cmp_" OP "_f32_e64 %[m], " T ", v33\n"             \
  "s_and_b64 %[f2], " S2 ", vcc\n"                      \
  "v_cmp_" OP "_f32_e32 vcc, " T ", v32\n"              \
  "s_and_b64 %[f1], " S1 ", %[m]\n"                     \
  "s_and_b64 %[f0], " S0 ", vcc\n"

// Feature-vs-feature compare of the products in v32..v35 and v36..v39.
#define AERL_FF_CMP(OP, S0, S1, S2, S3)                 \
  "v_cmp_" OP "_f32_e64 %[m], v35, v39\n"               \
  "v_cmp_" OP "_f32_e32 vcc, v34, v38\n"                \
  "s_and_b64 %[f3], " S3 ", %[m]\n"                     \
  "v_cmp_" OP "_f32_e64 %[m], v33, v37\n"               \
  "s_and_b64 %[f2], " S2 ", vcc\n"                      \
  "v_cmp_" OP "_f32_e32 vcc, v32, v36\n"                \
  "s_and_b64 %[f1], " S1 ", %[m]\n"                     \
  "s_and_b64 %[f0], " S0 ", vcc\n"

// Start of a record whose row is at byte offset XX: read the row; special
// kinds go to SPEC, the <= direction to LE; falls through (row waited for)
// with a >= record.  kRecSpecial = 0xa03, kRecLE = bit 10.
#define AERL_FETCH(XX, XW, SPEC, LE)                    \
  "v_add_u32 %[vt], " XX ", %[lds]\n"                   \
  "ds_read_b128 v[32:35], %[vt]\n"                      \
  "s_and_b32 %[t0], " XW ", 0xa03\n"                    \
  "s_cbranch_scc1 " SPEC "\n"                           \
  "s_bitcmp1_b32 " XW ", 10\n"                          \
  "s_waitcnt lgkmcnt(0)\n"                              \
  "s_cbranch_scc1 " LE "\n"

// Special threshold kinds of the record (y in Y, z in Z, flags in W), row
// already requested: zero coefficient (y*x > z), <=, or >= (a last record);
// then on to POST with SCC = (f0 != 0).
#define AERL_TSPEC(Y, Z, W, S0, S1, S2, S3, TAG, POST)  \
  "s_waitcnt lgkmcnt(0)\n"                              \
  "s_bitcmp1_b32 " W ", 0\n"                            \
  "s_cbranch_scc1 .Lmul_" TAG "_%=\n"                   \
  "s_bitcmp1_b32 " W ", 10\n"                           \
  "s_cbranch_scc1 .Lle_" TAG "_%=\n"                    \
  AERL_CMP4("le", Y, S0, S1, S2, S3)                    \
  "s_branch " POST "\n"                                 \
  ".Lle_" TAG "_%=:\n"                                  \
  AERL_CMP4("ge", Y, S0, S1, S2, S3)                    \
  "s_branch " POST "\n"                                 \
  ".Lmul_" TAG "_%=:\n"                                 \
  "v_mul_f32 v32, " Y ", v32\n"                         \
  "v_mul_f32 v33, " Y ", v33\n"                         \
  "v_mul_f32 v34, " Y ", v34\n"                         \
  "v_mul_f32 v35, " Y ", v35\n"                         \
  AERL_CMP4("lt", Z, S0, S1, S2, S3)                    \
  "s_branch " POST "\n"

// Feature-vs-feature record (a in Y, b in Z, g and the >= flag in W), first
// row already requested: f_i = S_i & (a*x_i > b*x'_i) or (>=); then POST.
#define AERL_FF_BODY(W, Y, Z, S0, S1, S2, S3, TAG, POST) \
  "s_bfe_u32 %[t0], " W ", 0x90000\n"                   \
  "s_lshl_b32 %[t0], %[t0], 10\n"                       \
  "v_add_u32 %[vt2], %[t0], %[lds]\n"                   \
  "ds_read_b128 v[36:39], %[vt2]\n"                     \
  "s_waitcnt lgkmcnt(0)\n"                              \
  "v_mul_f32 v32, " Y ", v32\n"                         \
  "v_mul_f32 v33, " Y ", v33\n"                         \
  "v_mul_f32 v34, " Y ", v34\n"                         \
  "v_mul_f32 v35, " Y ", v35\n"                         \
  "v_mul_f32 v36, " Z ", v36\n"                         \
  "v_mul_f32 v37, " Z ", v37\n"                         \
  "v_mul_f32 v38, " Z ", v38\n"                         \
  "v_mul_f32 v39, " Z ", v39\n"                         \
  "s_bitcmp1_b32 " W ", 10\n"                           \
  "s_cbranch_scc1 .Lge_" TAG "_%=\n"                    \
  AERL_FF_CMP("gt", S0, S1, S2, S3)                     \
  "s_branch " POST "\n"                                 \
  ".Lge_" TAG "_%=:\n"                                  \
  AERL_FF_CMP("ge", S0, S1, S2, S3)                     \
  "s_branch " POST "\n"

// Special record entry: feature-vs-feature to FFL, always-true (rule starts
// only) to ALW, else a special threshold kind; then POST.
#define AERL_SPEC(Y, Z, W, S0, S1, S2, S3, TAG, POST, ALW) \
  "s_bitcmp1_b32 " W ", 9\n"                            \
  "s_cbranch_scc1 .Lff_" TAG "_%=\n"                    \
  ALW                                                   \
  AERL_TSPEC(Y, Z, W, S0, S1, S2, S3, TAG, POST)        \
  ".Lff_" TAG "_%=:\n"                                  \
  AERL_FF_BODY(W, Y, Z, S0, S1, S2, S3, TAG, POST)

#define AERL_POPC4(A, B, C, D)                          \
  "s_bcnt1_i32_b64 %[t0], " A "\n"                      \
  "s_bcnt1_i32_b64 %[t1], " B "\n"                      \
  "s_add_u32 %[t0], %[t0], %[t1]\n"                     \
  "s_bcnt1_i32_b64 %[t1], " C "\n"                      \
  "s_add_u32 %[t0], %[t0], %[t1]\n"                     \
  "s_bcnt1_i32_b64 %[t1], " D "\n"                      \
  "s_add_u32 %[t0], %[t0], %[t1]\n"

// Adds the t0 samples of the class in W to the class's lane of acc.
#define AERL_ADD_CLASS(W)                               \
  "s_bfe_u32 %[t1], " W ", 0x6000c\n"                   \
  "v_cmp_eq_u32_e32 vcc, %[t1], %[lane]\n"              \
  "v_mov_b32 %[vt], %[t0]\n"                            \
  "v_cndmask_b32_e32 %[vt], 0, %[vt], vcc\n"            \
  "v_add_u32 %[acc], %[acc], %[vt]\n"

// The rule of the (last) record in W fires for the lanes in f: count them
// for its class and retire them (SCC = some lane still undecided).
#define AERL_COMMIT_COUNT(W)                            \
  AERL_POPC4("%[f0]", "%[f1]", "%[f2]", "%[f3]")        \
  AERL_ADD_CLASS(W)                                     \
  "s_andn2_b64 %[u0], %[u0], %[f0]\n"                   \
  "s_andn2_b64 %[u1], %[u1], %[f1]\n"                   \
  "s_andn2_b64 %[u2], %[u2], %[f2]\n"                   \
  "s_andn2_b64 %[u3], %[u3], %[f3]\n"                   \
  "s_or_b64 %[m], %[u0], %[u1]\n"                       \
  "s_or_b64 %[m], %[m], %[u2]\n"                        \
  "s_or_b64 %[m], %[m], %[u3]\n"

// SCC = (f0 != 0) after a compare: to ALIVE when some f_i is non-zero.
#define AERL_ANY_F(ALIVE)                               \
  "s_cbranch_scc1 " ALIVE "\n"                          \
  "s_or_b64 %[m], %[f1], %[f2]\n"                       \
  "s_or_b64 %[m], %[m], %[f3]\n"                        \
  "s_cbranch_scc1 " ALIVE "\n"

#define AERL_U "%[u0]", "%[u1]", "%[u2]", "%[u3]"
#define AERL_F "%[f0]", "%[f1]", "%[f2]", "%[f3]"
#define AERL_X(M, ...) M(__VA_ARGS__)

__device__ __forceinline__ int eval_set_s4_count(uint32_t lds_lane, int lane, int4 set,
                                                 const uint4 *__restrict__ stream,
                                                 const uint64_t (&vm)[4]) {
  const uint4 *base = stream + set.x;
  uint64_t u0 = vm[0], u1 = vm[1], u2 = vm[2], u3 = vm[3];
  uint64_t f0, f1, f2, f3, m;
  uint32_t o, t0, t1, vt, vt2;
  int acc = 0;
  asm volatile(
      "s_mov_b32 %[o], 0\n"
      "s_or_b64 %[m], %[u0], %[u1]\n"
      "s_or_b64 %[m], %[m], %[u2]\n"
      "s_or_b64 %[m], %[m], %[u3]\n"
      "s_cbranch_scc0 .Ldone_%=\n"
      // load the pair (o, o+16) into A, B; a rule starts at A
      ".Lload_%=:\n"
      "s_load_dwordx8 s[64:71], %[base], %[o]\n"
      "s_waitcnt lgkmcnt(0)\n"
      AERL_X(AERL_FETCH, "s64", "s67", ".Lpsa_%=", ".Llsa_%=")
      AERL_X(AERL_CMP4, "le", "s65", AERL_U)
      // after a fast record in A: on with B unless no f_i fires
      ".Lqa_%=:\n"
      "s_cbranch_scc0 .Lka_%=\n"
      // B continues the rule
      ".Lnb_%=:\n"
      AERL_X(AERL_FETCH, "s68", "s71", ".Lpnb_%=", ".Llnb_%=")
      AERL_X(AERL_CMP4, "le", "s69", AERL_F)
      ".Lqb_%=:\n"
      "s_cbranch_scc0 .Lkb_%=\n"
      // the next pair continues the rule
      ".Llna_load_%=:\n"
      "s_add_u32 %[o], %[o], 32\n"
      "s_load_dwordx8 s[64:71], %[base], %[o]\n"
      "s_waitcnt lgkmcnt(0)\n"
      AERL_X(AERL_FETCH, "s64", "s67", ".Lpna_%=", ".Llna_%=")
      AERL_X(AERL_CMP4, "le", "s65", AERL_F)
      "s_cbranch_scc1 .Lnb_%=\n"
      // f0 == 0 after a fast record in A: alive if another slot fires, else
      // the next rule starts past B (A is not a rule's last record)
      ".Lka_%=:\n"
      "s_or_b64 %[m], %[f1], %[f2]\n"
      "s_or_b64 %[m], %[m], %[f3]\n"
      "s_cbranch_scc1 .Lnb_%=\n"
      "s_lshr_b32 %[o], s67, 18\n"
      "s_branch .Lload_%=\n"
      ".Lkb_%=:\n"
      "s_or_b64 %[m], %[f1], %[f2]\n"
      "s_or_b64 %[m], %[m], %[f3]\n"
      "s_cbranch_scc1 .Llna_load_%=\n"
      "s_lshr_b32 %[o], s71, 18\n"
      "s_branch .Lload_%=\n"
      // a rule starts at B (the previous one ended at A)
      ".Lsb_%=:\n"
      AERL_X(AERL_FETCH, "s68", "s71", ".Lpsb_%=", ".Llsb_%=")
      AERL_X(AERL_CMP4, "le", "s69", AERL_U)
      "s_branch .Lqb_%=\n"
      // fast records in the <= direction
      ".Llsa_%=:\n"
      AERL_X(AERL_CMP4, "ge", "s65", AERL_U)
      "s_branch .Lqa_%=\n"
      ".Llna_%=:\n"
      AERL_X(AERL_CMP4, "ge", "s65", AERL_F)
      "s_branch .Lqa_%=\n"
      ".Llsb_%=:\n"
      AERL_X(AERL_CMP4, "ge", "s69", AERL_U)
      "s_branch .Lqb_%=\n"
      ".Llnb_%=:\n"
      AERL_X(AERL_CMP4, "ge", "s69", AERL_F)
      "s_branch .Lqb_%=\n"
      // special records
      ".Lpsa_%=:\n"
      AERL_X(AERL_SPEC, "s65", "s66", "s67", AERL_U, "sa", ".Lxa_%=",
             "s_bitcmp1_b32 s67, 1\n s_cbranch_scc1 .Lalwa_%=\n")
      ".Lpna_%=:\n"
      AERL_X(AERL_SPEC, "s65", "s66", "s67", AERL_F, "na", ".Lxa_%=", "")
      ".Lpsb_%=:\n"
      AERL_X(AERL_SPEC, "s69", "s70", "s71", AERL_U, "sb", ".Lxb_%=",
             "s_bitcmp1_b32 s71, 1\n s_cbranch_scc1 .Lalwb_%=\n")
      ".Lpnb_%=:\n"
      AERL_X(AERL_SPEC, "s69", "s70", "s71", AERL_F, "nb", ".Lxb_%=", "")
      // after a special record in A
      ".Lxa_%=:\n"
      AERL_ANY_F(".Lya_%=")
      "s_bitcmp1_b32 s67, 11\n"
      "s_cbranch_scc1 .Lsb_%=\n"  // dead, and the next rule starts at B
      "s_lshr_b32 %[o], s67, 18\n"
      "s_branch .Lload_%=\n"
      ".Lya_%=:\n"
      "s_bitcmp1_b32 s67, 11\n"
      "s_cbranch_scc0 .Lnb_%=\n"
      AERL_COMMIT_COUNT("s67")
      "s_cbranch_scc1 .Lsb_%=\n"
      "s_branch .Ldone_%=\n"
      // after a special record in B
      ".Lxb_%=:\n"
      AERL_ANY_F(".Lyb_%=")
      "s_lshr_b32 %[o], s71, 18\n"
      "s_branch .Lload_%=\n"
      ".Lyb_%=:\n"
      "s_bitcmp1_b32 s71, 11\n"
      "s_cbranch_scc0 .Llna_load_%=\n"
      AERL_COMMIT_COUNT("s71")
      "s_cbranch_scc0 .Ldone_%=\n"
      "s_add_u32 %[o], %[o], 32\n"
      "s_branch .Lload_%=\n"
      // an always-true rule decides every undecided lane
      ".Lalwa_%=:\n"
      "s_waitcnt lgkmcnt(0)\n"
      AERL_POPC4("%[u0]", "%[u1]", "%[u2]", "%[u3]")
      AERL_ADD_CLASS("s67")
      "s_branch .Ldone_%=\n"
      ".Lalwb_%=:\n"
      "s_waitcnt lgkmcnt(0)\n"
      AERL_POPC4("%[u0]", "%[u1]", "%[u2]", "%[u3]")
      AERL_ADD_CLASS("s71")
      ".Ldone_%=:\n"
      : [acc] "+v"(acc), [u0] "+s"(u0), [u1] "+s"(u1), [u2] "+s"(u2), [u3] "+s"(u3),
        [f0] "=&s"(f0), [f1] "=&s"(f1), [f2] "=&s"(f2), [f3] "=&s"(f3), [m] "=&s"(m),
        [o] "=&s"(o), [t0] "=&s"(t0), [t1] "=&s"(t1), [vt] "=&v"(vt), [vt2] "=&v"(vt2)
      : [base] "s"(base), [lds] "v"(lds_lane), [lane] "v"(lane)
      : "s64", "s65", "s66", "s67", "s68", "s69", "s70", "s71", "v32", "v33", "v34", "v35",
        "v36", "v37", "v38", "v39", "vcc", "scc", "memory");
  return acc;
}

}  // namespace aerl
