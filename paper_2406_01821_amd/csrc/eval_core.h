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
//   threshold:        a*x[f] >  b
//   feature (gt):     a*x[f] >  b*x[g]
//   feature (ge):     a*x[f] >= b*x[g]
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
// sample is real.
// COUNT mode (PRED = false): returns, in lane c, the number of the tile's
//   real samples predicted as class c.
// PRED mode: pred[s] receives the predicted class of each lane's samples.
// Portable form (any S, both modes); the 4-slot counting path below is the
// same loop written for the scalar unit by hand.
template <int S, bool PRED>
__device__ __forceinline__ int eval_set(const float *__restrict__ xs, int lane, int4 set,
                                        const uint4 *__restrict__ stream,
                                        const uint64_t (&vm)[S], int (&pred)[S]) {
  uint64_t und[S], fire[S];
#pragma unroll
  for (int s = 0; s < S; ++s) und[s] = fire[s] = vm[s];
  int acc = 0;
  const uint4 *base = stream + set.x;
  uint32_t end = (uint32_t)set.y * 16u;
  uint32_t o = 0;
  bool decided = false;
  while (o < end) {
    const uint4 r = ldc_at(base, o);
    const float ca = __uint_as_float(r.y), cb = __uint_as_float(r.z);
    uint64_t m[S];
    if ((r.w & kRecFF) == 0) {
      float v[S];
      load_row<S>(xs, r.x, lane, v);
#pragma unroll
      for (int s = 0; s < S; ++s) m[s] = ballot(ca * v[s] > cb);
    } else {
      float v1[S], v2[S];
      load_row<S>(xs, r.x, lane, v1);
      load_row<S>(xs, (r.w & kRecGMask) * 1024u, lane, v2);
      const bool ge = (r.w & kRecGE) != 0;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const float p = ca * v1[s], q = cb * v2[s];
        m[s] = ge ? ballot(p >= q) : ballot(p > q);
      }
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
      if (left == 0) {  // every lane decided
        decided = true;
        next = end;
      }
    }
    o = next;
  }
  if (!decided) {
    int nleft = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if constexpr (PRED) {
        if ((und[s] >> lane) & 1ull) pred[s] = set.z;
      }
      nleft += __builtin_popcountll(und[s]);
    }
    if constexpr (!PRED) acc += (lane == set.z) ? nleft : 0;
  }
  return acc;
}

// 4-slot counting evaluation written for the scalar unit.  Same semantics as
// eval_set<4, false>.  Records are loaded two at a time (s_load_dwordx8
// into quads A = s[64:67] and B = s[68:71]): the record after the current
// one arrives with it, so a rule that goes on past an A record, or a rule
// that starts right after one, continues without another scalar load or
// wait.  The record after a rule set's last one lies inside the packed
// stream (it ends with a spare record).  Every load is waited on inside the
// asm block.  v[32:39] hold the feature values of the lane's four samples
// (two rows for feature-vs-feature records).
//   lds_lane: LDS byte address of the tile plus lane*16.

// Threshold record (a in Y, b in Z): f_i = S_i & (b < a*x_i).  The compare
// masks go through two temporaries (m and vcc), alternating, so that each
// AND waits only for its own compare; f0 is written last, so SCC = (f0 != 0).
#define AERL_T_BODY(Y, Z, S0, S1, S2, S3)               \
  "s_waitcnt lgkmcnt(0)\n"                              \
  "v_mul_f32 v32, " Y ", v32\n"                         \
  "v_mul_f32 v33, " Y ", v33\n"                         \
  "v_mul_f32 v34, " Y ", v34\n"                         \
  "v_mul_f32 v35, " Y ", v35\n"                         \
  "v_cmp_lt_f32_e64 %[m], " Z ", v35\n"                 \
  "v_cmp_lt_f32_e32 vcc, " Z ", v34\n"                  \
  "s_and_b64 %[f3], " S3 ", %[m]\n"                     \
  "v_cmp_lt_f32_e64 %[m], " Z ", v33\n"                 \
  "s_and_b64 %[f2], " S2 ", vcc\n"                      \
  "v_cmp_lt_f32_e32 vcc, " Z ", v32\n"                  \
  "s_and_b64 %[f1], " S1 ", %[m]\n"                     \
  "s_and_b64 %[f0], " S0 ", vcc\n"

#define AERL_FF_CMP(OP, S0, S1, S2, S3)                 \
  "v_cmp_" OP "_f32_e64 %[m], v35, v39\n"               \
  "v_cmp_" OP "_f32_e32 vcc, v34, v38\n"                \
  "s_and_b64 %[f3], " S3 ", %[m]\n"                     \
  "v_cmp_" OP "_f32_e64 %[m], v33, v37\n"               \
  "s_and_b64 %[f2], " S2 ", vcc\n"                      \
  "v_cmp_" OP "_f32_e32 vcc, v32, v36\n"                \
  "s_and_b64 %[f1], " S1 ", %[m]\n"                     \
  "s_and_b64 %[f0], " S0 ", vcc\n"

// Feature-vs-feature record (a in Y, b in Z, g and the >= flag in W):
// f_i = S_i & (a*x_i > b*x'_i) or (>=); then on to POST.
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

// Record in quad X at offset o: read its feature row, then compare
// (threshold inline, feature-vs-feature at FFL).
#define AERL_RECORD(XX, XY, XZ, XW, S0, S1, S2, S3, FFL) \
  "v_add_u32 %[vt], " XX ", %[lds]\n"                   \
  "ds_read_b128 v[32:35], %[vt]\n"                      \
  "s_bitcmp1_b32 " XW ", 9\n"                           \
  "s_cbranch_scc1 " FFL "\n"                            \
  AERL_T_BODY(XY, XZ, S0, S1, S2, S3)

#define AERL_POPC4(A, B, C, D)                          \
  "s_bcnt1_i32_b64 %[t0], " A "\n"                      \
  "s_bcnt1_i32_b64 %[t1], " B "\n"                      \
  "s_add_u32 %[t0], %[t0], %[t1]\n"                     \
  "s_bcnt1_i32_b64 %[t1], " C "\n"                      \
  "s_add_u32 %[t0], %[t0], %[t1]\n"                     \
  "s_bcnt1_i32_b64 %[t1], " D "\n"                      \
  "s_add_u32 %[t0], %[t0], %[t1]\n"

// The rule of the (last) record in W fires for the lanes in f: count them
// for its class and retire them (SCC = some lane still undecided).
#define AERL_COMMIT_COUNT(W)                            \
  AERL_POPC4("%[f0]", "%[f1]", "%[f2]", "%[f3]")        \
  "s_bfe_u32 %[t1], " W ", 0x6000c\n"                   \
  "v_cmp_eq_u32_e32 vcc, %[t1], %[lane]\n"              \
  "v_mov_b32 %[vt], %[t0]\n"                            \
  "v_cndmask_b32_e32 %[vt], 0, %[vt], vcc\n"            \
  "v_add_u32 %[acc], %[acc], %[vt]\n"                   \
  "s_andn2_b64 %[u0], %[u0], %[f0]\n"                   \
  "s_andn2_b64 %[u1], %[u1], %[f1]\n"                   \
  "s_andn2_b64 %[u2], %[u2], %[f2]\n"                   \
  "s_andn2_b64 %[u3], %[u3], %[f3]\n"                   \
  "s_or_b64 %[m], %[u0], %[u1]\n"                       \
  "s_or_b64 %[m], %[m], %[u2]\n"                        \
  "s_or_b64 %[m], %[m], %[u3]\n"

// SCC = (f0 != 0) after a compare; true when any f_i is non-zero.
#define AERL_ANY_F(ALIVE)                               \
  "s_cbranch_scc1 " ALIVE "\n"                          \
  "s_or_b64 %[m], %[f1], %[f2]\n"                      \
  "s_or_b64 %[m], %[m], %[f3]\n"                      \
  "s_cbranch_scc1 " ALIVE "\n"

#define AERL_U "%[u0]", "%[u1]", "%[u2]", "%[u3]"
#define AERL_F "%[f0]", "%[f1]", "%[f2]", "%[f3]"
#define AERL_RECORD_X(...) AERL_RECORD(__VA_ARGS__)
#define AERL_FF_BODY_X(...) AERL_FF_BODY(__VA_ARGS__)

__device__ __forceinline__ int eval_set_s4_count(uint32_t lds_lane, int lane, int4 set,
                                                 const uint4 *__restrict__ stream,
                                                 const uint64_t (&vm)[4]) {
  const uint4 *base = stream + set.x;
  const uint32_t end = (uint32_t)set.y * 16u;
  const int dflt = set.z;
  uint64_t u0 = vm[0], u1 = vm[1], u2 = vm[2], u3 = vm[3];
  uint64_t f0, f1, f2, f3, m;
  uint32_t o, t0, t1, vt, vt2;
  int acc = 0;
  asm volatile(
      "s_mov_b32 %[o], 0\n"
      "s_cmp_eq_u32 %[end], 0\n"
      "s_cbranch_scc1 .Ldefault_%=\n"
      // load the pair (o, o+16) into A, B
      ".Lfirst_%=:\n"
      "s_load_dwordx8 s[64:71], %[base], %[o]\n"
      "s_waitcnt lgkmcnt(0)\n"
      // first record of a rule in A: f = undecided & m
      ".Lstart_A_%=:\n"
      AERL_RECORD_X("s64", "s65", "s66", "s67", AERL_U, ".Lffs_A_%=")
      // after a record in A
      ".Lpost_A_%=:\n"
      AERL_ANY_F(".Lalive_A_%=")
      // the rule cannot fire for any undecided lane: next rule
      "s_lshr_b32 %[t1], s67, 18\n"
      "s_add_u32 %[t0], %[o], 16\n"
      "s_cmp_ge_u32 %[t1], %[end]\n"
      "s_cbranch_scc1 .Ldefault_%=\n"
      "s_cmp_eq_u32 %[t1], %[t0]\n"
      "s_mov_b32 %[o], %[t1]\n"
      "s_cbranch_scc1 .Lstart_B_%=\n"
      "s_branch .Lfirst_%=\n"
      ".Lalive_A_%=:\n"
      "s_bitcmp1_b32 s67, 11\n"
      "s_cbranch_scc1 .Lcommit_A_%=\n"
      "s_add_u32 %[o], %[o], 16\n"
      // later record of the same rule in B: f &= m
      ".Lnext_B_%=:\n"
      AERL_RECORD_X("s68", "s69", "s70", "s71", AERL_F, ".Lffn_B_%=")
      // after a record in B
      ".Lpost_B_%=:\n"
      AERL_ANY_F(".Lalive_B_%=")
      "s_lshr_b32 %[o], s71, 18\n"
      "s_cmp_lt_u32 %[o], %[end]\n"
      "s_cbranch_scc1 .Lfirst_%=\n"
      "s_branch .Ldefault_%=\n"
      ".Lalive_B_%=:\n"
      "s_bitcmp1_b32 s71, 11\n"
      "s_cbranch_scc1 .Lcommit_B_%=\n"
      "s_add_u32 %[o], %[o], 16\n"
      "s_load_dwordx8 s[64:71], %[base], %[o]\n"
      "s_waitcnt lgkmcnt(0)\n"
      // later record of the same rule in A
      AERL_RECORD_X("s64", "s65", "s66", "s67", AERL_F, ".Lffn_A_%=")
      "s_branch .Lpost_A_%=\n"
      // first record of a rule in B
      ".Lstart_B_%=:\n"
      AERL_RECORD_X("s68", "s69", "s70", "s71", AERL_U, ".Lffs_B_%=")
      "s_branch .Lpost_B_%=\n"
      ".Lffs_A_%=:\n"
      AERL_FF_BODY_X("s67", "s65", "s66", AERL_U, "sA", ".Lpost_A_%=")
      ".Lffn_A_%=:\n"
      AERL_FF_BODY_X("s67", "s65", "s66", AERL_F, "nA", ".Lpost_A_%=")
      ".Lffs_B_%=:\n"
      AERL_FF_BODY_X("s71", "s69", "s70", AERL_U, "sB", ".Lpost_B_%=")
      ".Lffn_B_%=:\n"
      AERL_FF_BODY_X("s71", "s69", "s70", AERL_F, "nB", ".Lpost_B_%=")
      // the rule of the record in A fires; the next rule starts with B
      ".Lcommit_A_%=:\n"
      AERL_COMMIT_COUNT("s67")
      "s_cbranch_scc0 .Ldone_%=\n"
      "s_add_u32 %[o], %[o], 16\n"
      "s_cmp_lt_u32 %[o], %[end]\n"
      "s_cbranch_scc1 .Lstart_B_%=\n"
      "s_branch .Ldefault_%=\n"
      // the rule of the record in B fires; the next rule needs a new pair
      ".Lcommit_B_%=:\n"
      AERL_COMMIT_COUNT("s71")
      "s_cbranch_scc0 .Ldone_%=\n"
      "s_add_u32 %[o], %[o], 16\n"
      "s_cmp_lt_u32 %[o], %[end]\n"
      "s_cbranch_scc1 .Lfirst_%=\n"
      // no rule fired for the remaining lanes: default class
      ".Ldefault_%=:\n"
      AERL_POPC4("%[u0]", "%[u1]", "%[u2]", "%[u3]")
      "v_cmp_eq_u32_e32 vcc, %[dflt], %[lane]\n"
      "v_mov_b32 %[vt], %[t0]\n"
      "v_cndmask_b32_e32 %[vt], 0, %[vt], vcc\n"
      "v_add_u32 %[acc], %[acc], %[vt]\n"
      ".Ldone_%=:\n"
      : [acc] "+v"(acc), [u0] "+s"(u0), [u1] "+s"(u1), [u2] "+s"(u2), [u3] "+s"(u3),
        [f0] "=&s"(f0), [f1] "=&s"(f1), [f2] "=&s"(f2), [f3] "=&s"(f3), [m] "=&s"(m), [o] "=&s"(o), [t0] "=&s"(t0),
        [t1] "=&s"(t1), [vt] "=&v"(vt), [vt2] "=&v"(vt2)
      : [base] "s"(base), [end] "s"(end), [dflt] "s"(dflt), [lds] "v"(lds_lane),
        [lane] "v"(lane)
      : "s64", "s65", "s66", "s67", "s68", "s69", "s70", "s71", "v32", "v33", "v34", "v35",
        "v36", "v37", "v38", "v39", "vcc", "scc", "memory");
  return acc;
}

}  // namespace aerl
