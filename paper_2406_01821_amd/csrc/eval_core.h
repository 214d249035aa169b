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

// Two consecutive 16-byte records in one 32-byte scalar load.
__device__ __forceinline__ void ldc_pair(const int4 *p, int4 (&out)[2]) {
  typedef int32_t v8i __attribute__((ext_vector_type(8)));
  typedef const __attribute__((address_space(4))) v8i *cptr;
  const v8i v = *(cptr)(p);
  out[0] = make_int4(v[0], v[1], v[2], v[3]);
  out[1] = make_int4(v[4], v[5], v[6], v[7]);
}

// Evaluation of one rule set `set` = {first record, record count, default,
// -} of the hard stream for the S*64 samples of the staged tile.  vm[s]:
// lanes whose slot-s sample is real.  Records are read in order; a
// condition ANDs its compare into the rule's per-slot fire masks; a rule
// whose masks hold no undecided lane is abandoned (its next-rule offset
// says where the next rule starts); a rule that reaches its last record
// with lanes still set fires for them: they take its class and leave the
// undecided masks; the set's closing record (always true, default class)
// decides every lane no rule fired for, and the walk stops as soon as
// every lane is decided.
// Counting evaluation written for the scalar unit, for S = 4, 2 or 1
// samples per lane; returns, in lane c, the number of the tile's real
// samples predicted as class c.  Records are
// loaded two at a time (s_load_dwordx8 at byte offset o into quads
// A = s[64:67] and B = s[68:71]): a rule that goes on past an A record, or
// starts right after one, continues from B without another scalar load or
// wait.  The record after a rule set's last one lies inside the packed
// stream (the stream ends with a spare record).
//
// A non-last record with a folded threshold takes the fast path: one flag
// test, S compares and S mask ANDs.  Inside a rule the >= records come
// before the <= ones, so the walk runs in the >= direction until a rule's
// first <= record (flagged) and in the <= direction to the rule's end.
// Special kinds (feature-vs-feature, zero coefficient, always true, a rule's
// last record) branch out to their own bodies.  Every walk ends in a commit
// of an always-true record or with no undecided lane left, so no
// end-of-stream test is needed (a walk that starts with no undecided lane
// ends at the closing record, counting none).  Every load is waited on
// inside the asm block.  v32.. hold the feature values of the
// lane's S samples, v36.. the second row of a feature-vs-feature record; the
// fire masks live in the fixed pairs s[56:57], s[58:59], ... so that a commit
// can count them 32 bits at a time on the VALU.
//   lds_lane: LDS byte address of the tile plus lane*4*S; record x fields
//   are row offsets in a 256-sample tile (f*1024), scaled down for S < 4.

#define AERL_CAT_(a, b) a##b
#define AERL_CAT(a, b) AERL_CAT_(a, b)
#define AERL_SM(S, MODE) AERL_CAT(S, MODE)

// Row address and read (first row into v32.., second into v36..).
#define AERL_ADDR_4(XX) "v_add_u32 %[vt], " XX ", %[lds]\n"
#define AERL_ADDR_2(XX) "v_lshrrev_b32_e64 %[vt], 1, " XX "\n v_add_u32 %[vt], %[vt], %[lds]\n"
#define AERL_ADDR_1(XX) "v_lshrrev_b32_e64 %[vt], 2, " XX "\n v_add_u32 %[vt], %[vt], %[lds]\n"
#define AERL_RD_4 "ds_read_b128 v[32:35], %[vt]\n"
#define AERL_RD_2 "ds_read_b64 v[32:33], %[vt]\n"
#define AERL_RD_1 "ds_read_b32 v32, %[vt]\n"
#define AERL_RD2_4 "ds_read_b128 v[36:39], %[vt2]\n"
#define AERL_RD2_2 "ds_read_b64 v[36:37], %[vt2]\n"
#define AERL_RD2_1 "ds_read_b32 v36, %[vt2]\n"
#define AERL_GSHIFT_4 "10"
#define AERL_GSHIFT_2 "9"
#define AERL_GSHIFT_1 "8"

// S compares of the first row (or of the products in it) against T with
// opcode OP (T op x_i), ANDed into f_i = src_i & m_i.  The masks go through
// two temporaries (m and vcc), alternating, so that each AND waits only for
// its own compare; f0 is written last, so SCC = (f0 != 0).
#define AERL_CMPT_4(OP, T, S0, S1, S2, S3)              \
  "v_cmp_" OP "_f32_e64 %[m], " T ", v35\n"             \
  "v_cmp_" OP "_f32_e32 vcc, " T ", v34\n"              \
  "s_and_b64 s[62:63], " S3 ", %[m]\n"                     \
  "v_cmp_" OP "_f32_e64 %[m], " T ", v33\n"             \
  "s_and_b64 s[60:61], " S2 ", vcc\n"                      \
  "v_cmp_" OP "_f32_e32 vcc, " T ", v32\n"              \
  "s_and_b64 s[58:59], " S1 ", %[m]\n"                     \
  "s_and_b64 s[56:57], " S0 ", vcc\n"
#define AERL_CMPT_2(OP, T, S0, S1)                      \
  "v_cmp_" OP "_f32_e64 %[m], " T ", v33\n"             \
  "v_cmp_" OP "_f32_e32 vcc, " T ", v32\n"              \
  "s_and_b64 s[58:59], " S1 ", %[m]\n"                     \
  "s_and_b64 s[56:57], " S0 ", vcc\n"
#define AERL_CMPT_1(OP, T, S0)                          \
  "v_cmp_" OP "_f32_e32 vcc, " T ", v32\n"              \
  "s_and_b64 s[56:57], " S0 ", vcc\n"
#define AERL_CMP_4U(OP, T) AERL_CMPT_4(OP, T, "%[u0]", "%[u1]", "%[u2]", "%[u3]")
#define AERL_CMP_4F(OP, T) AERL_CMPT_4(OP, T, "s[56:57]", "s[58:59]", "s[60:61]", "s[62:63]")
#define AERL_CMP_2U(OP, T) AERL_CMPT_2(OP, T, "%[u0]", "%[u1]")
#define AERL_CMP_2F(OP, T) AERL_CMPT_2(OP, T, "s[56:57]", "s[58:59]")
#define AERL_CMP_1U(OP, T) AERL_CMPT_1(OP, T, "%[u0]")
#define AERL_CMP_1F(OP, T) AERL_CMPT_1(OP, T, "s[56:57]")

// Feature-vs-feature compare of the products in v32.. and v36...
#define AERL_FFCMPT_4(OP, S0, S1, S2, S3)               \
  "v_cmp_" OP "_f32_e64 %[m], v35, v39\n"               \
  "v_cmp_" OP "_f32_e32 vcc, v34, v38\n"                \
  "s_and_b64 s[62:63], " S3 ", %[m]\n"                     \
  "v_cmp_" OP "_f32_e64 %[m], v33, v37\n"               \
  "s_and_b64 s[60:61], " S2 ", vcc\n"                      \
  "v_cmp_" OP "_f32_e32 vcc, v32, v36\n"                \
  "s_and_b64 s[58:59], " S1 ", %[m]\n"                     \
  "s_and_b64 s[56:57], " S0 ", vcc\n"
#define AERL_FFCMPT_2(OP, S0, S1)                       \
  "v_cmp_" OP "_f32_e64 %[m], v33, v37\n"               \
  "v_cmp_" OP "_f32_e32 vcc, v32, v36\n"                \
  "s_and_b64 s[58:59], " S1 ", %[m]\n"                     \
  "s_and_b64 s[56:57], " S0 ", vcc\n"
#define AERL_FFCMPT_1(OP, S0)                           \
  "v_cmp_" OP "_f32_e32 vcc, v32, v36\n"                \
  "s_and_b64 s[56:57], " S0 ", vcc\n"
#define AERL_FFCMP_4U(OP) AERL_FFCMPT_4(OP, "%[u0]", "%[u1]", "%[u2]", "%[u3]")
#define AERL_FFCMP_4F(OP) AERL_FFCMPT_4(OP, "s[56:57]", "s[58:59]", "s[60:61]", "s[62:63]")
#define AERL_FFCMP_2U(OP) AERL_FFCMPT_2(OP, "%[u0]", "%[u1]")
#define AERL_FFCMP_2F(OP) AERL_FFCMPT_2(OP, "s[56:57]", "s[58:59]")
#define AERL_FFCMP_1U(OP) AERL_FFCMPT_1(OP, "%[u0]")
#define AERL_FFCMP_1F(OP) AERL_FFCMPT_1(OP, "s[56:57]")

// Products of the first row by Y (and of the second by Z).
#define AERL_MUL1_4(Y)                                  \
  "v_mul_f32 v32, " Y ", v32\n"                         \
  "v_mul_f32 v33, " Y ", v33\n"                         \
  "v_mul_f32 v34, " Y ", v34\n"                         \
  "v_mul_f32 v35, " Y ", v35\n"
#define AERL_MUL1_2(Y) "v_mul_f32 v32, " Y ", v32\n v_mul_f32 v33, " Y ", v33\n"
#define AERL_MUL1_1(Y) "v_mul_f32 v32, " Y ", v32\n"
#define AERL_MUL2_4(Z)                                  \
  "v_mul_f32 v36, " Z ", v36\n"                         \
  "v_mul_f32 v37, " Z ", v37\n"                         \
  "v_mul_f32 v38, " Z ", v38\n"                         \
  "v_mul_f32 v39, " Z ", v39\n"
#define AERL_MUL2_2(Z) "v_mul_f32 v36, " Z ", v36\n v_mul_f32 v37, " Z ", v37\n"
#define AERL_MUL2_1(Z) "v_mul_f32 v36, " Z ", v36\n"

// SCC = (f0 != 0) after a compare: to ALIVE when some f_i is non-zero.
#define AERL_ANY_F_4(ALIVE)                             \
  "s_cbranch_scc1 " ALIVE "\n"                          \
  "s_or_b64 %[m], s[58:59], s[60:61]\n"                       \
  "s_or_b64 %[m], %[m], s[62:63]\n"                        \
  "s_cbranch_scc1 " ALIVE "\n"
#define AERL_ANY_F_2(ALIVE)                             \
  "s_cbranch_scc1 " ALIVE "\n"                          \
  "s_cmp_lg_u64 s[58:59], 0\n"                             \
  "s_cbranch_scc1 " ALIVE "\n"
#define AERL_ANY_F_1(ALIVE) "s_cbranch_scc1 " ALIVE "\n"

// Lanes set in the fire masks, counted 32 bits at a time on the VALU (the
// scalar unit is the walk's busiest), into vt; in the undecided masks U_i,
// on the scalar unit into t0 (o as the temporary: the walk ends there).
#define AERL_POPC_4F                                    \
  "v_bcnt_u32_b32 %[vt], s56, 0\n"                       \
  "v_bcnt_u32_b32 %[vt], s57, %[vt]\n"                   \
  "v_bcnt_u32_b32 %[vt], s58, %[vt]\n"                   \
  "v_bcnt_u32_b32 %[vt], s59, %[vt]\n"                   \
  "v_bcnt_u32_b32 %[vt], s60, %[vt]\n"                   \
  "v_bcnt_u32_b32 %[vt], s61, %[vt]\n"                   \
  "v_bcnt_u32_b32 %[vt], s62, %[vt]\n"                   \
  "v_bcnt_u32_b32 %[vt], s63, %[vt]\n"
#define AERL_POPC_4U                                    \
  "s_bcnt1_i32_b64 %[t0], %[u0]\n"                      \
  "s_bcnt1_i32_b64 %[o], %[u1]\n"                       \
  "s_add_u32 %[t0], %[t0], %[o]\n"                     \
  "s_bcnt1_i32_b64 %[o], %[u2]\n"                       \
  "s_add_u32 %[t0], %[t0], %[o]\n"                     \
  "s_bcnt1_i32_b64 %[o], %[u3]\n"                       \
  "s_add_u32 %[t0], %[t0], %[o]\n"
#define AERL_POPC_2F                                    \
  "v_bcnt_u32_b32 %[vt], s56, 0\n"                       \
  "v_bcnt_u32_b32 %[vt], s57, %[vt]\n"                   \
  "v_bcnt_u32_b32 %[vt], s58, %[vt]\n"                   \
  "v_bcnt_u32_b32 %[vt], s59, %[vt]\n"
#define AERL_POPC_2U                                    \
  "s_bcnt1_i32_b64 %[t0], %[u0]\n"                      \
  "s_bcnt1_i32_b64 %[o], %[u1]\n"                       \
  "s_add_u32 %[t0], %[t0], %[o]\n"
#define AERL_POPC_1F "v_bcnt_u32_b32 %[vt], s56, 0\n v_bcnt_u32_b32 %[vt], s57, %[vt]\n"
#define AERL_POPC_1U "s_bcnt1_i32_b64 %[t0], %[u0]\n"

// Retire the fired lanes: to ALIVE as soon as the last slot still has an
// undecided lane, else falls through with SCC = some lane still undecided.
#define AERL_RETIRE_4(ALIVE)                            \
  "s_andn2_b64 %[u0], %[u0], s[56:57]\n"                   \
  "s_andn2_b64 %[u1], %[u1], s[58:59]\n"                   \
  "s_andn2_b64 %[u2], %[u2], s[60:61]\n"                   \
  "s_andn2_b64 %[u3], %[u3], s[62:63]\n"                   \
  "s_cbranch_scc1 " ALIVE "\n"                          \
  "s_or_b64 %[m], %[u0], %[u1]\n"                       \
  "s_or_b64 %[m], %[m], %[u2]\n"
#define AERL_RETIRE_2(ALIVE)                            \
  "s_andn2_b64 %[u0], %[u0], s[56:57]\n"                   \
  "s_andn2_b64 %[u1], %[u1], s[58:59]\n"                   \
  "s_cbranch_scc1 " ALIVE "\n"                          \
  "s_cmp_lg_u64 %[u0], 0\n"
#define AERL_RETIRE_1(ALIVE) "s_andn2_b64 %[u0], %[u0], s[56:57]\n"

// Adds the vt (t0) samples of the class in W to the class's lane of acc.
#define AERL_ADD_CLASS_V(W)                             \
  "v_bfe_u32 %[vt2], " W ", 12, 6\n"                    \
  "v_cmp_eq_u32_e32 vcc, %[vt2], %[lane]\n"             \
  "v_cndmask_b32_e32 %[vt], 0, %[vt], vcc\n"            \
  "v_add_u32 %[acc], %[acc], %[vt]\n"
#define AERL_ADD_CLASS(W)                               \
  "v_mov_b32 %[vt], %[t0]\n"                            \
  AERL_ADD_CLASS_V(W)

// Prediction: lanes set in the masks M_i take the class in W (pred_i).
#define AERL_SET_CLASS_4(W, M0, M1, M2, M3)             \
  "v_bfe_u32 %[vt], " W ", 12, 6\n"                     \
  "v_cndmask_b32_e64 %[p0], %[p0], %[vt], " M0 "\n"     \
  "v_cndmask_b32_e64 %[p1], %[p1], %[vt], " M1 "\n"     \
  "v_cndmask_b32_e64 %[p2], %[p2], %[vt], " M2 "\n"     \
  "v_cndmask_b32_e64 %[p3], %[p3], %[vt], " M3 "\n"
#define AERL_SET_CLASS_2(W, M0, M1)                     \
  "v_bfe_u32 %[vt], " W ", 12, 6\n"                     \
  "v_cndmask_b32_e64 %[p0], %[p0], %[vt], " M0 "\n"     \
  "v_cndmask_b32_e64 %[p1], %[p1], %[vt], " M1 "\n"
#define AERL_SET_CLASS_1(W, M0)                         \
  "v_bfe_u32 %[vt], " W ", 12, 6\n"                     \
  "v_cndmask_b32_e64 %[p0], %[p0], %[vt], " M0 "\n"
#define AERL_SETC_4F(W) AERL_SET_CLASS_4(W, "s[56:57]", "s[58:59]", "s[60:61]", "s[62:63]")
#define AERL_SETC_4U(W) AERL_SET_CLASS_4(W, "%[u0]", "%[u1]", "%[u2]", "%[u3]")
#define AERL_SETC_2F(W) AERL_SET_CLASS_2(W, "s[56:57]", "s[58:59]")
#define AERL_SETC_2U(W) AERL_SET_CLASS_2(W, "%[u0]", "%[u1]")
#define AERL_SETC_1F(W) AERL_SET_CLASS_1(W, "s[56:57]")
#define AERL_SETC_1U(W) AERL_SET_CLASS_1(W, "%[u0]")

// The rule of the (last) record in W fires for the lanes in f: count them
// for its class (COUNT) or give them its class (PRED), and retire them (to
// ALIVE, or on with SCC = some lane still undecided).
#define AERL_COMMIT_COUNT(S, W, ALIVE) \
  AERL_CAT(AERL_POPC_, AERL_SM(S, F)) AERL_ADD_CLASS_V(W) AERL_CAT(AERL_RETIRE_, S)(ALIVE)
#define AERL_COMMIT_PRED(S, W, ALIVE) \
  AERL_CAT(AERL_SETC_, AERL_SM(S, F))(W) AERL_CAT(AERL_RETIRE_, S)(ALIVE)
// An always-true rule in W decides every undecided lane.
#define AERL_ALWAYS_COUNT(S, W) AERL_CAT(AERL_POPC_, AERL_SM(S, U)) AERL_ADD_CLASS(W)
#define AERL_ALWAYS_PRED(S, W) AERL_CAT(AERL_SETC_, AERL_SM(S, U))(W)

// Start of a record whose row is at byte offset XX: read the row; records
// with a flag in MASK go to SPEC; falls through (row waited for) with a fast
// record of the walk's current direction.  In the >= direction MASK is
// kRecSpecial | kRecDirChg = 0xa0f, in the <= direction kRecSpecial = 0xa0b.
#define AERL_FETCH(S, XX, XW, MASK, SPEC)               \
  AERL_CAT(AERL_ADDR_, S)(XX)                           \
  AERL_CAT(AERL_RD_, S)                                 \
  "s_and_b32 %[t0], " XW ", " MASK "\n"                 \
  "s_cbranch_scc1 " SPEC "\n"                           \
  "s_waitcnt lgkmcnt(0)\n"

// Zero-coefficient record (y*x > z; y in Y, z in Z), row already
// requested; then on to POST with SCC = (f0 != 0).
#define AERL_MULREC(S, MODE, Y, Z, POST)                \
  "s_waitcnt lgkmcnt(0)\n"                              \
  AERL_CAT(AERL_MUL1_, S)(Y)                            \
  AERL_CAT(AERL_CMP_, AERL_SM(S, MODE))("lt", Z)        \
  "s_branch " POST "\n"

// A rule's last record with a folded threshold (x >= y, or x <= y when
// flagged; y in Y, flags in W), row already requested; then on to POST with
// SCC = (f0 != 0).
#define AERL_LASTREC(S, MODE, Y, W, TAG, POST)          \
  "s_waitcnt lgkmcnt(0)\n"                              \
  "s_bitcmp1_b32 " W ", 10\n"                           \
  "s_cbranch_scc1 .Lle_" TAG "_%=\n"                    \
  AERL_CAT(AERL_CMP_, AERL_SM(S, MODE))("le", Y)        \
  "s_branch " POST "\n"                                 \
  ".Lle_" TAG "_%=:\n"                                  \
  AERL_CAT(AERL_CMP_, AERL_SM(S, MODE))("ge", Y)        \
  "s_branch " POST "\n"

// Feature-vs-feature record (a in Y, b in Z, g and the >= flag in W), first
// row already requested: f_i = src_i & (a*x_i > b*x'_i) or (>=); then POST.
#define AERL_FF_BODY(S, MODE, W, Y, Z, TAG, POST)       \
  "v_bfe_u32 %[vt2], " W ", 0, 9\n"                     \
  "v_lshl_add_u32 %[vt2], %[vt2], " AERL_CAT(AERL_GSHIFT_, S) ", %[lds]\n" \
  AERL_CAT(AERL_RD2_, S)                                \
  "s_waitcnt lgkmcnt(0)\n"                              \
  AERL_CAT(AERL_MUL1_, S)(Y)                            \
  AERL_CAT(AERL_MUL2_, S)(Z)                            \
  "s_bitcmp1_b32 " W ", 10\n"                           \
  "s_cbranch_scc1 .Lge_" TAG "_%=\n"                    \
  AERL_CAT(AERL_FFCMP_, AERL_SM(S, MODE))("gt")         \
  "s_branch " POST "\n"                                 \
  ".Lge_" TAG "_%=:\n"                                  \
  AERL_CAT(AERL_FFCMP_, AERL_SM(S, MODE))("ge")         \
  "s_branch " POST "\n"

// Categorical record (code set in Y, Z), row already requested: per slot,
// the value's code k = cvt_u32(x) names the sample's category when
// cvt_f32(k) == x (an exact integer, not NaN) and k < 64; the sample is in
// the set when, further, bit k of the 64-bit mask (v[38:39]) is set.  Slots
// are taken last to first, so that f0 is written last: SCC = (f0 != 0).
#define AERL_CATSLOT(V, DST, SRC)                       \
  "v_cvt_u32_f32_e32 v36, " V "\n"                      \
  "v_cvt_f32_u32_e32 v37, v36\n"                        \
  "v_cmp_eq_f32_e32 vcc, v37, " V "\n"                  \
  "v_cmp_gt_u32_e64 %[m], 64, v36\n"                    \
  "s_and_b64 vcc, vcc, %[m]\n"                          \
  "v_lshrrev_b64 v[36:37], v36, v[38:39]\n"             \
  "v_and_b32_e32 v36, 1, v36\n"                         \
  "v_cmp_ne_u32_e64 %[m], 0, v36\n"                     \
  "s_and_b64 %[m], %[m], vcc\n"                         \
  "s_and_b64 " DST ", " SRC ", %[m]\n"
#define AERL_CATT_4(S0, S1, S2, S3)                     \
  AERL_CATSLOT("v35", "s[62:63]", S3)                   \
  AERL_CATSLOT("v34", "s[60:61]", S2)                   \
  AERL_CATSLOT("v33", "s[58:59]", S1)                   \
  AERL_CATSLOT("v32", "s[56:57]", S0)
#define AERL_CATT_2(S0, S1)                             \
  AERL_CATSLOT("v33", "s[58:59]", S1)                   \
  AERL_CATSLOT("v32", "s[56:57]", S0)
#define AERL_CATT_1(S0) AERL_CATSLOT("v32", "s[56:57]", S0)
#define AERL_CAT_4U AERL_CATT_4("%[u0]", "%[u1]", "%[u2]", "%[u3]")
#define AERL_CAT_4F AERL_CATT_4("s[56:57]", "s[58:59]", "s[60:61]", "s[62:63]")
#define AERL_CAT_2U AERL_CATT_2("%[u0]", "%[u1]")
#define AERL_CAT_2F AERL_CATT_2("s[56:57]", "s[58:59]")
#define AERL_CAT_1U AERL_CATT_1("%[u0]")
#define AERL_CAT_1F AERL_CATT_1("s[56:57]")
#define AERL_CAT_BODY(S, MODE, Y, Z, POST)              \
  "s_waitcnt lgkmcnt(0)\n"                              \
  "v_mov_b32_e32 v38, " Y "\n"                          \
  "v_mov_b32_e32 v39, " Z "\n"                          \
  AERL_CAT(AERL_CAT_, AERL_SM(S, MODE))                 \
  "s_branch " POST "\n"

// Special record entry once a plain last record is ruled out:
// feature-vs-feature, always-true (rule starts only, ALW), categorical
// (AERL_SPEC_C only), else a zero coefficient; then POST.  Walks of
// populations without categorical conditions use AERL_SPEC_N, which leaves
// the code-set body out of the walk's code.
#define AERL_SPEC_N(S, MODE, Y, Z, W, TAG, POST, ALW)   \
  "s_bitcmp1_b32 " W ", 9\n"                            \
  "s_cbranch_scc1 .Lff_" TAG "_%=\n"                    \
  ALW                                                   \
  AERL_MULREC(S, MODE, Y, Z, POST)                      \
  ".Lff_" TAG "_%=:\n"                                  \
  AERL_FF_BODY(S, MODE, W, Y, Z, TAG, POST)
#define AERL_SPEC_C(S, MODE, Y, Z, W, TAG, POST, ALW)   \
  "s_bitcmp1_b32 " W ", 9\n"                            \
  "s_cbranch_scc1 .Lff_" TAG "_%=\n"                    \
  ALW                                                   \
  "s_bitcmp1_b32 " W ", 3\n"                            \
  "s_cbranch_scc1 .Lcat_" TAG "_%=\n"                   \
  AERL_MULREC(S, MODE, Y, Z, POST)                      \
  ".Lff_" TAG "_%=:\n"                                  \
  AERL_FF_BODY(S, MODE, W, Y, Z, TAG, POST)             \
  ".Lcat_" TAG "_%=:\n"                                 \
  AERL_CAT_BODY(S, MODE, Y, Z, POST)

// How a walk moves between rules.  SEQ visits every rule in order (the
// next rule starts where a record's next field points, or right after a
// rule's last record); FLT visits only the rules whose bit is set in the mask
// mk (rule k starts at byte offset vst of lane k), lowest first, and needs
// the closing record's bit set so that every walk ends in a commit.
#define AERL_START_SEQ "s_mov_b32 %[o], 0\n"
#define AERL_START_FLT                                  \
  ".Lnext_%=:\n"                                        \
  "s_ff1_i32_b64 %[t0], %[mk]\n"                        \
  "v_readlane_b32 %[o], %[vst], %[t0]\n"                \
  "s_bitset0_b64 %[mk], %[t0]\n"
// the rule of the (non-last) record in W is dead
#define AERL_NXD_SEQ(W) "s_lshr_b32 %[o], " W ", 18\n s_branch .Lload_%=\n"
#define AERL_NXD_FLT(W) "s_branch .Lnext_%=\n"
// a special record in A (flags in s67) left no lane alive
#define AERL_XAD_SEQ                                    \
  "s_bitcmp1_b32 s67, 11\n"                             \
  "s_cbranch_scc1 .Lsb_%=\n"                            \
  "s_lshr_b32 %[o], s67, 18\n"                          \
  "s_branch .Lload_%=\n"
#define AERL_XAD_FLT "s_branch .Lnext_%=\n"
// where the walk goes after a rule ending at A
#define AERL_NXA_SEQ ".Lsb_%="
#define AERL_NXA_FLT ".Lnext_%="
// after a commit at B: CBL is taken with lanes still undecided, then NXB
// follows the retire (SCC = some lane still undecided)
#define AERL_CBL_SEQ ".Lcb_%="
#define AERL_CBL_FLT ".Lnext_%="
#define AERL_NXB_SEQ                                    \
  "s_cbranch_scc0 .Ldone_%=\n"                          \
  ".Lcb_%=:\n"                                          \
  "s_add_u32 %[o], %[o], 32\n"                          \
  "s_branch .Lload_%=\n"
#define AERL_NXB_FLT                                    \
  "s_cbranch_scc1 .Lnext_%=\n"                          \
  "s_branch .Ldone_%=\n"

// The whole walk for S samples per lane; KIND is COUNT or PRED.  Labels:
// s/n = a rule starts / continues at the record, a/b = quad A / B, _le = the
// <= direction (taken from a rule's first <= record to its end).
#define AERL_WALK(S, KIND, WAY, SP)                                            \
  AERL_CAT(AERL_START_, WAY)                                               \
  /* load the pair (o, o+16) into A, B; a rule starts at A */              \
  ".Lload_%=:\n"                                                           \
  "s_load_dwordx8 s[64:71], %[base], %[o]\n"                               \
  "s_waitcnt lgkmcnt(0)\n"                                                 \
  AERL_FETCH(S, "s64", "s67", "0xa0f", ".Lpsa_%=")                         \
  AERL_CAT(AERL_CMP_, AERL_SM(S, U))("le", "s65")                          \
  /* after a fast record in A: on with B unless no f_i fires */            \
  ".Lqa_%=:\n"                                                             \
  "s_cbranch_scc0 .Lka_%=\n"                                               \
  /* B continues the rule */                                               \
  ".Lnb_%=:\n"                                                             \
  AERL_FETCH(S, "s68", "s71", "0xa0f", ".Lpnb_%=")                         \
  AERL_CAT(AERL_CMP_, AERL_SM(S, F))("le", "s69")                          \
  ".Lqb_%=:\n"                                                             \
  "s_cbranch_scc0 .Lkb_%=\n"                                               \
  /* the next pair continues the rule */                                   \
  ".Llna_load_%=:\n"                                                       \
  "s_add_u32 %[o], %[o], 32\n"                                             \
  "s_load_dwordx8 s[64:71], %[base], %[o]\n"                               \
  "s_waitcnt lgkmcnt(0)\n"                                                 \
  AERL_FETCH(S, "s64", "s67", "0xa0f", ".Lpna_%=")                         \
  AERL_CAT(AERL_CMP_, AERL_SM(S, F))("le", "s65")                          \
  "s_cbranch_scc1 .Lnb_%=\n"                                               \
  /* f0 == 0 after a fast record in A: alive if another slot fires, else */ \
  /* the next rule starts past B (A is not a rule's last record) */        \
  ".Lka_%=:\n"                                                             \
  AERL_CAT(AERL_ANY_F_, S)(".Lnb_%=")                                      \
  AERL_CAT(AERL_NXD_, WAY)("s67")                                          \
  ".Lkb_%=:\n"                                                             \
  AERL_CAT(AERL_ANY_F_, S)(".Llna_load_%=")                                \
  AERL_CAT(AERL_NXD_, WAY)("s71")                                          \
  /* a rule starts at B (the previous one ended at A) */                   \
  ".Lsb_%=:\n"                                                             \
  AERL_FETCH(S, "s68", "s71", "0xa0f", ".Lpsb_%=")                         \
  AERL_CAT(AERL_CMP_, AERL_SM(S, U))("le", "s69")                          \
  "s_branch .Lqb_%=\n"                                                     \
  /* the same walk in the <= direction (rules continue, never start) */    \
  ".Lqa_le_%=:\n"                                                          \
  "s_cbranch_scc0 .Lka_le_%=\n"                                            \
  ".Lnb_le_%=:\n"                                                          \
  AERL_FETCH(S, "s68", "s71", "0xa0b", ".Lpnb_%=")                         \
  AERL_CAT(AERL_CMP_, AERL_SM(S, F))("ge", "s69")                          \
  ".Lqb_le_%=:\n"                                                          \
  "s_cbranch_scc0 .Lkb_le_%=\n"                                            \
  ".Llna_load_le_%=:\n"                                                    \
  "s_add_u32 %[o], %[o], 32\n"                                             \
  "s_load_dwordx8 s[64:71], %[base], %[o]\n"                               \
  "s_waitcnt lgkmcnt(0)\n"                                                 \
  AERL_FETCH(S, "s64", "s67", "0xa0b", ".Lpna_%=")                         \
  AERL_CAT(AERL_CMP_, AERL_SM(S, F))("ge", "s65")                          \
  "s_cbranch_scc1 .Lnb_le_%=\n"                                            \
  ".Lka_le_%=:\n"                                                          \
  AERL_CAT(AERL_ANY_F_, S)(".Lnb_le_%=")                                   \
  AERL_CAT(AERL_NXD_, WAY)("s67")                                          \
  ".Lkb_le_%=:\n"                                                          \
  AERL_CAT(AERL_ANY_F_, S)(".Llna_load_le_%=")                             \
  AERL_CAT(AERL_NXD_, WAY)("s71")                                          \
  /* a rule's first <= record (no other flag): compare, then <= walk */    \
  ".Ldsa_%=:\n"                                                            \
  "s_waitcnt lgkmcnt(0)\n"                                                 \
  AERL_CAT(AERL_CMP_, AERL_SM(S, U))("ge", "s65")                          \
  "s_branch .Lqa_le_%=\n"                                                  \
  ".Ldna_%=:\n"                                                            \
  "s_waitcnt lgkmcnt(0)\n"                                                 \
  AERL_CAT(AERL_CMP_, AERL_SM(S, F))("ge", "s65")                          \
  "s_branch .Lqa_le_%=\n"                                                  \
  ".Ldsb_%=:\n"                                                            \
  "s_waitcnt lgkmcnt(0)\n"                                                 \
  AERL_CAT(AERL_CMP_, AERL_SM(S, U))("ge", "s69")                          \
  "s_branch .Lqb_le_%=\n"                                                  \
  ".Ldnb_%=:\n"                                                            \
  "s_waitcnt lgkmcnt(0)\n"                                                 \
  AERL_CAT(AERL_CMP_, AERL_SM(S, F))("ge", "s69")                          \
  "s_branch .Lqb_le_%=\n"                                                  \
  /* special records (the direction change alone goes to .Ld*, a plain */  \
  /* last record, flags 0x203 clear, to .Lt*) */                           \
  ".Lpsa_%=:\n"                                                            \
  "s_and_b32 %[t0], s67, 0xa0b\n"                                          \
  "s_cbranch_scc0 .Ldsa_%=\n"                                              \
  "s_and_b32 %[t0], s67, 0x20b\n"                                          \
  "s_cbranch_scc0 .Ltsa_%=\n"                                              \
  AERL_CAT(AERL_SPEC_, SP)(S, U, "s65", "s66", "s67", "sa", ".Lxa_%=",                    \
            "s_bitcmp1_b32 s67, 1\n s_cbranch_scc1 .Lalwa_%=\n")           \
  ".Ltsa_%=:\n"                                                            \
  AERL_LASTREC(S, U, "s65", "s67", "tsa", ".Lza_%=")                       \
  ".Lpna_%=:\n"                                                            \
  "s_and_b32 %[t0], s67, 0xa0b\n"                                          \
  "s_cbranch_scc0 .Ldna_%=\n"                                              \
  "s_and_b32 %[t0], s67, 0x20b\n"                                          \
  "s_cbranch_scc0 .Ltna_%=\n"                                              \
  AERL_CAT(AERL_SPEC_, SP)(S, F, "s65", "s66", "s67", "na", ".Lxa_%=", "")                \
  ".Ltna_%=:\n"                                                            \
  AERL_LASTREC(S, F, "s65", "s67", "tna", ".Lza_%=")                       \
  ".Lpsb_%=:\n"                                                            \
  "s_and_b32 %[t0], s71, 0xa0b\n"                                          \
  "s_cbranch_scc0 .Ldsb_%=\n"                                              \
  "s_and_b32 %[t0], s71, 0x20b\n"                                          \
  "s_cbranch_scc0 .Ltsb_%=\n"                                              \
  AERL_CAT(AERL_SPEC_, SP)(S, U, "s69", "s70", "s71", "sb", ".Lxb_%=",                    \
            "s_bitcmp1_b32 s71, 1\n s_cbranch_scc1 .Lalwb_%=\n")           \
  ".Ltsb_%=:\n"                                                            \
  AERL_LASTREC(S, U, "s69", "s71", "tsb", ".Lzb_%=")                       \
  ".Lpnb_%=:\n"                                                            \
  "s_and_b32 %[t0], s71, 0xa0b\n"                                          \
  "s_cbranch_scc0 .Ldnb_%=\n"                                              \
  "s_and_b32 %[t0], s71, 0x20b\n"                                          \
  "s_cbranch_scc0 .Ltnb_%=\n"                                              \
  AERL_CAT(AERL_SPEC_, SP)(S, F, "s69", "s70", "s71", "nb", ".Lxb_%=", "")                \
  ".Ltnb_%=:\n"                                                            \
  AERL_LASTREC(S, F, "s69", "s71", "tnb", ".Lzb_%=")                       \
  /* after a special record in A (what follows it in its rule is special */ \
  /* too, or starts a new rule, so the >= labels serve both directions) */ \
  ".Lxa_%=:\n"                                                             \
  AERL_CAT(AERL_ANY_F_, S)(".Lya_%=")                                      \
  AERL_CAT(AERL_XAD_, WAY)                                                 \
  /* after a rule's last record in A */                                    \
  ".Lza_%=:\n"                                                             \
  AERL_CAT(AERL_ANY_F_, S)(".Lwa_%=")                                      \
  "s_branch " AERL_CAT(AERL_NXA_, WAY) "\n"                                \
  ".Lya_%=:\n"                                                             \
  "s_bitcmp1_b32 s67, 11\n"                                                \
  "s_cbranch_scc0 .Lnb_%=\n"                                               \
  ".Lwa_%=:\n"                                                             \
  AERL_CAT(AERL_COMMIT_, KIND)(S, "s67", AERL_CAT(AERL_NXA_, WAY))         \
  "s_cbranch_scc1 " AERL_CAT(AERL_NXA_, WAY) "\n"                          \
  "s_branch .Ldone_%=\n"                                                   \
  /* after a special record in B, or a rule's last record in B */          \
  ".Lxb_%=:\n"                                                             \
  AERL_CAT(AERL_ANY_F_, S)(".Lyb_%=")                                      \
  AERL_CAT(AERL_NXD_, WAY)("s71")                                          \
  ".Lzb_%=:\n"                                                             \
  AERL_CAT(AERL_ANY_F_, S)(".Lwb_%=")                                      \
  AERL_CAT(AERL_NXD_, WAY)("s71")                                          \
  ".Lyb_%=:\n"                                                             \
  "s_bitcmp1_b32 s71, 11\n"                                                \
  "s_cbranch_scc0 .Llna_load_%=\n"                                         \
  ".Lwb_%=:\n"                                                             \
  AERL_CAT(AERL_COMMIT_, KIND)(S, "s71", AERL_CAT(AERL_CBL_, WAY))         \
  AERL_CAT(AERL_NXB_, WAY)                                                 \
  /* an always-true rule decides every undecided lane */                   \
  ".Lalwa_%=:\n"                                                           \
  "s_waitcnt lgkmcnt(0)\n"                                                 \
  AERL_CAT(AERL_ALWAYS_, KIND)(S, "s67")                                   \
  "s_branch .Ldone_%=\n"                                                   \
  ".Lalwb_%=:\n"                                                           \
  "s_waitcnt lgkmcnt(0)\n"                                                 \
  AERL_CAT(AERL_ALWAYS_, KIND)(S, "s71")                                   \
  ".Ldone_%=:\n"

#define AERL_WALK_CLOBBERS                                                 \
  "s56", "s57", "s58", "s59", "s60", "s61", "s62", "s63", "s64", "s65", "s66", "s67", "s68", "s69", "s70", "s71", "v32", "v33", "v34", \
      "v35", "v36", "v37", "v38", "v39", "vcc", "scc", "memory"

// Counting walk over every rule of the set (SEQ) or over the rules whose bit
// is set in mk (FLT; vst holds the rules' byte offsets, one per lane).  CAT:
// the walk takes categorical records (populations that have them).
template <int S, bool FLT, bool CAT>
__device__ __forceinline__ int eval_set_count(uint32_t lds_lane, int lane, int4 set,
                                              const uint4 *__restrict__ stream,
                                              const uint64_t (&vm)[S], uint64_t mk = 0,
                                              uint32_t vst = 0);

#define AERL_COUNT_OUTS_4 [acc] "+v"(acc), [u0] "+s"(u0), [u1] "+s"(u1), [u2] "+s"(u2), [u3] "+s"(u3)
#define AERL_COUNT_OUTS_2 [acc] "+v"(acc), [u0] "+s"(u0), [u1] "+s"(u1)
#define AERL_COUNT_OUTS_1 [acc] "+v"(acc), [u0] "+s"(u0)
#define AERL_TEMPS [m] "=&s"(m), [o] "=&s"(o), [t0] "=&s"(t0), [vt] "=&v"(vt), [vt2] "=&v"(vt2)
#define AERL_U_4 uint64_t u0 = vm[0], u1 = vm[1], u2 = vm[2], u3 = vm[3];
#define AERL_U_2 uint64_t u0 = vm[0], u1 = vm[1];
#define AERL_U_1 uint64_t u0 = vm[0];

#define AERL_COUNT_SPECIALIZE(S, CAT, SP)                                                     \
  template <>                                                                                 \
  __device__ __forceinline__ int eval_set_count<S, false, CAT>(                               \
      uint32_t lds_lane, int lane, int4 set, const uint4 *__restrict__ stream,                \
      const uint64_t(&vm)[S], uint64_t, uint32_t) {                                           \
    const uint4 *base = stream + set.x;                                                       \
    AERL_U_##S                                                                                \
    uint64_t m;                                                                               \
    uint32_t o, t0, vt, vt2;                                                                  \
    int acc = 0;                                                                              \
    asm volatile(AERL_WALK(S, COUNT, SEQ, SP)                                                 \
                 : AERL_COUNT_OUTS_##S, AERL_TEMPS                                            \
                 : [base] "s"(base), [lds] "v"(lds_lane), [lane] "v"(lane)                    \
                 : AERL_WALK_CLOBBERS);                                                       \
    return acc;                                                                               \
  }                                                                                           \
  template <>                                                                                 \
  __device__ __forceinline__ int eval_set_count<S, true, CAT>(                                \
      uint32_t lds_lane, int lane, int4 set, const uint4 *__restrict__ stream,                \
      const uint64_t(&vm)[S], uint64_t mk, uint32_t vst) {                                    \
    const uint4 *base = stream + set.x;                                                       \
    AERL_U_##S                                                                                \
    uint64_t m;                                                                               \
    uint32_t o, t0, vt, vt2;                                                                  \
    int acc = 0;                                                                              \
    asm volatile(AERL_WALK(S, COUNT, FLT, SP)                                                 \
                 : AERL_COUNT_OUTS_##S, AERL_TEMPS, [mk] "+s"(mk)                             \
                 : [base] "s"(base), [lds] "v"(lds_lane), [lane] "v"(lane), [vst] "v"(vst)    \
                 : AERL_WALK_CLOBBERS);                                                       \
    return acc;                                                                               \
  }

AERL_COUNT_SPECIALIZE(4, false, N)
AERL_COUNT_SPECIALIZE(2, false, N)
AERL_COUNT_SPECIALIZE(1, false, N)
AERL_COUNT_SPECIALIZE(4, true, C)
AERL_COUNT_SPECIALIZE(2, true, C)
AERL_COUNT_SPECIALIZE(1, true, C)

// Prediction form of the sequential walk: pred[s] receives the class of each
// lane's samples in vm (others keep their value).
template <int S>
__device__ __forceinline__ void eval_set_pred(uint32_t lds_lane, int lane, int4 set,
                                              const uint4 *__restrict__ stream,
                                              const uint64_t (&vm)[S], int (&pred)[S]);

template <>
__device__ __forceinline__ void eval_set_pred<4>(uint32_t lds_lane, int lane, int4 set,
                                                 const uint4 *__restrict__ stream,
                                                 const uint64_t (&vm)[4], int (&pred)[4]) {
  const uint4 *base = stream + set.x;
  AERL_U_4
  uint64_t m;
  uint32_t o, t0, vt, vt2;
  int p0 = pred[0], p1 = pred[1], p2 = pred[2], p3 = pred[3];
  asm volatile(AERL_WALK(4, PRED, SEQ, C)
               : [p0] "+v"(p0), [p1] "+v"(p1), [p2] "+v"(p2), [p3] "+v"(p3), [u0] "+s"(u0),
                 [u1] "+s"(u1), [u2] "+s"(u2), [u3] "+s"(u3), AERL_TEMPS
               : [base] "s"(base), [lds] "v"(lds_lane)
               : AERL_WALK_CLOBBERS);
  (void)lane;
  pred[0] = p0; pred[1] = p1; pred[2] = p2; pred[3] = p3;
}

template <>
__device__ __forceinline__ void eval_set_pred<2>(uint32_t lds_lane, int lane, int4 set,
                                                 const uint4 *__restrict__ stream,
                                                 const uint64_t (&vm)[2], int (&pred)[2]) {
  const uint4 *base = stream + set.x;
  AERL_U_2
  uint64_t m;
  uint32_t o, t0, vt, vt2;
  int p0 = pred[0], p1 = pred[1];
  asm volatile(AERL_WALK(2, PRED, SEQ, C)
               : [p0] "+v"(p0), [p1] "+v"(p1), [u0] "+s"(u0), [u1] "+s"(u1), AERL_TEMPS
               : [base] "s"(base), [lds] "v"(lds_lane)
               : AERL_WALK_CLOBBERS);
  (void)lane;
  pred[0] = p0; pred[1] = p1;
}

template <>
__device__ __forceinline__ void eval_set_pred<1>(uint32_t lds_lane, int lane, int4 set,
                                                 const uint4 *__restrict__ stream,
                                                 const uint64_t (&vm)[1], int (&pred)[1]) {
  const uint4 *base = stream + set.x;
  AERL_U_1
  uint64_t m;
  uint32_t o, t0, vt, vt2;
  int p0 = pred[0];
  asm volatile(AERL_WALK(1, PRED, SEQ, C)
               : [p0] "+v"(p0), [u0] "+s"(u0), AERL_TEMPS
               : [base] "s"(base), [lds] "v"(lds_lane)
               : AERL_WALK_CLOBBERS);
  (void)lane;
  pred[0] = p0;
}

}  // namespace aerl
