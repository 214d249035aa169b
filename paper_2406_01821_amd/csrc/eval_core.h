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

// Evaluates rule set `set` = {first rule, #rules, default, -} for the S*64
// samples of the tile.  vm[s]: lanes whose slot-s sample is real.
// COUNT mode (PRED = false): returns, in lane c, the number of the tile's
//   real samples predicted as class c.
// PRED mode: pred[s] receives the predicted class of each lane's samples.
template <int S, bool PRED>
__device__ __forceinline__ int eval_set(const float *__restrict__ xs, int lane, int4 set,
                                        const int4 *__restrict__ rules,
                                        const uint4 *__restrict__ conds, const uint64_t (&vm)[S],
                                        int (&pred)[S]) {
  uint64_t und[S];
#pragma unroll
  for (int s = 0; s < S; ++s) und[s] = vm[s];
  int acc = 0;
  const int rb = set.x, nr = set.y;
  for (int k = 0; k < nr; ++k) {
    const int4 r = ldc(rules, rb + k);
    uint64_t fire[S];
#pragma unroll
    for (int s = 0; s < S; ++s) fire[s] = und[s];
    const int nt = r.y & 255, ng = (r.y >> 8) & 255, ne = (r.y >> 16) & 255;
    const uint4 *cp = conds + r.x;
    // Three single-exit loops (thresholds, feature >, feature >=).  When no
    // lane can fire the rule any more (any == 0) the offset jumps to the end;
    // a dead rule leaves all fire masks zero, so the bookkeeping below needs
    // no extra branch.
    uint64_t any = ~0ull;
    {
      const uint32_t end = (uint32_t)nt * 16u;
      for (uint32_t o = 0; o < end;) {
        const uint4 cc = ldc_at(cp, o);
        float v[S];
        load_row<S>(xs, cc.x, lane, v);
        const float ca = __uint_as_float(cc.y), cb = __uint_as_float(cc.z);
        any = 0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          fire[s] &= ballot(ca * v[s] > cb);
          any |= fire[s];
        }
        o = any == 0 ? end : o + 16u;
      }
    }
    {
      const uint32_t end = (uint32_t)(nt + ng) * 16u;
      for (uint32_t o = any == 0 ? end : (uint32_t)nt * 16u; o < end;) {
        const uint4 cc = ldc_at(cp, o);
        float v1[S], v2[S];
        load_row<S>(xs, cc.x, lane, v1);
        load_row<S>(xs, cc.w, lane, v2);
        const float ca = __uint_as_float(cc.y), cb = __uint_as_float(cc.z);
        any = 0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          fire[s] &= ballot(ca * v1[s] > cb * v2[s]);
          any |= fire[s];
        }
        o = any == 0 ? end : o + 16u;
      }
    }
    {
      const uint32_t end = (uint32_t)(nt + ng + ne) * 16u;
      for (uint32_t o = any == 0 ? end : (uint32_t)(nt + ng) * 16u; o < end;) {
        const uint4 cc = ldc_at(cp, o);
        float v1[S], v2[S];
        load_row<S>(xs, cc.x, lane, v1);
        load_row<S>(xs, cc.w, lane, v2);
        const float ca = __uint_as_float(cc.y), cb = __uint_as_float(cc.z);
        any = 0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          fire[s] &= ballot(ca * v1[s] >= cb * v2[s]);
          any |= fire[s];
        }
        o = any == 0 ? end : o + 16u;
      }
    }
    if (any == 0) continue;
    int nfire = 0;
    uint64_t left = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if constexpr (PRED) {
        if ((fire[s] >> lane) & 1ull) pred[s] = r.z;
      }
      nfire += __builtin_popcountll(fire[s]);
      und[s] &= ~fire[s];
      left |= und[s];
    }
    if constexpr (!PRED) acc += (lane == r.z) ? nfire : 0;
    if (left == 0) return acc;
  }
  int nleft = 0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    if constexpr (PRED) {
      if ((und[s] >> lane) & 1ull) pred[s] = set.z;
    }
    nleft += __builtin_popcountll(und[s]);
  }
  if constexpr (!PRED) acc += (lane == set.z) ? nleft : 0;
  return acc;
}

}  // namespace aerl
