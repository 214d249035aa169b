// One workgroup's share of a hard fitness evaluation: rule sets
// [q0, q0+Q) of one population on tiles [tile_lo, tile_hi) of one class
// region (every sample has label `label`).  Shared by the one-launch-per-
// population kernel and the persistent batch kernel.
#pragma once

#include "eval_core.h"
#include "internal.h"

namespace aerl {

// Kernels running hard_block with 1024-thread blocks: two such blocks share a
// CU (eight waves per SIMD) only when a wave holds at most 80 SGPRs; measured
// on gfx950, 82 already leaves room for one block.  The cap makes the
// compiler keep within it (spilling a few loop-invariant values to VGPR lanes
// outside the rule-set loop); the asm walk's fixed quads s[64:71] lie below it.
#define AERL_HARD_SGPR_CAP __attribute__((amdgpu_num_sgpr(80)))

typedef float f4v __attribute__((ext_vector_type(4)));

struct HardTask {
  const float *x_fm;
  int64_t n_pad;
  int32_t nf, nc;
  const int32_t *tile_info;
  const int4 *sets;   // the population's set records
  const uint4 *conds; // the population's record stream
  const uint4 *heads; // the population's head table
  int32_t *correct;   // [n_sets]
  int32_t *confusion; // [n_sets][nc][nc] or null
  uint32_t *part;     // this chunk's per-tile counter words (row stride part_stride), or null
  int32_t part_stride;
  int32_t q0, Q, tile_lo, tile_hi, label;
};

// Stages one wave tile (64*S samples x nf features) at a time into LDS,
// with the largest value and the negated smallest value of each feature
// over the tile's samples, and lets the waves pull rule sets, two at a time,
// from an LDS counter.  A rule with one of its first two records a folded
// threshold that no sample of the tile passes (x >= t with t above the
// tile's largest x, or x <= t with t below its smallest) cannot fire for any
// of them: the walk skips it without reading its records (exact).
// Per-class prediction counts live in LDS (one writer per rule set and
// wave tile) and reach the outputs once, through integer atomics; the last
// class's count is what the other classes leave of the block's samples.
// smem holds nf*64*S floats, then nf (max, -min) pairs, then the counters
// of the classes but the last, hard_counter_bytes(Q, nc, C10) bytes: with
// C10 (a block of one layout tile, so a count is at most 256) a set's
// counters in 10-bit fields, three per 32-bit word, else two 16-bit ones
// per word, counter q*(nc-1) + c for set q and class c (a block covers at
// most 255 layout tiles, so a counter stays below 2^16).  With C10, at most
// four classes and t.part set, the block stores its counters to t.part's
// row of its tile instead (row stride t.part_stride words), packed across
// sets three fields to a word, for a second kernel to sum.  sh[0] is the
// rule-set counter, sh[1] the block's real sample count (kept in LDS by one
// thread, so that it holds no register through the walk).  Ends with a
// barrier, so the caller may reuse smem.
template <int S, bool CAT, bool C10 = false>
__device__ __forceinline__ void hard_block(const HardTask &t, float *smem, int32_t *sh) {
  int32_t *next_q = sh;
  constexpr int TS = 64 * S;           // samples per wave tile
  constexpr int WPT = AERL_TILE / TS;  // wave tiles per layout tile
  float *xs = smem;                                                    // [nf][TS]
  float *ext = smem + (size_t)t.nf * TS;                               // [nf][max, -min]
  const int ncc = hard_counters_per_set(t.nc);                        // counted classes
  uint32_t *cnt32 = reinterpret_cast<uint32_t *>(ext + 2 * t.nf);
  const int lane = threadIdx.x & 63;
  // with C10: counter words per rule set, and lane c's word and bit offset
  // in a set's counters
  const int wps = (ncc + 2) / 3;
  const uint32_t lane_word = (uint32_t)lane / 3u;
  const uint32_t lane_bit = (uint32_t)lane % 3u * 10u;
  for (int i = threadIdx.x; i < (int)(hard_counter_bytes(t.Q, t.nc, C10) / 4); i += blockDim.x)
    cnt32[i] = 0u;
  if (threadIdx.x == 0) sh[1] = 0;
  const int n4 = t.nf * (TS / 4);
  const float4 *src = reinterpret_cast<const float4 *>(t.x_fm);
  float4 *dst = reinterpret_cast<float4 *>(xs);
  const int64_t row4 = t.n_pad / 4;
  const uint32_t lds_lane =
      (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) float *)xs + (uint32_t)lane * (4u * S);
  for (int64_t wt = (int64_t)t.tile_lo * WPT; wt < (int64_t)t.tile_hi * WPT; ++wt) {
    __syncthreads();  // everyone is done with the previous tile
    const int64_t base4 = wt * (TS / 4);
    for (int i = threadIdx.x; i < n4; i += blockDim.x) {
      const int f = i / (TS / 4), k = i % (TS / 4);
      // streamed once per block: a non-temporal load keeps it from pushing
      // the rule records out of the L2
      reinterpret_cast<f4v *>(dst)[i] =
          __builtin_nontemporal_load(reinterpret_cast<const f4v *>(src + (int64_t)f * row4 + base4 + k));
    }
    if (threadIdx.x == 0) *next_q = 0;
    __syncthreads();
    const int info = ldc(t.tile_info, wt / WPT);
    const int valid = min(max((info >> 8) - (int)(wt % WPT) * TS, 0), TS);
    uint64_t vm[S];
#pragma unroll
    for (int s = 0; s < S; ++s) vm[s] = ballot(lane * S + s < valid);
    if (valid == 0) continue;  // an empty wave tile (S < 4 at a region's end)
    if (threadIdx.x == 0) sh[1] += valid;
    // largest and negated smallest value of each feature over the valid
    // samples: 16 threads per feature
    for (int f0 = 0; f0 < t.nf; f0 += 64) {
      const int f = f0 + (threadIdx.x >> 4), part = threadIdx.x & 15;
      float hi = -INFINITY, lo = INFINITY;
      if (f < t.nf) {
        for (int i = part; i < valid; i += 16) {
          const float v = xs[f * TS + i];
          hi = fmaxf(hi, v);
          lo = fminf(lo, v);
        }
      }
      for (int d = 1; d < 16; d <<= 1) {
        hi = fmaxf(hi, __shfl_xor(hi, d));
        lo = fminf(lo, __shfl_xor(lo, d));
      }
      if (f < t.nf && part == 0) {
        ext[2 * f] = hi;
        ext[2 * f + 1] = -lo;
      }
    }
    __syncthreads();
    for (;;) {
      int q0 = 0;
      if (lane == 0) q0 = atomicAdd(next_q, 2);  // two rule sets per grab
      q0 = __builtin_amdgcn_readfirstlane(q0);
      if (q0 >= t.Q) break;
      const int q1 = min(q0 + 2, t.Q);
      // both set records in one scalar load (at the chunk's odd end the
      // second is the record after it, inside the population image and
      // never used), and both sets' head entries requested before the
      // first walk; a lane past a set's last entry reads that entry again
      // (its value is never used), so the loads need no lane mask
      int4 set[2];
      ldc_pair(t.sets + t.q0 + q0, set);
      uint4 head[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int nh = set[k].y >> 16;
        if (q0 + k < q1 && nh >= 1 && nh <= kMaxHeads)
          head[k] = t.heads[set[k].x + min(lane, nh - 1)];
      }
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int q = q0 + k;
        if (q >= q1) break;
        const int4 s4 = set[k];
        const int nh = s4.y >> 16;
        int acc;
        if (nh >= 1 && nh <= kMaxHeads) {
          // lane j: rule j; table[e] < t' when no sample of the tile passes
          const uint4 h = head[k];
          const char *tb = reinterpret_cast<const char *>(ext);
          const float e1 = *reinterpret_cast<const float *>(tb + (h.x >> kHeadExtShift));
          const float e2 = *reinterpret_cast<const float *>(tb + h.z);
          // rules 0..nh-1, less those a test rules out; the closing record
          // (last entry) is always visited
          const uint64_t rules = ~0ull >> (64 - nh);
          const uint64_t mk = (ballot(!(e1 < __uint_as_float(h.y))) &
                               ballot(!(e2 < __uint_as_float(h.w))) & rules) |
                              (1ull << (nh - 1));
          acc = eval_set_count<S, true, CAT>(lds_lane, lane, s4, t.conds, vm, mk, h.x & kHeadOffMask);
        } else {
          acc = eval_set_count<S, false, CAT>(lds_lane, lane, s4, t.conds, vm);
        }
        // lane c < ncc adds class c's count: a no-return atomic add with no
        // carry between the fields of a word (each count fits its field)
        if (lane < ncc) {
          if (C10) {
            atomicAdd(cnt32 + (uint32_t)(q * wps) + lane_word, (uint32_t)acc << lane_bit);
          } else {
            const int i = q * ncc + lane;
            atomicAdd(cnt32 + (i >> 1), (uint32_t)acc << ((i & 1) * 16));
          }
        }
      }
    }
  }
  __syncthreads();
  if (C10 && t.part != nullptr) {
    // word w of the row holds counters 3w..3w+2 of the chunk (counter
    // i = q*ncc + c), ten bits each; with four classes that is set w's word
    uint32_t *dst = t.part + (int64_t)t.tile_lo * t.part_stride;
    const int nw = hard_part_chunk_words(t.Q, t.nc), ni = t.Q * ncc;
    if (ncc == 3) {
      for (int w = threadIdx.x; w < nw; w += blockDim.x) dst[w] = cnt32[w];
    } else if (ncc == 2) {
      // one word per set in LDS, counters c = 0, 1 in bits 0 and 10
      for (int w = threadIdx.x; w < nw; w += blockDim.x) {
        uint32_t v = 0u;
        for (int k = 0; k < 3 && 3 * w + k < ni; ++k) {
          const int i = 3 * w + k;
          v |= (cnt32[i >> 1] >> ((i & 1) * 10) & 1023u) << (10 * k);
        }
        dst[w] = v;
      }
    } else if (ncc == 1) {
      for (int w = threadIdx.x; w < nw; w += blockDim.x) {
        uint32_t v = 0u;
        for (int k = 0; k < 3 && 3 * w + k < ni; ++k) v |= cnt32[3 * w + k] << (10 * k);
        dst[w] = v;
      }
    }
    __syncthreads();
    return;
  }
  // the block's real samples (every set predicts one class for each)
  const int n_block = sh[1];
  for (int q = threadIdx.x; q < t.Q; q += blockDim.x) {
    const int64_t p = t.q0 + q;
    int rest = n_block;
    for (int c = 0; c < t.nc; ++c) {
      int v = rest;
      if (c < ncc) {
        if (C10) {
          v = (int)(cnt32[q * wps + c / 3] >> (c % 3 * 10)) & 1023;
        } else {
          const int i = q * ncc + c;
          v = (int)(cnt32[i >> 1] >> ((i & 1) * 16)) & 0xffff;
        }
      }
      rest -= v;
      if (v == 0) continue;
      if (t.confusion) atomicAdd(&t.confusion[(p * t.nc + t.label) * t.nc + c], v);
      if (c == t.label) atomicAdd(&t.correct[p], v);
    }
  }
  __syncthreads();
}

}  // namespace aerl
