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
  int32_t *correct;   // [n_sets]
  int32_t *confusion; // [n_sets][nc][nc] or null
  int32_t q0, Q, tile_lo, tile_hi, label;
};

// Stages one wave tile (64*S samples x nf features) at a time into LDS and
// lets the waves pull rule sets, two at a time, from an LDS counter;
// per-class prediction counts live in LDS (one writer per rule set and tile)
// and reach the outputs once, through integer atomics.  smem holds nf*64*S floats followed
// by Q*nc 16-bit counters (a block covers at most 255 layout tiles, so a
// counter stays below 2^16).  Ends with a barrier, so the caller may reuse
// smem.
template <int S>
__device__ __forceinline__ void hard_block(const HardTask &t, float *smem, int32_t *next_q) {
  constexpr int TS = 64 * S;           // samples per wave tile
  constexpr int WPT = AERL_TILE / TS;  // wave tiles per layout tile
  float *xs = smem;                                                    // [nf][TS]
  uint16_t *cnt = reinterpret_cast<uint16_t *>(smem + (size_t)t.nf * TS);  // [Q][nc]
  const int lane = threadIdx.x & 63;
  for (int i = threadIdx.x; i < t.Q * t.nc; i += blockDim.x) cnt[i] = 0;
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
    for (;;) {
      int q0 = 0;
      if (lane == 0) q0 = atomicAdd(next_q, 2);  // two rule sets per grab
      q0 = __builtin_amdgcn_readfirstlane(q0);
      if (q0 >= t.Q) break;
      const int q1 = min(q0 + 2, t.Q);
      for (int q = q0; q < q1; ++q) {
        const int4 set = ldc(t.sets, t.q0 + q);
        const int acc = eval_set_count<S>(lds_lane, lane, set, t.conds, vm);
        if (lane < t.nc) cnt[q * t.nc + lane] += (uint16_t)acc;
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < t.Q * t.nc; i += blockDim.x) {
    const int v = cnt[i];
    if (v == 0) continue;
    const int q = i / t.nc, c = i - q * t.nc;
    const int64_t p = t.q0 + q;
    if (t.confusion) atomicAdd(&t.confusion[(p * t.nc + t.label) * t.nc + c], v);
    if (c == t.label) atomicAdd(&t.correct[p], v);
  }
  __syncthreads();
}

}  // namespace aerl
