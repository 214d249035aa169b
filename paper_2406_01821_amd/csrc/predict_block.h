// One wave's share of a prediction: 64*S consecutive rows of a row-major
// request, evaluated with one rule set (Section 3: step activation, AND of
// conditions, first firing rule, else the default class).  Shared by the
// single-request kernel and the batched one.
#pragma once

#include "eval_core.h"

namespace aerl {

// xs: LDS of nf*64*S floats.  Rows [base, base+64*S) of the n rows; rows past
// n are staged as zeros and never written.  Called by a 64-thread block.
template <int S>
__device__ __forceinline__ void predict_block(const float *__restrict__ rows, int64_t n, int32_t nf,
                                              const int4 set, const uint4 *__restrict__ conds,
                                              int32_t *__restrict__ out, int64_t base, float *xs) {
  constexpr int TS = 64 * S;
  const int lane = threadIdx.x & 63;
  const int64_t m = min((int64_t)TS, n - base);
  const int64_t total = (int64_t)TS * nf;
  for (int64_t i = lane; i < total; i += 64) {
    const int64_t r = i / nf, f = i - r * nf;
    xs[f * TS + r] = r < m ? rows[(base + r) * nf + f] : 0.0f;
  }
  __syncthreads();
  uint64_t vm[S];
  int pred[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    vm[s] = ballot(lane * S + s < m);
    pred[s] = set.z;
  }
  const uint32_t lds_lane =
      (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) float *)xs + (uint32_t)lane * (4u * S);
  eval_set_pred<S>(lds_lane, lane, set, conds, vm, pred);
#pragma unroll
  for (int s = 0; s < S; ++s)
    if (lane * S + s < m) out[base + lane * S + s] = pred[s];
}

}  // namespace aerl
