// Hard fitness (correct counts + confusion) and prediction kernels.
//
// Fitness of a rule set is its classification accuracy on the labeled
// dataset (Section 1), with rules read as a first-firing decision list of
// ANDed step-activated conditions (Section 3, Fig. 1).
//
// Work decomposition of k_hard: block (chunk, group) evaluates rule sets
// [chunk*Q, chunk*Q+Q) on the layout tiles of one tile group; a group lies
// inside one class region, so every sample of the block has the same label.
// The block stages one wave tile (64*S samples x F features, fp32) at a time
// into LDS with coalesced 16-byte loads; its waves then pull rule sets from
// an LDS counter and evaluate them against the staged tile.  Per-class
// prediction counts accumulate in LDS (one writer per rule set and tile) and
// are added to the global outputs once per block with integer atomics, so
// the result does not depend on the schedule.
#include "eval_core.h"
#include "internal.h"

namespace aerl {

namespace {

constexpr int kHardBlock = 1024;

struct HardArgs {
  const float *x_fm;
  int64_t n_pad;
  int32_t nf, nc;
  const int32_t *tile_info;
  const int4 *sets;
  const int4 *rules;
  const uint4 *conds;
  int32_t set_begin, set_count;
  int32_t *correct;
  int32_t *confusion;
  int32_t sets_per_chunk, tiles_per_group;
  int32_t region_tile0[AERL_MAX_CLASSES];
  int32_t region_tiles[AERL_MAX_CLASSES];
};

template <int S, bool CONF>
__global__ __launch_bounds__(kHardBlock) void k_hard(const HardArgs a) {
  constexpr int TS = 64 * S;           // samples per wave tile
  constexpr int WPT = AERL_TILE / TS;  // wave tiles per layout tile
  extern __shared__ __align__(16) float smem[];
  float *xs = smem;                                      // [nf][TS]
  int32_t *cnt = reinterpret_cast<int32_t *>(smem + (size_t)a.nf * TS);  // [Q][nc]
  __shared__ int32_t next_q;
  const int lane = threadIdx.x & 63;

  // Which class region and which tiles this block covers (uniform loop).
  int label = 0, tile_lo = 0, tile_hi = 0;
  {
    int g = blockIdx.y;
    for (int c = 0; c < a.nc; ++c) {
      const int ng = (a.region_tiles[c] + a.tiles_per_group - 1) / a.tiles_per_group;
      if (g < ng) {
        label = c;
        tile_lo = a.region_tile0[c] + g * a.tiles_per_group;
        tile_hi = min(tile_lo + a.tiles_per_group, a.region_tile0[c] + a.region_tiles[c]);
        break;
      }
      g -= ng;
    }
  }
  const int q0 = blockIdx.x * a.sets_per_chunk;
  const int Q = min(a.sets_per_chunk, a.set_count - q0);
  for (int i = threadIdx.x; i < Q * a.nc; i += blockDim.x) cnt[i] = 0;

  const int n4 = a.nf * (TS / 4);
  const float4 *src = reinterpret_cast<const float4 *>(a.x_fm);
  float4 *dst = reinterpret_cast<float4 *>(xs);
  const int64_t row4 = a.n_pad / 4;
  for (int64_t wt = (int64_t)tile_lo * WPT; wt < (int64_t)tile_hi * WPT; ++wt) {
    __syncthreads();  // everyone is done with the previous tile
    const int64_t base4 = wt * (TS / 4);
    for (int i = threadIdx.x; i < n4; i += blockDim.x) {
      const int f = i / (TS / 4), k = i % (TS / 4);
      dst[i] = src[(int64_t)f * row4 + base4 + k];
    }
    if (threadIdx.x == 0) next_q = 0;
    __syncthreads();
    const int info = ldc(a.tile_info, wt / WPT);
    const int valid = min(max((info >> 8) - (int)(wt % WPT) * TS, 0), TS);
    uint64_t vm[S];
#pragma unroll
    for (int s = 0; s < S; ++s) vm[s] = ballot(lane * S + s < valid);
    int dummy[S];
    for (;;) {
      const int q = next_item(&next_q);
      if (q >= Q) break;
      const int4 set = ldc(a.sets, a.set_begin + q0 + q);
      int acc;
      if constexpr (S == 4) {
        const uint32_t lds_lane =
            (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) float *)xs + (uint32_t)lane * 16u;
        acc = eval_set_s4_count(lds_lane, lane, set, a.conds, vm);
      } else {
        acc = eval_set<S, false>(xs, lane, set, a.conds, vm, dummy);
      }
      if (lane < a.nc) cnt[q * a.nc + lane] += acc;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < Q * a.nc; i += blockDim.x) {
    const int v = cnt[i];
    if (v == 0) continue;
    const int q = i / a.nc, c = i - (i / a.nc) * a.nc;
    const int64_t p = q0 + q;
    if (CONF) atomicAdd(&a.confusion[(p * a.nc + label) * a.nc + c], v);
    if (c == label) atomicAdd(&a.correct[p], v);
  }
}

// Prediction for one rule set over row-major rows: one wave per 64*S rows.
template <int S>
__global__ __launch_bounds__(64) void k_predict(const float *__restrict__ rows, int64_t n,
                                                int32_t nf, const int4 *__restrict__ sets,
                                                int32_t set_idx, const int4 *__restrict__ rules,
                                                const uint4 *__restrict__ conds,
                                                int32_t *__restrict__ out) {
  constexpr int TS = 64 * S;
  extern __shared__ __align__(16) float xs[];  // [nf][TS]
  const int lane = threadIdx.x;
  const int4 set = ldc(sets, set_idx);
  const int64_t base = (int64_t)blockIdx.x * TS;
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
  eval_set<S, true>(xs, lane, set, conds, vm, pred);
#pragma unroll
  for (int s = 0; s < S; ++s)
    if (lane * S + s < m) out[base + lane * S + s] = pred[s];
}

template <int S>
hipError_t hard_dispatch(const HardArgs &a, dim3 grid, size_t lds, bool conf, hipStream_t st) {
  if (conf)
    hipLaunchKernelGGL((k_hard<S, true>), grid, dim3(kHardBlock), lds, st, a);
  else
    hipLaunchKernelGGL((k_hard<S, false>), grid, dim3(kHardBlock), lds, st, a);
  return hipGetLastError();
}

constexpr size_t kMaxLds = 160 * 1024;

}  // namespace

hipError_t launch_hard_eval(const HardLaunch &h, hipStream_t st) {
  const DatasetRec &ds = *h.ds;
  const PopRec &pop = *h.pop;
  if (h.set_count <= 0) return hipSuccess;
  HardArgs a{};
  a.x_fm = ds.x_fm;
  a.n_pad = ds.n_pad;
  a.nf = ds.nf;
  a.nc = ds.nc;
  a.tile_info = ds.tile_info;
  a.sets = pop.sets;
  a.rules = pop.rules;
  a.conds = pop.hconds;
  a.set_begin = h.set_begin;
  a.set_count = h.set_count;
  a.correct = h.correct;
  a.confusion = h.confusion;
  a.sets_per_chunk = h.sets_per_chunk;
  a.tiles_per_group = h.tiles_per_group;
  int64_t n_groups = 0;
  for (int c = 0; c < ds.nc; ++c) {
    a.region_tile0[c] = ds.region_tile0[c];
    a.region_tiles[c] = ds.region_tiles[c];
    n_groups += (ds.region_tiles[c] + h.tiles_per_group - 1) / h.tiles_per_group;
  }
  if (n_groups == 0) return hipSuccess;
  const int64_t n_chunks = (h.set_count + h.sets_per_chunk - 1) / h.sets_per_chunk;
  const size_t lds = (size_t)ds.nf * 64 * h.samples_per_lane * 4 +
                     (size_t)h.sets_per_chunk * ds.nc * 4;
  if (lds > kMaxLds || n_groups > 65535 || n_chunks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)n_chunks, (unsigned)n_groups);
  const bool conf = h.confusion != nullptr;
  switch (h.samples_per_lane) {
    case 4: return hard_dispatch<4>(a, grid, lds, conf, st);
    case 2: return hard_dispatch<2>(a, grid, lds, conf, st);
    case 1: return hard_dispatch<1>(a, grid, lds, conf, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_predict(const PopRec &pop, int32_t set, const float *rows, int64_t n,
                          int32_t *pred, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if ((size_t)pop.nf * 256 * 4 <= kMaxLds) {
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_predict<4>, dim3((unsigned)blocks), dim3(64), (size_t)pop.nf * 256 * 4,
                       st, rows, n, pop.nf, pop.sets, set, pop.rules, pop.hconds, pred);
  } else if ((size_t)pop.nf * 64 * 4 <= kMaxLds) {
    const int64_t blocks = (n + 63) / 64;
    hipLaunchKernelGGL(k_predict<1>, dim3((unsigned)blocks), dim3(64), (size_t)pop.nf * 64 * 4,
                       st, rows, n, pop.nf, pop.sets, set, pop.rules, pop.hconds, pred);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace aerl
