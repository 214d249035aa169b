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
#include "hard_block.h"
#include "predict_block.h"
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
  const uint4 *conds;
  const uint4 *heads;
  int32_t set_begin, set_count;
  int32_t *correct;
  int32_t *confusion;
  uint32_t *part;
  int32_t sets_per_chunk, tiles_per_group, n_chunks;
  int32_t region_tile0[AERL_MAX_CLASSES];
  int32_t region_tiles[AERL_MAX_CLASSES];
};

// CAT: the population has categorical conditions (their walk body is left
// out of the other instantiation, which keeps the common walk's code tight).
// C10: single-tile groups (10-bit LDS counters).
template <int S, bool CAT, bool C10>
__global__ __launch_bounds__(kHardBlock) AERL_HARD_SGPR_CAP void k_hard(const HardArgs a) {
  extern __shared__ __align__(16) float smem[];
  __shared__ int32_t sh[2];
  // Which class region and which tiles this block covers (uniform loop).
  HardTask t;
  t.x_fm = a.x_fm;
  t.n_pad = a.n_pad;
  t.nf = a.nf;
  t.nc = a.nc;
  t.tile_info = a.tile_info;
  t.sets = a.sets + a.set_begin;
  t.conds = a.conds;
  t.heads = a.heads;
  t.correct = a.correct;
  t.confusion = a.confusion;
  t.part = nullptr;
  t.part_stride = 0;
  t.label = 0;
  t.tile_lo = t.tile_hi = 0;
  // one-dimensional grid, set chunk fastest: consecutive blocks share a tile
  // group, and (blocks being spread over the XCDs in turn) an XCD keeps
  // seeing the same chunk's records when the chunk count divides eight
  const int chunk = (int)(blockIdx.x % (unsigned)a.n_chunks);
  {
    int g = (int)(blockIdx.x / (unsigned)a.n_chunks);
    for (int c = 0; c < a.nc; ++c) {
      const int ng = (a.region_tiles[c] + a.tiles_per_group - 1) / a.tiles_per_group;
      if (g < ng) {
        t.label = c;
        t.tile_lo = a.region_tile0[c] + g * a.tiles_per_group;
        t.tile_hi = min(t.tile_lo + a.tiles_per_group, a.region_tile0[c] + a.region_tiles[c]);
        break;
      }
      g -= ng;
    }
  }
  t.q0 = chunk * a.sets_per_chunk;
  t.Q = min(a.sets_per_chunk, a.set_count - t.q0);
  if (C10 && a.part) {
    const int wpc = hard_part_chunk_words(a.sets_per_chunk, a.nc);
    t.part = a.part + (int64_t)chunk * wpc;
    t.part_stride = a.n_chunks * wpc;
  }
  hard_block<S, CAT, C10>(t, smem, sh);
}

// Sums the per-tile counter words of a hard-eval launch over the tiles of
// each class region.  A tile's row holds, chunk by chunk of Q rule sets,
// the 10-bit counters of classes 0..nc-2 among the tile's real samples,
// counter i = q*(nc-1) + c of the chunk's set q in bits 10*(i%3) of word
// i/3 (at most two words per set); class nc-1 gets the rest of them.
// Thread p of block (x, y) takes rule set 256x + p over the tiles of slice
// y (neighbouring threads read neighbouring words of a tile's row) and adds
// each class region's totals to the outputs.
constexpr int kReduceBlock = 256;
__global__ __launch_bounds__(kReduceBlock) void k_hard_reduce(
    const uint32_t *__restrict__ part, const int32_t *__restrict__ tile_info, int64_t n_tiles,
    int32_t n_sets, int32_t Q, int32_t nc, int32_t *__restrict__ correct,
    int32_t *__restrict__ confusion) {
  const int p = blockIdx.x * kReduceBlock + threadIdx.x;
  if (p >= n_sets) return;
  const int ncc = nc - 1;
  const int wpc = hard_part_chunk_words(Q, nc);
  const int64_t stride = (int64_t)((n_sets + Q - 1) / Q) * wpc;
  const int i = (p % Q) * ncc;
  const int64_t w = (int64_t)(p / Q) * wpc + i / 3;
  const int b = i % 3 * 10;
  // the word after w when the set's counters run into it, else w again (a
  // second read of the same word keeps the loop free of branches)
  const int w2 = i % 3 + ncc > 3 ? 1 : 0;
  const int64_t t0 = n_tiles * blockIdx.y / gridDim.y, t1 = n_tiles * (blockIdx.y + 1) / gridDim.y;
  int label = -1;
  int32_t c0 = 0, c1 = 0, c2 = 0, n = 0;
  auto emit = [&]() {
    if (label < 0) return;
    for (int c = 0; c < nc; ++c) {
      const int32_t v = c == nc - 1 ? n - c0 - c1 - c2 : c == 0 ? c0 : c == 1 ? c1 : c2;
      if (v == 0) continue;
      if (confusion) atomicAdd(&confusion[((int64_t)p * nc + label) * nc + c], v);
      if (c == label) atomicAdd(&correct[p], v);
    }
  };
  // tiles in order, the words of eight requested before they are used
  constexpr int kBatch = 8;
  for (int64_t tb = t0; tb < t1; tb += kBatch) {
    uint32_t lo[kBatch], hi[kBatch];
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      const int64_t t = min(tb + k, t1 - 1);  // past the slice: its last tile again, unused
      const uint32_t *row = part + t * stride + w;
      lo[k] = row[0];
      hi[k] = row[w2];
    }
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      if (tb + k >= t1) break;
      const int info = ldc(tile_info, tb + k);
      if ((info & 0xff) != label) {
        emit();
        label = info & 0xff;
        c0 = c1 = c2 = n = 0;
      }
      // the set's fields from bit 0 on, ten bits each (those past its ncc
      // are not used)
      const uint64_t v = ((uint64_t)hi[k] << 30 | lo[k]) >> b;
      c0 += (int32_t)(v & 1023u);
      if (ncc > 1) c1 += (int32_t)(v >> 10 & 1023u);
      if (ncc > 2) c2 += (int32_t)(v >> 20 & 1023u);
      n += info >> 8;
    }
  }
  emit();
}

// Prediction for one rule set over row-major rows: one wave per 64*S rows.
template <int S>
__global__ __launch_bounds__(64) void k_predict(const float *__restrict__ rows, int64_t n,
                                                int32_t nf, const int4 *__restrict__ sets,
                                                int32_t set_idx, const uint4 *__restrict__ conds,
                                                int32_t *__restrict__ out) {
  extern __shared__ __align__(16) float xs[];  // [nf][64*S]
  predict_block<S>(rows, n, nf, ldc(sets, set_idx), conds, out, (int64_t)blockIdx.x * 64 * S, xs);
}

template <int S>
hipError_t hard_dispatch(const HardArgs &a, dim3 grid, size_t lds, bool cat, bool c10,
                         hipStream_t st) {
  if (cat && c10)
    hipLaunchKernelGGL((k_hard<S, true, true>), grid, dim3(kHardBlock), lds, st, a);
  else if (cat)
    hipLaunchKernelGGL((k_hard<S, true, false>), grid, dim3(kHardBlock), lds, st, a);
  else if (c10)
    hipLaunchKernelGGL((k_hard<S, false, true>), grid, dim3(kHardBlock), lds, st, a);
  else
    hipLaunchKernelGGL((k_hard<S, false, false>), grid, dim3(kHardBlock), lds, st, a);
  return hipGetLastError();
}

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
  a.conds = pop.hconds;
  a.heads = pop.heads;
  a.set_begin = h.set_begin;
  a.set_count = h.set_count;
  a.correct = h.correct;
  a.confusion = h.confusion;
  a.part = h.part;
  if (h.part && !(hard_c10(h.tiles_per_group) && ds.nc >= 2 && ds.nc <= 4))
    return hipErrorInvalidValue;
  a.sets_per_chunk = h.sets_per_chunk;
  a.tiles_per_group = h.tiles_per_group;
  for (int c = 0; c < ds.nc; ++c) {
    a.region_tile0[c] = ds.region_tile0[c];
    a.region_tiles[c] = ds.region_tiles[c];
  }
  if (h.tiles_per_group < 1 || h.tiles_per_group > kMaxTilesPerBlock || h.sets_per_chunk < 1)
    return hipErrorInvalidValue;
  const int64_t n_groups = hard_group_count(ds, h.tiles_per_group);
  if (n_groups == 0) return hipSuccess;
  const int64_t n_chunks = (h.set_count + h.sets_per_chunk - 1) / h.sets_per_chunk;
  const bool c10 = hard_c10(h.tiles_per_group);
  const size_t lds = hard_block_lds(ds.nf, h.samples_per_lane, h.sets_per_chunk, ds.nc, c10);
  if (lds > kDynLdsMax || n_chunks * n_groups > kMaxHardBlocks) return hipErrorInvalidValue;
  a.n_chunks = (int32_t)n_chunks;
  const dim3 grid((unsigned)(n_chunks * n_groups));
  switch (h.samples_per_lane) {
    case 4: return hard_dispatch<4>(a, grid, lds, pop.n_cat > 0, c10, st);
    case 2: return hard_dispatch<2>(a, grid, lds, pop.n_cat > 0, c10, st);
    case 1: return hard_dispatch<1>(a, grid, lds, pop.n_cat > 0, c10, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_hard_reduce(const HardLaunch &h, int n_cu, hipStream_t st) {
  const DatasetRec &ds = *h.ds;
  if (h.set_count <= 0 || ds.n_tiles == 0) return hipSuccess;
  if (!h.part || ds.nc < 2 || ds.nc > 4 || h.sets_per_chunk < 1) return hipErrorInvalidValue;
  const int64_t bx = (h.set_count + kReduceBlock - 1) / kReduceBlock;
  const int64_t by = std::max<int64_t>(1, std::min<int64_t>(ds.n_tiles, (2LL * n_cu + bx - 1) / bx));
  hipLaunchKernelGGL(k_hard_reduce, dim3((unsigned)bx, (unsigned)by), dim3(kReduceBlock), 0, st,
                     h.part, ds.tile_info, ds.n_tiles, h.set_count, h.sets_per_chunk, ds.nc,
                     h.correct, h.confusion);
  return hipGetLastError();
}

hipError_t launch_predict(const PopRec &pop, int32_t set, const float *rows, int64_t n,
                          int32_t *pred, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if ((size_t)pop.nf * 256 * 4 <= kDynLdsMax) {
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_predict<4>, dim3((unsigned)blocks), dim3(64), (size_t)pop.nf * 256 * 4,
                       st, rows, n, pop.nf, pop.sets, set, pop.hconds, pred);
  } else if ((size_t)pop.nf * 64 * 4 <= kDynLdsMax) {
    const int64_t blocks = (n + 63) / 64;
    hipLaunchKernelGGL(k_predict<1>, dim3((unsigned)blocks), dim3(64), (size_t)pop.nf * 64 * 4,
                       st, rows, n, pop.nf, pop.sets, set, pop.hconds, pred);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace aerl
