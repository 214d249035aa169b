// Ragged batches: many (dataset, population) evaluations in one persistent
// launch.  The host builds a work list (batch.cpp); every workgroup of the
// persistent grid pulls work items from a device counter until the list is
// exhausted, and runs the same block body as the one-launch-per-population
// kernel, so the results are bit-identical to it.  Each work item fixes its
// own tile width (samples per lane), so items of different feature counts
// share the launch.
#include "batch.h"
#include "hard_block.h"
#include "predict_block.h"

namespace aerl {

namespace {

constexpr int kBatchBlock = 1024;

__global__ void k_batch_zero(const BatchZero *__restrict__ z, int32_t n_z, int32_t *__restrict__ counter) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
  for (int e = blockIdx.x; e < n_z; e += gridDim.x) {
    int32_t *p = z[e].p;
    const int64_t n = z[e].n;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
  }
}

// CAT: some item has categorical conditions.
template <bool CAT>
__global__ __launch_bounds__(kBatchBlock) AERL_HARD_SGPR_CAP void k_hard_batch(
    const BatchItem *__restrict__ items, const BatchTask *__restrict__ tasks, int32_t n_tasks,
    int32_t *__restrict__ counter) {
  extern __shared__ __align__(16) float smem[];
  __shared__ int32_t sh[2];
  __shared__ int32_t task_id;
  for (;;) {
    if (threadIdx.x == 0) task_id = atomicAdd(counter, 1);
    __syncthreads();
    const int ti = __builtin_amdgcn_readfirstlane(task_id);
    if (ti >= n_tasks) break;  // same value in every thread: the whole block leaves
    const BatchTask tk = tasks[ti];
    const BatchItem it = items[tk.item];
    HardTask t;
    t.x_fm = it.x_fm;
    t.n_pad = it.n_pad;
    t.nf = it.nf;
    t.nc = it.nc;
    t.tile_info = it.tile_info;
    t.sets = it.sets;
    t.conds = it.conds;
    t.heads = it.heads;
    t.correct = it.correct;
    t.confusion = it.confusion;
    t.part = nullptr;
    t.part_stride = 0;
    t.q0 = tk.q0;
    t.Q = tk.Q;
    t.tile_lo = tk.tile_lo;
    t.tile_hi = tk.tile_hi;
    t.label = tk.label;
    switch (it.S) {
      case 4: hard_block<4, CAT>(t, smem, sh); break;
      case 2: hard_block<2, CAT>(t, smem, sh); break;
      default: hard_block<1, CAT>(t, smem, sh); break;
    }
  }
}

// Batched prediction: block b runs task b (64*S rows of one request).
__global__ __launch_bounds__(64) void k_predict_batch(const PredictTask *__restrict__ tasks) {
  extern __shared__ __align__(16) float xs[];
  const PredictTask t = tasks[blockIdx.x];
  const int4 set = ldc(t.set, 0);
  if (t.S == 4) {
    predict_block<4>(t.rows, t.n, t.nf, set, t.conds, t.out, t.row0, xs);
  } else {
    predict_block<1>(t.rows, t.n, t.nf, set, t.conds, t.out, t.row0, xs);
  }
}

}  // namespace

hipError_t launch_predict_batch(const PredictLaunch &p, hipStream_t st) {
  if (p.n_tasks <= 0) return hipSuccess;
  if (p.lds > kDynLdsMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_predict_batch, dim3((unsigned)p.n_tasks), dim3(64), p.lds, st, p.tasks);
  return hipGetLastError();
}

hipError_t launch_batch(const BatchLaunch &b, hipStream_t st) {
  if (b.n_zero > 0) {
    hipLaunchKernelGGL(k_batch_zero, dim3((unsigned)std::min<int64_t>(b.n_zero, 1024)), dim3(256), 0,
                       st, b.zero, b.n_zero, b.counter);
  } else {
    hipLaunchKernelGGL(k_batch_zero, dim3(1), dim3(64), 0, st, b.zero, 0, b.counter);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || b.n_tasks == 0) return e;
  if (b.cat)
    hipLaunchKernelGGL(k_hard_batch<true>, dim3((unsigned)b.grid), dim3(kBatchBlock), b.lds, st,
                       b.items, b.tasks, b.n_tasks, b.counter);
  else
    hipLaunchKernelGGL(k_hard_batch<false>, dim3((unsigned)b.grid), dim3(kBatchBlock), b.lds, st,
                       b.items, b.tasks, b.n_tasks, b.counter);
  return hipGetLastError();
}

}  // namespace aerl
