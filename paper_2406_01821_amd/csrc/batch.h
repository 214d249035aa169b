// Device tables of a ragged batch plan (shared by batch.cpp and ragged.hip).
#pragma once

#include "internal.h"

namespace aerl {

struct BatchItem {
  const float *x_fm;
  int64_t n_pad;
  const int32_t *tile_info;
  const int4 *sets;
  const uint4 *conds;
  int32_t *correct;
  int32_t *confusion;
  int32_t nf, nc, S, pad;
};

struct BatchTask {
  int32_t item, q0, Q, tile_lo, tile_hi, label, pad0, pad1;
};

struct BatchZero {
  int32_t *p;
  int64_t n;
};

struct BatchLaunch {
  const BatchItem *items;
  const BatchTask *tasks;
  const BatchZero *zero;
  int32_t *counter;
  int32_t n_tasks, n_zero;
  int64_t grid;
  size_t lds;
};

hipError_t launch_batch(const BatchLaunch &b, hipStream_t st);

}  // namespace aerl
