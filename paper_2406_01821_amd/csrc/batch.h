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
  const uint4 *heads;
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
  bool cat;  // some item has categorical conditions
};

hipError_t launch_batch(const BatchLaunch &b, hipStream_t st);

constexpr size_t kBatchLdsMax = kDynLdsMax;

// Work split: rule sets and layout tiles per work item, and the LDS budget
// of a block's feature tile.
struct BatchSplit {
  int32_t Q = 512, TG = 1;
  size_t tile_budget = 64 * 1024;
};

// Samples per lane of an item with nf features: the most of {4, 2, 1} whose
// 64-lane tile of all features fits the budget.
int batch_samples_per_lane(int32_t nf, size_t tile_budget);

// One evaluation of a batch, as the table builder sees it.
struct BatchSource {
  const DatasetRec *ds;
  int32_t n_sets;
  const int4 *host_sets;  // host copy of the set records (cost estimates)
  const int4 *sets;       // device set records
  const uint4 *conds;     // device record stream
  const uint4 *heads;     // device head table
  int32_t *correct;       // device [n_sets]
  int32_t *confusion;     // device [n_sets][nc][nc] or null
  bool cat;               // the population has categorical conditions
};

// Work tables of a batch and their layout in one device copy.
struct BatchTables {
  std::vector<BatchItem> items;
  std::vector<BatchTask> tasks;
  std::vector<BatchZero> zero;
  size_t lds = 0;
  bool cat = false;
  size_t items_off = 0, tasks_off = 0, zero_off = 0, counter_off = 0, bytes = 0;
};

// Cuts every source into work items of Q rule sets x TG tiles (Q lowered per
// source until its block fits in LDS), sorts them by estimated cost
// (samples x nominal conditions), largest first, and lays the tables out.
void build_batch_tables(const std::vector<BatchSource> &src, const BatchSplit &sp,
                        BatchTables *t);

// Number of work items build_batch_tables makes for one source.
int64_t batch_task_count(const DatasetRec &ds, int32_t n_sets, const BatchSplit &sp);

// Writes the tables (t.bytes) to host memory `img` for a copy to device
// address `dev` and fills the launch record (persistent grid sized for n_cu
// CUs, never more blocks than work items).
void emit_batch_tables(const BatchTables &t, void *img, char *dev, int n_cu, BatchLaunch *l);

// Prediction work of a batch: one 64-thread block per task of 64*S rows.
struct PredictTask {
  const float *rows;  // device [n][nf] row-major
  const int4 *set;    // device set record of the rule set to apply
  const uint4 *conds; // device record stream of its population
  int32_t *out;       // device [n]
  int64_t n, row0;    // rows of the request, first row of this task
  int32_t nf, S;
};
struct PredictLaunch {
  const PredictTask *tasks;
  int32_t n_tasks;
  size_t lds;
};
hipError_t launch_predict_batch(const PredictLaunch &p, hipStream_t st);
int predict_samples_per_lane(int32_t nf);  // 4, or 1 when a 256-row tile does not fit LDS

}  // namespace aerl
