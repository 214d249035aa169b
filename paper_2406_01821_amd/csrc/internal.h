// Internal declarations shared by the libaerl sources (host and device).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "aerl.h"

namespace aerl {

struct Serve;

// ------------------------------------------------------------ error helpers
struct Error {
  aerl_status code;
  std::string msg;
};

// Fill ctx->err and return code.  printf-style message.
aerl_status fail(aerl_ctx *ctx, aerl_status code, const char *fmt, ...);

#define AERL_HIP(ctx, call)                                                              \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::aerl::fail((ctx), AERL_EDEVICE, "%s failed: %s (%s:%d)", #call,           \
                          hipGetErrorString(e_), __FILE__, __LINE__);                    \
  } while (0)

// ------------------------------------------------------------ packed records
// Rule set: {first hard-stream record, record count | head count << 16,
//            default class, nominal condition count}.
// Soft rule set: {first rule, rule count, first condition, condition count}.
// Rule (soft path): {first condition in the caller's order, condition count,
//                    class, 0}.
// Hard stream record (16 bytes), one per condition, rules of a set in order,
// then one closing record per set:
//   x: f*1024 (byte offset of the feature row in a 256-sample LDS tile)
//   y, z: fp32 operands (below)
//   w: flags | class << 12 | next << 18, where next is the byte offset (from
//      the set's first record) of the next rule's first record.
// Kinds (all exact rewrites of the caller's condition, pack.cpp), in this
// order inside a rule:
//   threshold, folded:      x[f] >= y            (no flag)
//                           x[f] <= y            (kRecLE)
//   threshold, zero coef:   y*x[f] > z           (kRecMul)
//   always true:            empty rule           (kRecAlways)
//   feature:                y*x[f] > z*x[g]      (kRecFF, g in the low bits)
//                           y*x[f] >= z*x[g]     (kRecFF | kRecGE)
// kRecLast marks a rule's last record.  The closing record is an always-true
// last record of the set's default class, so every walk ends in a commit.
// Soft condition (caller order): f | g << 12 | feature << 24 | (op >= 2) << 25
// | categorical << 26; a categorical condition's code set is in the packed
// image's mask array (caller order, two words per condition).
constexpr uint32_t kSoftFF = 1u << 24, kSoftCat = 1u << 26;
constexpr uint32_t kRecGMask = 0x1ffu;
constexpr uint32_t kRecMul = 1u << 0;     // threshold records only
constexpr uint32_t kRecAlways = 1u << 1;  // threshold records only
// Inside a rule the folded thresholds come >= first, then <=; the first <=
// record carries kRecDirChg, which moves the walk to its <= fast path.
constexpr uint32_t kRecDirChg = 1u << 2;  // threshold records only
// Categorical record: x[f] is a code k in 0..63 with bit k of the mask
// {y (codes 0..31), z (codes 32..63)} set.
constexpr uint32_t kRecCat = 1u << 3;     // non-feature records only
constexpr uint32_t kRecFF = 1u << 9;
constexpr uint32_t kRecGE = 1u << 10;  // feature records
constexpr uint32_t kRecLE = 1u << 10;  // threshold records
constexpr uint32_t kRecLast = 1u << 11;
// Records that leave the walk's fast path (the folded compare of a rule's
// non-last record in the walk's current direction).
constexpr uint32_t kRecSpecial = kRecFF | kRecLast | kRecMul | kRecAlways | kRecCat;
constexpr uint32_t kRecClsShift = 12;
constexpr uint32_t kRecNextShift = 18;
// Records of one rule set, closing record included: next-rule byte offsets
// fit 14 bits.
constexpr int32_t kMaxSetRecords = 1023;
// Head table (16 bytes per entry, parallel to the hard stream: the entries
// of a set start at its first record's index): one entry per rule in order,
// then one for the closing record.
//   x: the rule's first-record byte offset (from the set's first record) |
//      e1 << 14;  y: t1;  z: e2;  w: t2
// Tests i = 1, 2 stand for the rule's first two records: a folded threshold
// x[f] >= t gives e = 8f, t' = t, and x[f] <= t gives e = 8f + 4, t' = -t;
// any other record gives e = 0, t' = -inf.  With a tile's per-feature table
// {max x[f], -min x[f]} at byte offsets 8f and 8f + 4, table[e] < t' holds
// exactly when no sample of the tile passes the record, and then no sample
// of the tile can fire the rule.  (Tests of the third and fourth records
// skip about a third more record visits on the 2^20 x 64 workload, but the
// second 16-byte load per rule costs more than they save there.)
constexpr uint32_t kHeadOffMask = 0x3fffu;
constexpr uint32_t kHeadExtShift = 14;
// Sets with at most this many head entries take the filtered walk.
constexpr int32_t kMaxHeads = 64;
struct PackedLayout {
  size_t sets_off, ssets_off, rules_off, hconds_off, sconds_off, heads_off, cmask_off, total;
};

struct DatasetRec {
  int64_t n = 0, n_pad = 0, n_tiles = 0;
  int32_t nf = 0, nc = 0;
  float *x_fm = nullptr;       // [nf][n_pad]
  int32_t *y_pad = nullptr;    // [n_pad]
  int32_t *perm = nullptr;     // [n_pad]
  int32_t *tile_info = nullptr;// [n_tiles]: label | valid << 8
  float *tau = nullptr;        // [nf]
  float *inv_tau = nullptr;    // [nf], 1/tau (fp64 division rounded to float)
  int64_t class_count[AERL_MAX_CLASSES] = {};
  int32_t region_tile0[AERL_MAX_CLASSES] = {};
  int32_t region_tiles[AERL_MAX_CLASSES] = {};
};

struct PopRec {
  int32_t n_sets = 0, n_rules = 0, n_conds = 0, nf = 0, nc = 0;
  int32_t max_rules = 0, max_rule_conds = 0;
  int64_t nominal_conds = 0;
  int32_t max_set_conds = 0;
  int32_t n_ff = 0;            // feature-vs-feature conditions
  int32_t n_cat = 0;           // categorical conditions
  const int4 *sets = nullptr;
  const int4 *ssets = nullptr;
  const int4 *rules = nullptr;
  const uint4 *hconds = nullptr;
  const uint32_t *sconds = nullptr;
  const uint4 *heads = nullptr;
  const uint2 *cmask = nullptr;
  void *staging = nullptr;     // pinned host copy of the packed image (library-owned)
  size_t staging_cap = 0;      // its capacity in bytes
  hipEvent_t staged = nullptr; // completion of the staging copy
};

PackedLayout packed_layout(int32_t n_sets, int32_t n_rules, int32_t n_conds);
// Validates a host population; on success fills the rule and condition
// counts.  AERL_EINVAL with the message in ctx (ctx may be null).
aerl_status validate_population(aerl_ctx *ctx, const aerl_population *p, int32_t nf, int32_t nc,
                                int32_t *n_rules_out, int32_t *n_conds_out);
// Packed image of a validated population (PackedLayout::total bytes of host
// memory at dst); fills the summary fields of rec.
void pack_population_image(const aerl_population *p, int32_t nf, int32_t nc, int32_t n_rules,
                           int32_t n_conds, void *dst, PopRec *rec);

// Serving loop hooks (serve.cpp).
void serve_shutdown(aerl_ctx *ctx);
bool serve_uses_dataset(aerl_ctx *ctx, int32_t dataset_id);

struct BatchPlanRec;
void destroy_plan(BatchPlanRec *p);
struct PlanDeleter {
  void operator()(BatchPlanRec *p) const { destroy_plan(p); }
};

struct Evo;
void destroy_evo(Evo *e);
struct EvoDeleter {
  void operator()(Evo *e) const { destroy_evo(e); }
};

}  // namespace aerl

struct aerl_ctx {
  int device = 0;
  int n_cu = 0;
  std::string err;
  std::recursive_mutex mu;
  int32_t next_id = 1;
  std::unordered_map<int32_t, aerl::DatasetRec> datasets;
  std::unordered_map<int32_t, aerl::PopRec> pops;
  std::unordered_map<int32_t, std::unique_ptr<aerl::BatchPlanRec, aerl::PlanDeleter>> plans;
  std::map<std::string, std::array<int32_t, 3>> tuned;  // batch shape -> (sets, tiles, tile KiB)
  std::unordered_map<int32_t, std::unique_ptr<aerl::Evo, aerl::EvoDeleter>> evos;
  bool tune_file_loaded = false;
  aerl::Serve *serve = nullptr;
  void *noalloc_scratch = nullptr;  // this device's copy of the no-allocation scratch array
  // per-tile counter words of the plain hard path (grown on demand), and the
  // end of the last call that used them
  void *hard_part = nullptr;
  size_t hard_part_bytes = 0;
  hipEvent_t hard_part_done = nullptr;
  // pinned staging buffers of released populations, reused by later packs
  // (pinning host memory costs far more than packing into it)
  std::vector<std::pair<void *, size_t>> staging_pool;
};

namespace aerl {

// ------------------------------------------------------------ kernel launchers
// All return hipSuccess or the first HIP error.
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);

struct HardLaunch {
  const DatasetRec *ds;
  const PopRec *pop;
  int32_t set_begin, set_count;  // rule sets [set_begin, set_begin+set_count)
  int32_t *correct;              // indexed by set - set_begin
  int32_t *confusion;            // may be null
  int samples_per_lane;          // 1, 2 or 4
  int sets_per_chunk;
  int tiles_per_group;           // layout tiles per block
  // Per-tile counter words [n_tiles][set_count], or null.  With single-tile
  // groups and two to four classes the blocks store their counter words
  // here (one 32-bit word per rule set: classes 0..nc-2 in 10-bit fields)
  // and launch_hard_reduce sums them into the outputs; otherwise every
  // block adds its counts to the outputs with atomics.
  uint32_t *part = nullptr;
};
hipError_t launch_hard_eval(const HardLaunch &h, hipStream_t s);
// Sums h.part over the tiles of each class region into h.correct and
// h.confusion (which must be zeroed), about two workgroups per CU.
hipError_t launch_hard_reduce(const HardLaunch &h, int n_cu, hipStream_t s);
// Per-tile counter buffers the plain hard path uses: for launches of at
// least 4 Mi (tile, rule set) pairs (smaller ones flush per block, without
// a second kernel) and at most 512 MiB of counter words (larger ones flush
// per block too).
constexpr int64_t kHardPartMinPairs = (int64_t)4 << 20;
constexpr size_t kHardPartMaxBytes = (size_t)512 << 20;
// Workgroups of a hard-eval launch: one per (set chunk, tile group), in a
// one-dimensional grid of 1024-thread blocks whose work-item count must fit
// 32 bits.
constexpr int64_t kMaxHardBlocks = (((int64_t)1 << 32) - 1) / 1024;
inline int64_t hard_group_count(const DatasetRec &ds, int tiles_per_group) {
  int64_t g = 0;
  for (int c = 0; c < ds.nc; ++c) g += (ds.region_tiles[c] + tiles_per_group - 1) / tiles_per_group;
  return g;
}
inline int64_t hard_block_count(const DatasetRec &ds, int sets_per_chunk, int32_t n_sets,
                                int tiles_per_group) {
  const int64_t chunks = ((int64_t)std::max<int32_t>(n_sets, 0) + sets_per_chunk - 1) / sets_per_chunk;
  return chunks * hard_group_count(ds, tiles_per_group);
}

hipError_t launch_predict(const PopRec &pop, int32_t set, const float *rows, int64_t n,
                          int32_t *pred, hipStream_t s);

// Upload steps (layout.hip)
hipError_t launch_validate_count(const float *x, const int32_t *y, int64_t n, int32_t nf,
                                 int32_t nc, int32_t *block_counts, int32_t *flags,
                                 int64_t n_blocks, hipStream_t s);
hipError_t launch_scatter_transpose(const float *x, const int32_t *y, int64_t n, int32_t nf,
                                    int32_t nc, const int32_t *block_base, float *x_fm,
                                    int32_t *y_pad, int32_t *perm, int64_t n_pad,
                                    int64_t n_blocks, hipStream_t s);
// tau from the resident layout: part holds 2 * nf * kTauParts doubles.
constexpr int kTauParts = 64;
hipError_t launch_tau(const float *x_fm, const int32_t *tile_info, int64_t n_pad, int32_t nf,
                      int64_t n, double *part, float *tau, hipStream_t s);
constexpr int kUploadBlock = 256;  // samples per block in the upload kernels

// LDS of one CU, and the most dynamic LDS a hard-eval block may ask for (the
// rest is left for the kernels' own __shared__ words).
constexpr size_t kLdsPerCu = 160 * 1024;
constexpr size_t kStaticLds = 64;
constexpr size_t kDynLdsMax = kLdsPerCu - kStaticLds;

// Dynamic LDS of a hard-eval block: the feature tile (nf x 64*S floats),
// the tile's per-feature extremes and one prediction counter per (rule set,
// class) for every class but the last (a set predicts the last class for the
// block's samples the other counters leave): 16-bit counters, two per word,
// or, when the block covers one layout tile (a count is then at most 256),
// a set's 10-bit counters, three per word.  A block adds at most 256
// samples per layout tile to a counter, so it covers at most
// kMaxTilesPerBlock layout tiles.
constexpr int kMaxTilesPerBlock = 255;
// Most rule sets per block of the plain hard-eval path.
constexpr int kHardChunkMax = 2048;
__host__ __device__ inline int hard_counters_per_set(int nc) { return nc > 1 ? nc - 1 : 0; }
__host__ __device__ inline size_t hard_counter_bytes(int Q, int nc, bool c10) {
  const int ncc = hard_counters_per_set(nc);
  return c10 ? (size_t)Q * 4 * ((ncc + 2) / 3) : (((size_t)Q * ncc * 2 + 3) & ~size_t(3));
}
// Words of one chunk of Q rule sets in a row of the per-tile counter
// buffer: the chunk's 10-bit counters packed across sets, three per word.
__host__ __device__ inline int hard_part_chunk_words(int Q, int nc) {
  return (int)(((int64_t)Q * hard_counters_per_set(nc) + 2) / 3);
}
// Words per tile of the per-tile counter buffer: chunk k of Q rule sets at
// word k * hard_part_chunk_words(Q).
inline int64_t hard_part_row_words(int32_t n_sets, int Q, int nc) {
  return (int64_t)((n_sets + Q - 1) / Q) * hard_part_chunk_words(Q, nc);
}
// Blocks of one layout tile count in 10-bit fields.
inline bool hard_c10(int tiles_per_group) { return tiles_per_group == 1; }
inline size_t hard_block_lds(int nf, int S, int Q, int nc, bool c10 = false) {
  return (size_t)nf * 64 * S * 4 + (size_t)nf * 8 + hard_counter_bytes(Q, nc, c10);
}

// Soft path (soft.hip)
struct SoftLaunch {
  const DatasetRec *ds;
  const PopRec *pop;
  const float *coef, *coef2, *theta;
  const float *dloss;            // backward only
  float *loss;                   // forward only
  float *dcoef, *dcoef2, *dtheta;
  void *ws;
  size_t ws_bytes;
};
size_t soft_ws_bytes(const DatasetRec &ds, const PopRec &pop, bool backward);
bool soft_backward_supported(const DatasetRec &ds, const PopRec &pop);
hipError_t launch_soft_forward(const SoftLaunch &l, hipStream_t s);
hipError_t launch_soft_backward(const SoftLaunch &l, hipStream_t s);
// Softmax head (soft.hip): up to kSmaxMaxClasses classes; same workspace as
// the first-firing soft path (soft_ws_bytes).
constexpr int kSmaxMaxClasses = 16;
bool smax_supported(const DatasetRec &ds, const PopRec &pop);
hipError_t launch_smax_forward(const SoftLaunch &l, float beta, hipStream_t s);
hipError_t launch_smax_backward(const SoftLaunch &l, float beta, hipStream_t s);
hipError_t launch_smax_proba(const SoftLaunch &l, int32_t set, float beta, const float *rows,
                             int64_t n, float *probs, hipStream_t s);

// Fine-tuning (tune.hip): workspace layout and the epoch loop.
struct TuneLayout {
  size_t soft_off, grad_off, mom_off, dloss_off, total;
};
TuneLayout tune_layout(const DatasetRec &ds, const PopRec &pop);
struct TuneLaunch {
  const DatasetRec *ds;
  const PopRec *pop;
  float *coef, *coef2, *theta;  // updated in place
  float *loss_hist;             // [epochs + 1][n_sets] or null
  int32_t epochs, optimizer;
  float lr, beta1, beta2, eps;
  void *ws;
};
hipError_t run_finetune(const TuneLaunch &t, hipStream_t s);

// Evolution loop (evolve.cpp): device arena layout of a run.
constexpr int32_t kMaxEvolveRules = 64;
struct EvolveArena {
  size_t pack_off, pack_bytes, correct_off, param_off, tune_off, tune_bytes, staging_bytes, total;
  bool tune_ok;
};
EvolveArena evolve_arena(const DatasetRec &ds, const aerl_evolve_cfg &c);
// aerl_pack_population through a caller-owned pinned staging buffer (no
// per-call host allocation); the caller keeps the staging alive until the
// copy has completed on stream.
aerl_status pack_staged(aerl_ctx *ctx, const aerl_population *pop, int32_t nf, int32_t nc, void *ws,
                        size_t ws_bytes, void *staging, size_t staging_bytes, hipStream_t stream,
                        int32_t *pop_id);

// Device address of the current device's no-allocation scratch array
// (AERL_NOALLOC_SCRATCH_BYTES), resolved once per device; the device must be
// current.
hipError_t noalloc_scratch(int device, void **out);

}  // namespace aerl
