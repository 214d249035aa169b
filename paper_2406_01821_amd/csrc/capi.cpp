// C ABI of libaerl: context, datasets, populations and the direct calls.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <climits>
#include <cstring>

#include "internal.h"

namespace aerl {

aerl_status fail(aerl_ctx *ctx, aerl_status code, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

namespace {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct DatasetMem {
  int64_t n_pad_max, n_tiles_max, n_blocks;
  size_t x_off, y_off, perm_off, tile_off, tau_off, counts_off, base_off, flags_off, tpart_off, total;
};

DatasetMem dataset_mem(int64_t n, int32_t nf, int32_t nc) {
  DatasetMem m{};
  m.n_pad_max = n > 0 ? ((n + AERL_TILE - 1) / AERL_TILE + nc) * AERL_TILE : 0;
  m.n_tiles_max = m.n_pad_max / AERL_TILE;
  m.n_blocks = (n + kUploadBlock - 1) / kUploadBlock;
  size_t off = 0;
  m.x_off = off;     off = align256(off + sizeof(float) * (size_t)nf * (size_t)m.n_pad_max);
  m.y_off = off;     off = align256(off + sizeof(int32_t) * (size_t)m.n_pad_max);
  m.perm_off = off;  off = align256(off + sizeof(int32_t) * (size_t)m.n_pad_max);
  m.tile_off = off;  off = align256(off + sizeof(int32_t) * (size_t)(m.n_tiles_max + 1));
  m.tau_off = off;   off = align256(off + sizeof(float) * 2 * (size_t)nf);  // tau, 1/tau
  m.counts_off = off; off = align256(off + sizeof(int32_t) * (size_t)(m.n_blocks * nc + 1));
  m.base_off = off;  off = align256(off + sizeof(int32_t) * (size_t)(m.n_blocks * nc + 1));
  m.flags_off = off; off = align256(off + sizeof(int32_t) * 2);
  m.tpart_off = off; off = align256(off + sizeof(double) * 2 * (size_t)nf * kTauParts);
  m.total = off;
  return m;
}

aerl_status check_dataset_args(aerl_ctx *ctx, int64_t n, int32_t nf, int32_t nc) {
  if (nf < 1 || nf > AERL_MAX_FEATURES)
    return fail(ctx, AERL_EINVAL, "n_features %d outside [1, %d]", nf, AERL_MAX_FEATURES);
  if (nc < 1 || nc > AERL_MAX_CLASSES)
    return fail(ctx, AERL_EINVAL, "n_classes %d outside [1, %d]", nc, AERL_MAX_CLASSES);
  // Slots of the label-grouped layout (original indices, scatter bases) are
  // int32: the padded sample count must stay below 2^31.
  if (n < 0 || n > aerl_max_samples(nc))
    return fail(ctx, AERL_EINVAL, "n = %lld outside [0, %lld] for %d classes", (long long)n,
                (long long)aerl_max_samples(nc), nc);
  return AERL_OK;
}

// Class regions of the label-grouped layout from the per-class counts
// (d.nc set): each region padded to whole tiles, in class order.
void set_regions(DatasetRec &d, const int64_t *counts) {
  int64_t tile = 0;
  for (int c = 0; c < d.nc; ++c) {
    d.class_count[c] = counts[c];
    d.region_tile0[c] = (int32_t)tile;
    d.region_tiles[c] = (int32_t)((counts[c] + AERL_TILE - 1) / AERL_TILE);
    tile += d.region_tiles[c];
  }
  d.n_tiles = tile;
  d.n_pad = tile * AERL_TILE;
}

// RAII pinned host buffer.
struct Pinned {
  void *p = nullptr;
  ~Pinned() { if (p) (void)hipHostFree(p); }
};

// Launch configuration of the plain hard-eval path.  Large set chunks (up to
// 2048 rule sets per block) over single tiles: every staged tile serves many
// rule sets, so the per-tile barrier and the restaging of the dataset per
// chunk are amortized; chunks shrink only when the grid would be too small
// to fill the GPU (down to about 64 sets, or 32, two per wave of a block,
// on tables of at most four tiles, whose restaging costs next to nothing:
// on the 569 x 30 table with 100 sets 11.6 us per call against 13.3 us with
// 64-set chunks, while the 64-run ragged mix launched run by run slows by
// 5% with 32-set chunks) or their counters do not fit in LDS.
void hard_config(const DatasetRec &ds, int32_t n_sets, int n_cu, int *S, int *Q, int *TG) {
  const int64_t tiles = std::max<int64_t>(ds.n_tiles, 1);
  const int64_t target = 4LL * n_cu;
  const int q_floor = tiles <= 4 ? 32 : 64;
  int q = (int)std::min<int64_t>(std::max<int32_t>(n_sets, 1), kHardChunkMax);
  // Two blocks per CU (eight waves per SIMD) hide the latency of the scalar
  // record loads and LDS reads far better than one: take the most samples per
  // lane whose tile leaves room for two blocks with a chunk of at least 64
  // sets (measured: two samples per lane at two blocks beat four at one),
  // and then the largest chunk that keeps two blocks; with no such S, the
  // most samples per lane that fit one block.
  const size_t half = kLdsPerCu / 2 - kStaticLds;
  const int q_min2 = std::min(q, 64);
  int s = 4;
  while (s > 1 && hard_block_lds(ds.nf, s, q_min2, ds.nc) > half) s >>= 1;
  size_t budget = half;
  if (hard_block_lds(ds.nf, s, q_min2, ds.nc) > half) {
    s = 4;
    while (s > 1 && (size_t)ds.nf * 256 * s > 150 * 1024) s >>= 1;
    budget = kDynLdsMax;
  }
  *S = s;
  // Chunk size and tiles per group, planned first for single-tile groups
  // (10-bit counters) and again with 16-bit counters when the launch limit
  // forces larger groups.
  const int q_top = q;
  for (bool c10 = true;; c10 = false) {
    q = q_top;
    while (q > 1 && hard_block_lds(ds.nf, s, q, ds.nc, c10) > budget) q = (q + 1) / 2;
    while (q > q_floor && ((n_sets + q - 1) / q) * tiles < target) q = (q + 1) / 2;
    // equal chunks (a short last chunk leaves its blocks underused)
    const int chunks = (std::max<int32_t>(n_sets, 1) + q - 1) / q;
    *Q = (std::max<int32_t>(n_sets, 1) + chunks - 1) / chunks;
    // Single-tile groups (measured fastest: larger groups leave a partly
    // filled last round of blocks), unless the grid would exceed the launch
    // limit; then the fewest tiles per group that fit it.
    int tg = 1;
    while (tg < kMaxTilesPerBlock && hard_block_count(ds, *Q, n_sets, tg) > kMaxHardBlocks) ++tg;
    *TG = tg;
    if (!c10 || hard_c10(tg)) break;
  }
}

}  // namespace
}  // namespace aerl

namespace aerl {
namespace {
void set_device_views(PopRec &rec, const PackedLayout &L, void *ws) {
  char *b = static_cast<char *>(ws);
  rec.sets = reinterpret_cast<const int4 *>(b + L.sets_off);
  rec.ssets = reinterpret_cast<const int4 *>(b + L.ssets_off);
  rec.rules = reinterpret_cast<const int4 *>(b + L.rules_off);
  rec.hconds = reinterpret_cast<const uint4 *>(b + L.hconds_off);
  rec.sconds = reinterpret_cast<const uint32_t *>(b + L.sconds_off);
  rec.heads = reinterpret_cast<const uint4 *>(b + L.heads_off);
  rec.cmask = reinterpret_cast<const uint2 *>(b + L.cmask_off);
}
}  // namespace

// Pinned staging for a packed image of `bytes`: the smallest pooled buffer
// that holds it without wasting more than its size again, else a new one.
static hipError_t take_staging(aerl_ctx *ctx, size_t bytes, void **p, size_t *cap) {
  size_t best = SIZE_MAX;
  size_t k = ctx->staging_pool.size();
  for (size_t i = 0; i < ctx->staging_pool.size(); ++i) {
    const size_t c = ctx->staging_pool[i].second;
    if (c >= bytes && c / 2 <= bytes && c < best) {
      best = c;
      k = i;
    }
  }
  if (k < ctx->staging_pool.size()) {
    *p = ctx->staging_pool[k].first;
    *cap = ctx->staging_pool[k].second;
    ctx->staging_pool.erase(ctx->staging_pool.begin() + (std::ptrdiff_t)k);
    return hipSuccess;
  }
  *cap = 0;
  hipError_t e = hipHostMalloc(p, bytes, hipHostMallocDefault);
  if (e == hipSuccess) *cap = bytes;
  return e;
}

// Returns a staging buffer whose copy has completed to the pool, which keeps
// at most kStagingPoolBuffers buffers and kStagingPoolBytes bytes (the
// oldest go first).
constexpr size_t kStagingPoolBuffers = 8;
constexpr size_t kStagingPoolBytes = (size_t)512 << 20;
static void give_staging(aerl_ctx *ctx, void *p, size_t cap) {
  if (!p) return;
  ctx->staging_pool.emplace_back(p, cap);
  size_t total = 0;
  for (const auto &b : ctx->staging_pool) total += b.second;
  while (!ctx->staging_pool.empty() &&
         (ctx->staging_pool.size() > kStagingPoolBuffers || total > kStagingPoolBytes)) {
    total -= ctx->staging_pool.front().second;
    (void)hipHostFree(ctx->staging_pool.front().first);
    ctx->staging_pool.erase(ctx->staging_pool.begin());
  }
}

aerl_status pack_staged(aerl_ctx *ctx, const aerl_population *pop, int32_t nf, int32_t nc, void *ws,
                        size_t ws_bytes, void *staging, size_t staging_bytes, hipStream_t stream,
                        int32_t *pop_id) {
  int32_t n_rules = 0, n_conds = 0;
  aerl_status st = validate_population(ctx, pop, nf, nc, &n_rules, &n_conds);
  if (st) return st;
  const PackedLayout L = packed_layout(pop->n_sets, n_rules, n_conds);
  if (!ws || ((uintptr_t)ws & 255)) return fail(ctx, AERL_EINVAL, "ws is NULL or not 256-byte aligned");
  if (ws_bytes < L.total || staging_bytes < L.total)
    return fail(ctx, AERL_ENOMEM, "ws or staging holds less than the %zu bytes needed", L.total);
  PopRec rec;
  pack_population_image(pop, nf, nc, n_rules, n_conds, staging, &rec);
  AERL_HIP(ctx, hipMemcpyAsync(ws, staging, L.total, hipMemcpyHostToDevice, stream));
  set_device_views(rec, L, ws);
  const int32_t id = ctx->next_id++;
  ctx->pops[id] = rec;  // staging is the caller's: nothing to free on release
  *pop_id = id;
  return AERL_OK;
}
}  // namespace aerl

using namespace aerl;

extern "C" {

aerl_status aerl_create(aerl_ctx **out, int device_ordinal) {
  if (!out) return AERL_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device_ordinal < 0 || device_ordinal >= count)
    return AERL_EINVAL;
  aerl_ctx *ctx = new (std::nothrow) aerl_ctx();
  if (!ctx) return AERL_ENOMEM;
  ctx->device = device_ordinal;
  if (hipSetDevice(device_ordinal) != hipSuccess ||
      hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, device_ordinal) !=
          hipSuccess ||
      noalloc_scratch(device_ordinal, &ctx->noalloc_scratch) != hipSuccess) {
    delete ctx;
    return AERL_EDEVICE;
  }
  *out = ctx;
  return AERL_OK;
}

void aerl_destroy(aerl_ctx *ctx) {
  if (!ctx) return;
  serve_shutdown(ctx);
  if (ctx->hard_part_done) {
    (void)hipEventSynchronize(ctx->hard_part_done);
    (void)hipEventDestroy(ctx->hard_part_done);
  }
  if (ctx->hard_part) (void)hipFree(ctx->hard_part);
  for (auto &kv : ctx->pops) {
    if (kv.second.staged) {
      (void)hipEventSynchronize(kv.second.staged);
      (void)hipEventDestroy(kv.second.staged);
    }
    if (kv.second.staging) (void)hipHostFree(kv.second.staging);
  }
  for (const auto &b : ctx->staging_pool) (void)hipHostFree(b.first);
  delete ctx;
}

const char *aerl_last_error(const aerl_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int64_t aerl_max_samples(int32_t n_classes) {
  if (n_classes < 1 || n_classes > AERL_MAX_CLASSES) return 0;
  const int64_t tiles = (int64_t)INT32_MAX / AERL_TILE;  // whole padded tiles below 2^31
  return (tiles - n_classes) * AERL_TILE;
}

aerl_status aerl_dataset_bytes(int64_t n, int32_t f, int32_t n_classes, size_t *bytes) {
  if (!bytes) return AERL_EINVAL;
  aerl_status st = check_dataset_args(nullptr, n, f, n_classes);
  if (st) return st;
  *bytes = dataset_mem(n, f, n_classes).total;
  return AERL_OK;
}

aerl_status aerl_upload_dataset(aerl_ctx *ctx, const float *x, const int32_t *y, int64_t n,
                                int32_t nf, int32_t nc, void *mem, size_t mem_bytes,
                                hipStream_t stream, int32_t *dataset_id) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->err.clear();
  if (!dataset_id) return fail(ctx, AERL_EINVAL, "dataset_id is NULL");
  aerl_status st = check_dataset_args(ctx, n, nf, nc);
  if (st) return st;
  if (n > 0 && (!x || !y)) return fail(ctx, AERL_EINVAL, "x or y is NULL");
  if (!mem || ((uintptr_t)mem & 255)) return fail(ctx, AERL_EINVAL, "mem is NULL or not 256-byte aligned");
  const DatasetMem M = dataset_mem(n, nf, nc);
  if (mem_bytes < M.total)
    return fail(ctx, AERL_ENOMEM, "mem holds %zu bytes, %zu needed", mem_bytes, M.total);
  AERL_HIP(ctx, hipSetDevice(ctx->device));
  char *base = static_cast<char *>(mem);
  DatasetRec d;
  d.n = n;
  d.nf = nf;
  d.nc = nc;
  d.x_fm = reinterpret_cast<float *>(base + M.x_off);
  d.y_pad = reinterpret_cast<int32_t *>(base + M.y_off);
  d.perm = reinterpret_cast<int32_t *>(base + M.perm_off);
  d.tile_info = reinterpret_cast<int32_t *>(base + M.tile_off);
  d.tau = reinterpret_cast<float *>(base + M.tau_off);
  d.inv_tau = d.tau + nf;
  int32_t *counts_dev = reinterpret_cast<int32_t *>(base + M.counts_off);
  int32_t *base_dev = reinterpret_cast<int32_t *>(base + M.base_off);
  int32_t *flags_dev = reinterpret_cast<int32_t *>(base + M.flags_off);

  const size_t nbc = (size_t)M.n_blocks * nc;
  Pinned hbuf;
  const size_t hbytes = sizeof(int32_t) * (2 * nbc + 2 + (size_t)M.n_tiles_max + 1);
  AERL_HIP(ctx, hipHostMalloc(&hbuf.p, hbytes, hipHostMallocDefault));
  int32_t *h_counts = static_cast<int32_t *>(hbuf.p);
  int32_t *h_base = h_counts + nbc;
  int32_t *h_flags = h_base + nbc;
  int32_t *h_tiles = h_flags + 2;

  AERL_HIP(ctx, launch_fill_i32(flags_dev, 2, 0, stream));
  AERL_HIP(ctx, launch_validate_count(x, y, n, nf, nc, counts_dev, flags_dev, M.n_blocks, stream));
  if (nbc) AERL_HIP(ctx, hipMemcpyAsync(h_counts, counts_dev, nbc * 4, hipMemcpyDeviceToHost, stream));
  AERL_HIP(ctx, hipMemcpyAsync(h_flags, flags_dev, 8, hipMemcpyDeviceToHost, stream));
  AERL_HIP(ctx, hipStreamSynchronize(stream));
  if (h_flags[0]) return fail(ctx, AERL_EINVAL, "x holds a non-finite value");
  if (h_flags[1]) return fail(ctx, AERL_EINVAL, "y holds a label outside [0, %d)", nc);

  // Class regions, each padded to whole tiles, in class order.
  int64_t counts[AERL_MAX_CLASSES] = {};
  for (int c = 0; c < nc; ++c)
    for (int64_t b = 0; b < M.n_blocks; ++b) counts[c] += h_counts[b * nc + c];
  set_regions(d, counts);
  if (d.n_pad > M.n_pad_max) return fail(ctx, AERL_EINVAL, "internal: layout overflow");
  for (int c = 0; c < nc; ++c) {
    const int64_t tile = d.region_tile0[c];
    for (int64_t t = 0; t < d.region_tiles[c]; ++t) {
      const int64_t valid = std::min<int64_t>(AERL_TILE, counts[c] - t * AERL_TILE);
      h_tiles[tile + t] = c | (int32_t)(valid << 8);
    }
    int64_t run = tile * AERL_TILE;
    for (int64_t b = 0; b < M.n_blocks; ++b) {
      h_base[b * nc + c] = (int32_t)run;
      run += h_counts[b * nc + c];
    }
  }
  // The x_fm rows use stride n_pad.
  if (d.n_tiles) AERL_HIP(ctx, hipMemcpyAsync(d.tile_info, h_tiles, (size_t)d.n_tiles * 4, hipMemcpyHostToDevice, stream));
  if (nbc) AERL_HIP(ctx, hipMemcpyAsync(base_dev, h_base, nbc * 4, hipMemcpyHostToDevice, stream));
  AERL_HIP(ctx, launch_fill_i32(reinterpret_cast<int32_t *>(d.x_fm), (int64_t)nf * d.n_pad, 0, stream));
  AERL_HIP(ctx, launch_fill_i32(d.y_pad, d.n_pad, -1, stream));
  AERL_HIP(ctx, launch_fill_i32(d.perm, d.n_pad, -1, stream));
  AERL_HIP(ctx, launch_scatter_transpose(x, y, n, nf, nc, base_dev, d.x_fm, d.y_pad, d.perm, d.n_pad,
                                         M.n_blocks, stream));
  AERL_HIP(ctx, launch_tau(d.x_fm, d.tile_info, d.n_pad, nf, n,
                           reinterpret_cast<double *>(base + M.tpart_off), d.tau, stream));
  AERL_HIP(ctx, hipStreamSynchronize(stream));
  const int32_t id = ctx->next_id++;
  ctx->datasets[id] = d;
  *dataset_id = id;
  return AERL_OK;
}

aerl_status aerl_dataset_query(aerl_ctx *ctx, int32_t dataset_id, aerl_dataset_info *info) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (!info) return fail(ctx, AERL_EINVAL, "info is NULL");
  auto it = ctx->datasets.find(dataset_id);
  if (it == ctx->datasets.end()) return fail(ctx, AERL_ENOENT, "unknown dataset %d", dataset_id);
  const DatasetRec &d = it->second;
  std::memset(info, 0, sizeof *info);
  info->n = d.n;
  info->n_pad = d.n_pad;
  info->n_features = d.nf;
  info->n_classes = d.nc;
  for (int c = 0; c < d.nc; ++c) info->class_count[c] = d.class_count[c];
  info->x_fm = d.x_fm;
  info->y_pad = d.y_pad;
  info->perm = d.perm;
  info->tau = d.tau;
  return AERL_OK;
}

aerl_status aerl_release_dataset(aerl_ctx *ctx, int32_t dataset_id) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (!ctx->datasets.count(dataset_id)) return fail(ctx, AERL_ENOENT, "unknown dataset %d", dataset_id);
  if (serve_uses_dataset(ctx, dataset_id))
    return fail(ctx, AERL_ESTATE, "dataset %d has served requests in flight", dataset_id);
  ctx->datasets.erase(dataset_id);
  return AERL_OK;
}

aerl_status aerl_population_bytes(const aerl_population *pop, int32_t n_features, int32_t n_classes,
                                  size_t *bytes) {
  if (!bytes) return AERL_EINVAL;
  int32_t nr = 0, nc = 0;
  aerl_status st = validate_population(nullptr, pop, n_features, n_classes, &nr, &nc);
  if (st) return st;
  *bytes = packed_layout(pop->n_sets, nr, nc).total;
  return AERL_OK;
}


aerl_status aerl_pack_population(aerl_ctx *ctx, const aerl_population *pop, int32_t nf, int32_t nc,
                                 void *ws, size_t ws_bytes, hipStream_t stream, int32_t *pop_id) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->err.clear();
  if (!pop_id) return fail(ctx, AERL_EINVAL, "pop_id is NULL");
  int32_t n_rules = 0, n_conds = 0;
  aerl_status st = validate_population(ctx, pop, nf, nc, &n_rules, &n_conds);
  if (st) return st;
  const PackedLayout L = packed_layout(pop->n_sets, n_rules, n_conds);
  if (!ws || ((uintptr_t)ws & 255)) return fail(ctx, AERL_EINVAL, "ws is NULL or not 256-byte aligned");
  if (ws_bytes < L.total) return fail(ctx, AERL_ENOMEM, "ws holds %zu bytes, %zu needed", ws_bytes, L.total);
  AERL_HIP(ctx, hipSetDevice(ctx->device));
  PopRec rec;
  AERL_HIP(ctx, take_staging(ctx, L.total, &rec.staging, &rec.staging_cap));
  pack_population_image(pop, nf, nc, n_rules, n_conds, rec.staging, &rec);
  hipError_t e = hipMemcpyAsync(ws, rec.staging, L.total, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&rec.staged, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(rec.staged, stream);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(stream);
    if (rec.staged) (void)hipEventDestroy(rec.staged);
    give_staging(ctx, rec.staging, rec.staging_cap);
    return fail(ctx, AERL_EDEVICE, "staging copy failed: %s", hipGetErrorString(e));
  }
  set_device_views(rec, L, ws);
  const int32_t id = ctx->next_id++;
  ctx->pops[id] = rec;
  *pop_id = id;
  return AERL_OK;
}

aerl_status aerl_pack_population_host(const aerl_population *pop, int32_t nf, int32_t nc, void *dst,
                                      size_t dst_bytes) {
  int32_t n_rules = 0, n_conds = 0;
  aerl_status st = validate_population(nullptr, pop, nf, nc, &n_rules, &n_conds);
  if (st) return st;
  const PackedLayout L = packed_layout(pop->n_sets, n_rules, n_conds);
  if (!dst || dst_bytes < L.total) return AERL_ENOMEM;
  PopRec rec;
  pack_population_image(pop, nf, nc, n_rules, n_conds, dst, &rec);
  return AERL_OK;
}

aerl_status aerl_release_population(aerl_ctx *ctx, int32_t pop_id) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  auto it = ctx->pops.find(pop_id);
  if (it == ctx->pops.end()) return fail(ctx, AERL_ENOENT, "unknown population %d", pop_id);
  if (it->second.staged) {
    (void)hipEventSynchronize(it->second.staged);
    (void)hipEventDestroy(it->second.staged);
  }
  give_staging(ctx, it->second.staging, it->second.staging_cap);
  ctx->pops.erase(it);
  return AERL_OK;
}

// The context's per-tile counter buffer, at least `bytes` long, for a call
// on `stream`: the stream first waits for the last call that used it (calls
// that use it run one after another, across streams).  Grows it (after that
// call ends) when too small; *out stays null when the allocation fails, and
// the caller then counts with atomics instead.
static aerl_status hard_part_buffer(aerl_ctx *ctx, size_t bytes, hipStream_t stream,
                                    uint32_t **out) {
  *out = nullptr;
  if (!ctx->hard_part_done)
    AERL_HIP(ctx, hipEventCreateWithFlags(&ctx->hard_part_done, hipEventDisableTiming));
  if (ctx->hard_part_bytes < bytes) {
    AERL_HIP(ctx, hipEventSynchronize(ctx->hard_part_done));
    if (ctx->hard_part) AERL_HIP(ctx, hipFree(ctx->hard_part));
    ctx->hard_part = nullptr;
    ctx->hard_part_bytes = 0;
    if (hipMalloc(&ctx->hard_part, bytes) != hipSuccess) {
      (void)hipGetLastError();
      ctx->hard_part = nullptr;
      return AERL_OK;
    }
    ctx->hard_part_bytes = bytes;
  } else {
    AERL_HIP(ctx, hipStreamWaitEvent(stream, ctx->hard_part_done, 0));
  }
  *out = static_cast<uint32_t *>(ctx->hard_part);
  return AERL_OK;
}

static aerl_status eval_common(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id, int32_t *correct,
                               int32_t *confusion, int S, int Q, int TG, hipStream_t stream) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->err.clear();
  auto di = ctx->datasets.find(dataset_id);
  if (di == ctx->datasets.end()) return fail(ctx, AERL_ENOENT, "unknown dataset %d", dataset_id);
  auto pi = ctx->pops.find(pop_id);
  if (pi == ctx->pops.end()) return fail(ctx, AERL_ENOENT, "unknown population %d", pop_id);
  const DatasetRec &ds = di->second;
  const PopRec &pop = pi->second;
  if (pop.nf != ds.nf || pop.nc != ds.nc)
    return fail(ctx, AERL_EINVAL, "population has %d features / %d classes, dataset %d / %d", pop.nf,
                pop.nc, ds.nf, ds.nc);
  if (!correct && pop.n_sets > 0) return fail(ctx, AERL_EINVAL, "correct is NULL");
  HardLaunch h{};
  h.ds = &ds;
  h.pop = &pop;
  h.set_begin = 0;
  h.set_count = pop.n_sets;
  h.correct = correct;
  h.confusion = confusion;
  if (S == 0) {
    hard_config(ds, pop.n_sets, ctx->n_cu, &h.samples_per_lane, &h.sets_per_chunk, &h.tiles_per_group);
  } else {
    if (S != 1 && S != 2 && S != 4) return fail(ctx, AERL_EINVAL, "samples_per_lane %d not in {1,2,4}", S);
    if (Q < 1 || TG < 1) return fail(ctx, AERL_EINVAL, "sets_per_chunk and tiles_per_group must be >= 1");
    if (hard_block_lds(ds.nf, S, Q, ds.nc, hard_c10(TG)) > kDynLdsMax)
      return fail(ctx, AERL_EINVAL, "configuration needs more LDS than a workgroup can have");
    if (TG > kMaxTilesPerBlock)
      return fail(ctx, AERL_EINVAL, "tiles_per_group %d above %d", TG, kMaxTilesPerBlock);
    h.samples_per_lane = S;
    h.sets_per_chunk = Q;
    h.tiles_per_group = TG;
  }
  if (hard_block_count(ds, h.sets_per_chunk, pop.n_sets, h.tiles_per_group) > kMaxHardBlocks)
    return fail(ctx, AERL_EINVAL, "%lld workgroups exceed the launch limit %lld; raise tiles_per_group",
                (long long)hard_block_count(ds, h.sets_per_chunk, pop.n_sets, h.tiles_per_group),
                (long long)kMaxHardBlocks);
  AERL_HIP(ctx, hipSetDevice(ctx->device));
  // Large launches of single-tile groups with two to four classes store
  // per-tile counter words that a second kernel sums (far fewer output
  // atomics than a flush per block), in the context's buffer when it can
  // hold them; small ones keep the flush (no second launch).
  if (hard_c10(h.tiles_per_group) && ds.nc >= 2 && ds.nc <= 4) {
    const size_t need =
        (size_t)ds.n_tiles * (size_t)hard_part_row_words(pop.n_sets, h.sets_per_chunk, ds.nc) * 4;
    if (ds.n_tiles * pop.n_sets >= kHardPartMinPairs && need <= kHardPartMaxBytes) {
      aerl_status st = hard_part_buffer(ctx, need, stream, &h.part);
      if (st) return st;
    }
  }
  AERL_HIP(ctx, launch_fill_i32(correct, pop.n_sets, 0, stream));
  if (confusion) AERL_HIP(ctx, launch_fill_i32(confusion, (int64_t)pop.n_sets * ds.nc * ds.nc, 0, stream));
  AERL_HIP(ctx, launch_hard_eval(h, stream));
  if (h.part) {
    AERL_HIP(ctx, launch_hard_reduce(h, ctx->n_cu, stream));
    AERL_HIP(ctx, hipEventRecord(ctx->hard_part_done, stream));
  }
  return AERL_OK;
}

aerl_status aerl_eval_plan(const int64_t *class_count, int32_t n_classes, int32_t n_features,
                           int32_t n_sets, int32_t n_cu, aerl_eval_launch *out) {
  if (!class_count || !out || n_sets < 0 || n_cu < 1) return AERL_EINVAL;
  int64_t n = 0;
  for (int c = 0; c < std::max(n_classes, 0) && c < AERL_MAX_CLASSES; ++c) {
    if (class_count[c] < 0) return AERL_EINVAL;
    n += class_count[c];
    if (n > INT32_MAX) return AERL_EINVAL;
  }
  aerl_status st = check_dataset_args(nullptr, n, n_features, n_classes);
  if (st) return st;
  DatasetRec d;
  d.n = n;
  d.nf = n_features;
  d.nc = n_classes;
  set_regions(d, class_count);
  int S = 0, Q = 0, TG = 0;
  hard_config(d, n_sets, n_cu, &S, &Q, &TG);
  const int64_t blocks = hard_block_count(d, Q, n_sets, TG);
  if (blocks > kMaxHardBlocks) return AERL_EINVAL;
  out->samples_per_lane = S;
  out->sets_per_chunk = Q;
  out->tiles_per_group = TG;
  out->pad = 0;
  out->workgroups = blocks;
  return AERL_OK;
}

aerl_status aerl_eval_population(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id, int32_t *correct,
                                 int32_t *confusion, hipStream_t stream) {
  return eval_common(ctx, dataset_id, pop_id, correct, confusion, 0, 0, 0, stream);
}

aerl_status aerl_eval_population_cfg(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id,
                                     int32_t *correct, int32_t *confusion, int32_t samples_per_lane,
                                     int32_t sets_per_chunk, int32_t tiles_per_group,
                                     hipStream_t stream) {
  if (samples_per_lane == 0) samples_per_lane = -1;  // 0 is reserved for the default choice
  return eval_common(ctx, dataset_id, pop_id, correct, confusion, samples_per_lane, sets_per_chunk,
                     tiles_per_group, stream);
}

aerl_status aerl_predict(aerl_ctx *ctx, int32_t pop_id, int32_t set, const float *rows, int64_t n,
                         int32_t *pred, hipStream_t stream) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->err.clear();
  auto pi = ctx->pops.find(pop_id);
  if (pi == ctx->pops.end()) return fail(ctx, AERL_ENOENT, "unknown population %d", pop_id);
  const PopRec &pop = pi->second;
  if (set < 0 || set >= pop.n_sets) return fail(ctx, AERL_EINVAL, "set %d outside [0, %d)", set, pop.n_sets);
  if (n < 0 || n > INT32_MAX) return fail(ctx, AERL_EINVAL, "n = %lld outside [0, 2^31)", (long long)n);
  if (n > 0 && (!rows || !pred)) return fail(ctx, AERL_EINVAL, "rows or pred is NULL");
  AERL_HIP(ctx, hipSetDevice(ctx->device));
  AERL_HIP(ctx, launch_predict(pop, set, rows, n, pred, stream));
  return AERL_OK;
}

aerl_status aerl_soft_workspace_bytes(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id,
                                      size_t *forward_bytes, size_t *backward_bytes) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  auto di = ctx->datasets.find(dataset_id);
  if (di == ctx->datasets.end()) return fail(ctx, AERL_ENOENT, "unknown dataset %d", dataset_id);
  auto pi = ctx->pops.find(pop_id);
  if (pi == ctx->pops.end()) return fail(ctx, AERL_ENOENT, "unknown population %d", pop_id);
  if (forward_bytes) *forward_bytes = soft_ws_bytes(di->second, pi->second, false);
  if (backward_bytes) *backward_bytes = soft_ws_bytes(di->second, pi->second, true);
  return AERL_OK;
}

static aerl_status soft_common(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id, SoftLaunch *l,
                               bool backward, bool first_firing = true) {
  auto di = ctx->datasets.find(dataset_id);
  if (di == ctx->datasets.end()) return fail(ctx, AERL_ENOENT, "unknown dataset %d", dataset_id);
  auto pi = ctx->pops.find(pop_id);
  if (pi == ctx->pops.end()) return fail(ctx, AERL_ENOENT, "unknown population %d", pop_id);
  const DatasetRec &ds = di->second;
  const PopRec &pop = pi->second;
  if (pop.nf != ds.nf || pop.nc != ds.nc)
    return fail(ctx, AERL_EINVAL, "population and dataset shapes differ");
  if (pop.n_conds > 0 && (!l->coef || !l->coef2 || !l->theta))
    return fail(ctx, AERL_EINVAL, "a parameter array is NULL");
  if ((int64_t)pop.n_sets > kMaxHardBlocks)
    return fail(ctx, AERL_EINVAL, "%d rule sets exceed the soft kernels' launch limit %lld", pop.n_sets,
                (long long)kMaxHardBlocks);
  if (backward && first_firing && !soft_backward_supported(ds, pop))
    return fail(ctx, AERL_EINVAL, "rule sets of %d rules exceed the adjoint kernel's LDS", pop.max_rules);
  const size_t need = soft_ws_bytes(ds, pop, backward);
  if (need && (!l->ws || ((uintptr_t)l->ws & 255)))
    return fail(ctx, AERL_EINVAL, "ws is NULL or not 256-byte aligned");
  if (l->ws_bytes < need) return fail(ctx, AERL_ENOMEM, "ws holds %zu bytes, %zu needed", l->ws_bytes, need);
  l->ds = &ds;
  l->pop = &pop;
  return AERL_OK;
}

aerl_status aerl_soft_forward(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id, const float *coef,
                              const float *coef2, const float *theta, float *loss, void *ws,
                              size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->err.clear();
  SoftLaunch l{};
  l.coef = coef; l.coef2 = coef2; l.theta = theta; l.loss = loss; l.ws = ws; l.ws_bytes = ws_bytes;
  aerl_status st = soft_common(ctx, dataset_id, pop_id, &l, false);
  if (st) return st;
  if (!loss && l.pop->n_sets > 0) return fail(ctx, AERL_EINVAL, "loss is NULL");
  AERL_HIP(ctx, hipSetDevice(ctx->device));
  AERL_HIP(ctx, launch_soft_forward(l, stream));
  return AERL_OK;
}

static aerl_status smax_common(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id, SoftLaunch *l,
                               bool backward, float beta) {
  if (!(beta >= 0.0f) || !std::isfinite(beta)) return fail(ctx, AERL_EINVAL, "beta must be finite and >= 0");
  auto di = ctx->datasets.find(dataset_id);
  auto pi = ctx->pops.find(pop_id);
  if (di != ctx->datasets.end() && pi != ctx->pops.end()) {
    if (di->second.nc > kSmaxMaxClasses)
      return fail(ctx, AERL_EINVAL, "the softmax head takes at most %d classes", kSmaxMaxClasses);
    if (!smax_supported(di->second, pi->second))
      return fail(ctx, AERL_EINVAL, "rule sets of %d rules exceed the softmax kernel's LDS",
                  pi->second.max_rules);
  }
  return soft_common(ctx, dataset_id, pop_id, l, backward, false);
}

aerl_status aerl_softmax_forward(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id,
                                 const float *coef, const float *coef2, const float *theta,
                                 float beta, float *loss, void *ws, size_t ws_bytes,
                                 hipStream_t stream) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->err.clear();
  SoftLaunch l{};
  l.coef = coef; l.coef2 = coef2; l.theta = theta; l.loss = loss; l.ws = ws; l.ws_bytes = ws_bytes;
  aerl_status st = smax_common(ctx, dataset_id, pop_id, &l, false, beta);
  if (st) return st;
  if (!loss && l.pop->n_sets > 0) return fail(ctx, AERL_EINVAL, "loss is NULL");
  AERL_HIP(ctx, hipSetDevice(ctx->device));
  AERL_HIP(ctx, launch_smax_forward(l, beta, stream));
  return AERL_OK;
}

aerl_status aerl_softmax_backward(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id,
                                  const float *coef, const float *coef2, const float *theta,
                                  float beta, const float *dloss, float *dcoef, float *dcoef2,
                                  float *dtheta, void *ws, size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->err.clear();
  SoftLaunch l{};
  l.coef = coef; l.coef2 = coef2; l.theta = theta; l.dloss = dloss;
  l.dcoef = dcoef; l.dcoef2 = dcoef2; l.dtheta = dtheta; l.ws = ws; l.ws_bytes = ws_bytes;
  aerl_status st = smax_common(ctx, dataset_id, pop_id, &l, true, beta);
  if (st) return st;
  if (l.pop->n_conds > 0 && (!dcoef || !dcoef2 || !dtheta))
    return fail(ctx, AERL_EINVAL, "a gradient array is NULL");
  if (l.pop->n_sets > 0 && !dloss) return fail(ctx, AERL_EINVAL, "dloss is NULL");
  AERL_HIP(ctx, hipSetDevice(ctx->device));
  AERL_HIP(ctx, launch_smax_backward(l, beta, stream));
  return AERL_OK;
}

aerl_status aerl_softmax_proba(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id, int32_t set,
                               const float *coef, const float *coef2, const float *theta,
                               float beta, const float *rows, int64_t n, float *probs, void *ws,
                               size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->err.clear();
  SoftLaunch l{};
  l.coef = coef; l.coef2 = coef2; l.theta = theta; l.ws = ws; l.ws_bytes = ws_bytes;
  aerl_status st = smax_common(ctx, dataset_id, pop_id, &l, false, beta);
  if (st) return st;
  if (set < 0 || set >= l.pop->n_sets) return fail(ctx, AERL_EINVAL, "set %d outside [0, %d)", set, l.pop->n_sets);
  if (n < 0 || n > INT32_MAX) return fail(ctx, AERL_EINVAL, "n = %lld outside [0, 2^31)", (long long)n);
  if (n > 0 && (!rows || !probs)) return fail(ctx, AERL_EINVAL, "rows or probs is NULL");
  AERL_HIP(ctx, hipSetDevice(ctx->device));
  AERL_HIP(ctx, launch_smax_proba(l, set, beta, rows, n, probs, stream));
  return AERL_OK;
}

aerl_status aerl_finetune_workspace_bytes(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id,
                                          size_t *bytes) {
  if (!ctx || !bytes) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  auto di = ctx->datasets.find(dataset_id);
  if (di == ctx->datasets.end()) return fail(ctx, AERL_ENOENT, "unknown dataset %d", dataset_id);
  auto pi = ctx->pops.find(pop_id);
  if (pi == ctx->pops.end()) return fail(ctx, AERL_ENOENT, "unknown population %d", pop_id);
  *bytes = tune_layout(di->second, pi->second).total;
  return AERL_OK;
}

aerl_status aerl_finetune(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id,
                          const aerl_finetune_cfg *cfg, float *coef, float *coef2, float *theta,
                          float *loss_hist, void *ws, size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->err.clear();
  if (!cfg) return fail(ctx, AERL_EINVAL, "cfg is NULL");
  if (cfg->epochs < 0) return fail(ctx, AERL_EINVAL, "epochs %d < 0", cfg->epochs);
  if (!(cfg->lr > 0.0f) || !std::isfinite(cfg->lr)) return fail(ctx, AERL_EINVAL, "lr must be positive");
  if (cfg->optimizer == AERL_OPT_ADAM) {
    if (!(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) || !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) ||
        !(cfg->eps > 0.0f) || !std::isfinite(cfg->eps))
      return fail(ctx, AERL_EINVAL, "Adam needs beta1, beta2 in [0, 1) and eps > 0");
  } else if (cfg->optimizer != AERL_OPT_SGD) {
    return fail(ctx, AERL_EINVAL, "unknown optimizer %d", cfg->optimizer);
  }
  SoftLaunch l{};
  l.coef = coef; l.coef2 = coef2; l.theta = theta;
  l.ws = ws; l.ws_bytes = ws_bytes;
  aerl_status st = soft_common(ctx, dataset_id, pop_id, &l, true);
  if (st) return st;
  const TuneLayout L = tune_layout(*l.ds, *l.pop);
  if (ws_bytes < L.total) return fail(ctx, AERL_ENOMEM, "ws holds %zu bytes, %zu needed", ws_bytes, L.total);
  TuneLaunch t{};
  t.ds = l.ds;
  t.pop = l.pop;
  t.coef = coef; t.coef2 = coef2; t.theta = theta;
  t.loss_hist = loss_hist;
  t.epochs = cfg->epochs;
  t.optimizer = cfg->optimizer;
  t.lr = cfg->lr; t.beta1 = cfg->beta1; t.beta2 = cfg->beta2; t.eps = cfg->eps;
  t.ws = ws;
  AERL_HIP(ctx, hipSetDevice(ctx->device));
  AERL_HIP(ctx, run_finetune(t, stream));
  return AERL_OK;
}

aerl_status aerl_soft_forward_noalloc(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id,
                                      const float *coef, const float *coef2, const float *theta,
                                      float *loss, hipStream_t stream) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->err.clear();
  if (!ctx->noalloc_scratch) return fail(ctx, AERL_EDEVICE, "no scratch array on device %d", ctx->device);
  auto di = ctx->datasets.find(dataset_id);
  auto pi = ctx->pops.find(pop_id);
  if (di != ctx->datasets.end() && pi != ctx->pops.end()) {
    const size_t need = soft_ws_bytes(di->second, pi->second, false);
    if (need > AERL_NOALLOC_SCRATCH_BYTES)
      return fail(ctx, AERL_ENOMEM,
                  "the no-allocation soft forward needs %zu bytes of scratch; it holds %zu", need,
                  (size_t)AERL_NOALLOC_SCRATCH_BYTES);
  }
  SoftLaunch l{};
  l.coef = coef; l.coef2 = coef2; l.theta = theta; l.loss = loss;
  l.ws = ctx->noalloc_scratch;
  l.ws_bytes = AERL_NOALLOC_SCRATCH_BYTES;
  aerl_status st = soft_common(ctx, dataset_id, pop_id, &l, false);
  if (st) return st;
  if (!loss && l.pop->n_sets > 0) return fail(ctx, AERL_EINVAL, "loss is NULL");
  AERL_HIP(ctx, hipSetDevice(ctx->device));
  AERL_HIP(ctx, launch_soft_forward(l, stream));
  return AERL_OK;
}

aerl_status aerl_soft_backward(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id, const float *coef,
                               const float *coef2, const float *theta, const float *dloss,
                               float *dcoef, float *dcoef2, float *dtheta, void *ws, size_t ws_bytes,
                               hipStream_t stream) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->err.clear();
  SoftLaunch l{};
  l.coef = coef; l.coef2 = coef2; l.theta = theta; l.dloss = dloss;
  l.dcoef = dcoef; l.dcoef2 = dcoef2; l.dtheta = dtheta; l.ws = ws; l.ws_bytes = ws_bytes;
  aerl_status st = soft_common(ctx, dataset_id, pop_id, &l, true);
  if (st) return st;
  if (l.pop->n_conds > 0 && (!dcoef || !dcoef2 || !dtheta))
    return fail(ctx, AERL_EINVAL, "a gradient array is NULL");
  if (l.pop->n_sets > 0 && !dloss) return fail(ctx, AERL_EINVAL, "dloss is NULL");
  AERL_HIP(ctx, hipSetDevice(ctx->device));
  AERL_HIP(ctx, launch_soft_backward(l, stream));
  return AERL_OK;
}

}  // extern "C"
