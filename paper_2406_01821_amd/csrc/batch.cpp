// Ragged batch planning, hipGraph capture and the autotuner (host side).
//
// A plan turns a list of (dataset, population) evaluations into one work
// list: work item = (item, chunk of rule sets, group of label-uniform tiles).
// Items are cut with the same (rule sets, tiles) per work item; each item
// picks its own tile width from its feature count.  Work items are sorted by
// estimated cost (samples x nominal conditions), largest first, so that the
// persistent grid's dynamic pull ends evenly.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

#include "batch.h"

namespace aerl {

struct BatchPlanRec {
  BatchLaunch launch{};
  void *ws = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture = nullptr;
  std::vector<int32_t> dataset_ids, pop_ids;
};

void destroy_plan(BatchPlanRec *p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->capture) (void)hipStreamDestroy(p->capture);
  delete p;
}

int batch_samples_per_lane(int32_t nf, size_t tile_budget) {
  int s = 4;
  while (s > 1 && (size_t)nf * 256 * s > tile_budget) s >>= 1;
  return s;
}

namespace {
size_t align256_(size_t v) { return (v + 255) & ~size_t(255); }
}  // namespace

namespace {
int32_t sets_per_item(const DatasetRec &ds, int32_t n_sets, const BatchSplit &sp) {
  const int32_t Q = sp.Q;
  const size_t tile_bytes = (size_t)ds.nf * 64 * batch_samples_per_lane(ds.nf, sp.tile_budget) * 4;
  const int32_t q_fit =
      (int32_t)std::min<size_t>((kBatchLdsMax - tile_bytes - (size_t)ds.nf * 8 - 4) /
                                    ((size_t)std::max(hard_counters_per_set(ds.nc), 1) * 2),
                                1 << 20);
  return std::max(1, std::min({Q, n_sets, q_fit}));
}
}  // namespace

int64_t batch_task_count(const DatasetRec &ds, int32_t n_sets, const BatchSplit &sp) {
  if (n_sets <= 0) return 0;
  const int32_t q = sets_per_item(ds, n_sets, sp);
  const int32_t TG = sp.TG;
  int64_t groups = 0;
  for (int c = 0; c < ds.nc; ++c) groups += (ds.region_tiles[c] + TG - 1) / TG;
  return (int64_t)((n_sets + q - 1) / q) * groups;
}

void build_batch_tables(const std::vector<BatchSource> &src, const BatchSplit &sp, BatchTables *b) {
  const int32_t TG = sp.TG;
  b->items.clear();
  b->tasks.clear();
  b->zero.clear();
  b->lds = 0;
  b->cat = false;
  std::vector<std::pair<double, BatchTask>> costed;
  for (size_t i = 0; i < src.size(); ++i) {
    const DatasetRec &ds = *src[i].ds;
    const int32_t n_sets = src[i].n_sets;
    const int S = batch_samples_per_lane(ds.nf, sp.tile_budget);
    BatchItem it{};
    it.x_fm = ds.x_fm;
    it.n_pad = ds.n_pad;
    it.tile_info = ds.tile_info;
    it.sets = src[i].sets;
    it.conds = src[i].conds;
    it.heads = src[i].heads;
    it.correct = src[i].correct;
    it.confusion = src[i].confusion;
    it.nf = ds.nf;
    it.nc = ds.nc;
    it.S = S;
    b->items.push_back(it);
    if (n_sets <= 0) continue;
    b->cat = b->cat || src[i].cat;
    b->zero.push_back({it.correct, n_sets});
    if (it.confusion) b->zero.push_back({it.confusion, (int64_t)n_sets * ds.nc * ds.nc});
    const size_t tile_bytes = (size_t)ds.nf * 64 * S * 4;
    const int32_t q = sets_per_item(ds, n_sets, sp);
    b->lds = std::max(b->lds, hard_block_lds(ds.nf, S, q, ds.nc));
    const int4 *hs = src[i].host_sets;
    for (int32_t q0 = 0; q0 < n_sets; q0 += q) {
      const int32_t qe = std::min(q, n_sets - q0);
      double work = 0;
      for (int32_t k = q0; k < q0 + qe; ++k) work += (double)hs[k].w + 1.0;
      for (int c = 0; c < ds.nc; ++c) {
        for (int32_t t0 = 0; t0 < ds.region_tiles[c]; t0 += TG) {
          BatchTask tk{};
          tk.item = (int32_t)i;
          tk.q0 = q0;
          tk.Q = qe;
          tk.tile_lo = ds.region_tile0[c] + t0;
          tk.tile_hi = ds.region_tile0[c] + std::min(t0 + TG, ds.region_tiles[c]);
          tk.label = c;
          costed.push_back({work * (double)(tk.tile_hi - tk.tile_lo), tk});
        }
      }
    }
  }
  std::stable_sort(costed.begin(), costed.end(),
                   [](const auto &x, const auto &y) { return x.first > y.first; });
  for (auto &c : costed) b->tasks.push_back(c.second);
  size_t off = 0;
  b->items_off = off;   off = align256_(off + sizeof(BatchItem) * std::max<size_t>(b->items.size(), 1));
  b->tasks_off = off;   off = align256_(off + sizeof(BatchTask) * std::max<size_t>(b->tasks.size(), 1));
  b->zero_off = off;    off = align256_(off + sizeof(BatchZero) * std::max<size_t>(b->zero.size(), 1));
  b->counter_off = off; off = align256_(off + sizeof(int32_t));
  b->bytes = off;
}

void emit_batch_tables(const BatchTables &b, void *img, char *dev, int n_cu, BatchLaunch *bl) {
  char *h = static_cast<char *>(img);
  std::memset(h, 0, b.bytes);
  std::memcpy(h + b.items_off, b.items.data(), sizeof(BatchItem) * b.items.size());
  std::memcpy(h + b.tasks_off, b.tasks.data(), sizeof(BatchTask) * b.tasks.size());
  std::memcpy(h + b.zero_off, b.zero.data(), sizeof(BatchZero) * b.zero.size());
  bl->items = reinterpret_cast<const BatchItem *>(dev + b.items_off);
  bl->tasks = reinterpret_cast<const BatchTask *>(dev + b.tasks_off);
  bl->zero = reinterpret_cast<const BatchZero *>(dev + b.zero_off);
  bl->counter = reinterpret_cast<int32_t *>(dev + b.counter_off);
  bl->n_tasks = (int32_t)b.tasks.size();
  bl->n_zero = (int32_t)b.zero.size();
  bl->lds = b.lds;
  bl->cat = b.cat;
  const int per_cu = 2 * (b.lds + kStaticLds) <= kLdsPerCu ? 2 : 1;
  bl->grid = std::max<int64_t>(1, std::min<int64_t>((int64_t)n_cu * per_cu, (int64_t)b.tasks.size()));
}

int predict_samples_per_lane(int32_t nf) { return (size_t)nf * 256 * 4 <= kDynLdsMax ? 4 : 1; }

namespace {

struct ItemView {
  const DatasetRec *ds;
  const PopRec *pop;
  const aerl_batch_item *item;
};

aerl_status gather(aerl_ctx *ctx, const aerl_batch_item *items, int32_t n, std::vector<ItemView> *out) {
  if (n < 0 || (n > 0 && !items)) return fail(ctx, AERL_EINVAL, "bad item list");
  out->clear();
  for (int32_t i = 0; i < n; ++i) {
    auto di = ctx->datasets.find(items[i].dataset_id);
    if (di == ctx->datasets.end()) return fail(ctx, AERL_ENOENT, "item %d: unknown dataset %d", i, items[i].dataset_id);
    auto pi = ctx->pops.find(items[i].pop_id);
    if (pi == ctx->pops.end()) return fail(ctx, AERL_ENOENT, "item %d: unknown population %d", i, items[i].pop_id);
    if (pi->second.nf != di->second.nf || pi->second.nc != di->second.nc)
      return fail(ctx, AERL_EINVAL, "item %d: population and dataset shapes differ", i);
    if (pi->second.n_sets > 0 && !items[i].correct)
      return fail(ctx, AERL_EINVAL, "item %d: correct is NULL", i);
    if (hard_block_lds(di->second.nf, 1, 1, di->second.nc) > kBatchLdsMax)
      return fail(ctx, AERL_EINVAL, "item %d: %d features exceed the LDS tile", i, di->second.nf);
    out->push_back({&di->second, &pi->second, &items[i]});
  }
  return AERL_OK;
}

std::vector<BatchSource> sources(const std::vector<ItemView> &v) {
  std::vector<BatchSource> src;
  for (const auto &it : v) {
    // The set records lead the population's host staging copy of its image.
    src.push_back({it.ds, it.pop->n_sets, static_cast<const int4 *>(it.pop->staging),
                   it.pop->sets, it.pop->hconds, it.pop->heads, it.item->correct,
                   it.item->confusion, it.pop->n_cat > 0});
  }
  return src;
}

int log2_bucket(double v) { return v <= 1 ? 0 : (int)std::ceil(std::log2(v)); }

std::string shape_key(const std::vector<ItemView> &v) {
  std::ostringstream k;
  k << "n" << v.size();
  for (const auto &it : v) {
    const double conds = it.pop->n_sets > 0 ? (double)it.pop->nominal_conds / it.pop->n_sets : 0;
    k << "|" << log2_bucket(it.ds->nf) << "," << log2_bucket((double)it.ds->n_tiles) << ","
      << log2_bucket(it.pop->n_sets) << "," << log2_bucket(conds);
  }
  return k.str();
}

void load_tune_file(aerl_ctx *ctx) {
  if (ctx->tune_file_loaded) return;
  ctx->tune_file_loaded = true;
  const char *path = std::getenv("AERL_AUTOTUNE_CACHE");
  if (!path) return;
  std::ifstream in(path);
  std::string key;
  int32_t q, tg, kib;
  double ms;
  while (in >> key >> q >> tg >> kib >> ms) ctx->tuned[key] = {q, tg, kib};
}

// The caller's split, with zero fields taken from the tuned table for this
// batch shape or the defaults.
aerl_status resolve_split(aerl_ctx *ctx, const std::vector<ItemView> &v, const aerl_batch_cfg *cfg,
                          BatchSplit *sp) {
  std::array<int32_t, 3> d = {512, 1, 64};
  load_tune_file(ctx);
  auto it = ctx->tuned.find(shape_key(v));
  if (it != ctx->tuned.end()) d = it->second;
  const int32_t q = cfg && cfg->sets_per_task > 0 ? cfg->sets_per_task : d[0];
  const int32_t tg = cfg && cfg->tiles_per_task > 0 ? cfg->tiles_per_task : d[1];
  const int32_t kib = cfg && cfg->tile_kib > 0 ? cfg->tile_kib : d[2];
  if ((cfg && (cfg->sets_per_task < 0 || cfg->tiles_per_task < 0 || cfg->tile_kib < 0)) ||
      kib > (int32_t)(kBatchLdsMax / 1024) || tg > kMaxTilesPerBlock)
    return fail(ctx, AERL_EINVAL, "invalid work split (%d, %d, %d)", q, tg, kib);
  sp->Q = q;
  sp->TG = tg;
  sp->tile_budget = (size_t)kib * 1024;
  // work items are counted and indexed with int32 on the device
  int64_t tasks = 0;
  for (const auto &e : v) tasks += batch_task_count(*e.ds, e.pop->n_sets, *sp);
  if (tasks > INT32_MAX)
    return fail(ctx, AERL_EINVAL, "%lld work items exceed 2^31 - 1; raise tiles_per_task", (long long)tasks);
  return AERL_OK;
}

aerl_status upload_plan(aerl_ctx *ctx, const BatchTables &b, void *ws, size_t ws_bytes, hipStream_t st,
                        BatchPlanRec *plan) {
  if (!ws || ((uintptr_t)ws & 255)) return fail(ctx, AERL_EINVAL, "ws is NULL or not 256-byte aligned");
  if (ws_bytes < b.bytes) return fail(ctx, AERL_ENOMEM, "ws holds %zu bytes, %zu needed", ws_bytes, b.bytes);
  if (b.lds > kBatchLdsMax) return fail(ctx, AERL_EINVAL, "work split needs %zu bytes of LDS", b.lds);
  void *pinned = nullptr;
  AERL_HIP(ctx, hipHostMalloc(&pinned, b.bytes, hipHostMallocDefault));
  emit_batch_tables(b, pinned, static_cast<char *>(ws), ctx->n_cu, &plan->launch);
  hipError_t e = hipMemcpyAsync(ws, pinned, b.bytes, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipHostFree(pinned);
  if (e != hipSuccess) return fail(ctx, AERL_EDEVICE, "plan upload failed: %s", hipGetErrorString(e));
  plan->ws = ws;
  return AERL_OK;
}

}  // namespace
}  // namespace aerl

using namespace aerl;

extern "C" {

aerl_status aerl_batch_workspace_bytes(aerl_ctx *ctx, const aerl_batch_item *items, int32_t n_items,
                                       const aerl_batch_cfg *cfg, size_t *bytes) {
  if (!ctx || !bytes) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  std::vector<ItemView> v;
  aerl_status st = gather(ctx, items, n_items, &v);
  if (st) return st;
  BatchSplit sp;
  st = resolve_split(ctx, v, cfg, &sp);
  if (st) return st;
  BatchTables b;
  build_batch_tables(sources(v), sp, &b);
  *bytes = b.bytes;
  return AERL_OK;
}

aerl_status aerl_batch_plan(aerl_ctx *ctx, const aerl_batch_item *items, int32_t n_items,
                            const aerl_batch_cfg *cfg, void *ws, size_t ws_bytes, uint32_t flags,
                            hipStream_t stream, int32_t *plan_id) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->err.clear();
  if (!plan_id) return fail(ctx, AERL_EINVAL, "plan_id is NULL");
  std::vector<ItemView> v;
  aerl_status st = gather(ctx, items, n_items, &v);
  if (st) return st;
  BatchSplit sp;
  st = resolve_split(ctx, v, cfg, &sp);
  if (st) return st;
  AERL_HIP(ctx, hipSetDevice(ctx->device));
  BatchTables b;
  build_batch_tables(sources(v), sp, &b);
  std::unique_ptr<BatchPlanRec, PlanDeleter> plan(new BatchPlanRec());
  st = upload_plan(ctx, b, ws, ws_bytes, stream, plan.get());
  if (st) return st;
  for (const auto &it : v) {
    plan->dataset_ids.push_back(it.item->dataset_id);
    plan->pop_ids.push_back(it.item->pop_id);
  }
  if (flags & AERL_BATCH_GRAPH) {
    // Captured on a private stream (the caller's may be the legacy default
    // stream, which cannot be captured) and replayed on the caller's stream.
    AERL_HIP(ctx, hipStreamCreateWithFlags(&plan->capture, hipStreamNonBlocking));
    AERL_HIP(ctx, hipStreamBeginCapture(plan->capture, hipStreamCaptureModeThreadLocal));
    hipError_t e = launch_batch(plan->launch, plan->capture);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(plan->capture, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(ctx, AERL_EDEVICE, "graph capture failed: %s",
                  hipGetErrorString(e != hipSuccess ? e : e2));
    }
    plan->graph = g;
    AERL_HIP(ctx, hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0));
  }
  const int32_t id = ctx->next_id++;
  ctx->plans[id] = std::move(plan);
  *plan_id = id;
  return AERL_OK;
}

aerl_status aerl_batch_run(aerl_ctx *ctx, int32_t plan_id, hipStream_t stream) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->err.clear();
  auto it = ctx->plans.find(plan_id);
  if (it == ctx->plans.end()) return fail(ctx, AERL_ENOENT, "unknown plan %d", plan_id);
  for (size_t i = 0; i < it->second->dataset_ids.size(); ++i) {
    if (!ctx->datasets.count(it->second->dataset_ids[i]) || !ctx->pops.count(it->second->pop_ids[i]))
      return fail(ctx, AERL_ENOENT, "plan %d refers to a released dataset or population", plan_id);
  }
  AERL_HIP(ctx, hipSetDevice(ctx->device));
  if (it->second->exec) {
    AERL_HIP(ctx, hipGraphLaunch(it->second->exec, stream));
  } else {
    AERL_HIP(ctx, launch_batch(it->second->launch, stream));
  }
  return AERL_OK;
}

aerl_status aerl_batch_release(aerl_ctx *ctx, int32_t plan_id) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (!ctx->plans.erase(plan_id)) return fail(ctx, AERL_ENOENT, "unknown plan %d", plan_id);
  return AERL_OK;
}

aerl_status aerl_autotune(aerl_ctx *ctx, const aerl_batch_item *items, int32_t n_items, void *ws,
                          size_t ws_bytes, hipStream_t stream, aerl_batch_cfg *best,
                          float *best_ms) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->err.clear();
  if (!best) return fail(ctx, AERL_EINVAL, "best is NULL");
  std::vector<ItemView> v;
  aerl_status st = gather(ctx, items, n_items, &v);
  if (st) return st;
  AERL_HIP(ctx, hipSetDevice(ctx->device));
  static const int32_t kQ[] = {64, 128, 256, 512, 1024, 2048};
  static const int32_t kTG[] = {1, 2, 4, 8};
  static const int32_t kKiB[] = {64, 128};
  hipEvent_t e0, e1;
  AERL_HIP(ctx, hipEventCreate(&e0));
  AERL_HIP(ctx, hipEventCreate(&e1));
  float best_t = 1e30f;
  BatchSplit best_sp;
  for (int32_t kib : kKiB) {
    for (int32_t q : kQ) {
      for (int32_t tg : kTG) {
        BatchSplit sp;
        sp.Q = q;
        sp.TG = tg;
        sp.tile_budget = (size_t)kib * 1024;
        int64_t tasks = 0;
        for (const auto &e : v) tasks += batch_task_count(*e.ds, e.pop->n_sets, sp);
        if (tasks > INT32_MAX) continue;
        BatchTables b;
        build_batch_tables(sources(v), sp, &b);
        if (b.lds > kBatchLdsMax) continue;
        BatchPlanRec tmp;
        if (upload_plan(ctx, b, ws, ws_bytes, stream, &tmp) != AERL_OK) continue;
        hipError_t e = launch_batch(tmp.launch, stream);  // warm-up
        float t = 0.0f;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
          if (e == hipSuccess) e = hipEventRecord(e0, stream);
          if (e == hipSuccess) e = launch_batch(tmp.launch, stream);
          if (e == hipSuccess) e = hipEventRecord(e1, stream);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float ms = 0.0f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          t += ms;
        }
        if (e != hipSuccess) {
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
          return fail(ctx, AERL_EDEVICE, "autotune launch failed: %s", hipGetErrorString(e));
        }
        t *= 0.5f;
        if (t < best_t) {
          best_t = t;
          best_sp = sp;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best_t >= 1e30f) return fail(ctx, AERL_ENOMEM, "no candidate split fits ws (%zu bytes)", ws_bytes);
  const int32_t bkib = (int32_t)(best_sp.tile_budget / 1024);
  const std::string key = shape_key(v);
  ctx->tuned[key] = {best_sp.Q, best_sp.TG, bkib};
  if (const char *path = std::getenv("AERL_AUTOTUNE_CACHE")) {
    std::ofstream out(path, std::ios::app);
    out << key << " " << best_sp.Q << " " << best_sp.TG << " " << bkib << " " << best_t << "\n";
  }
  best->sets_per_task = best_sp.Q;
  best->tiles_per_task = best_sp.TG;
  best->tile_kib = bkib;
  if (best_ms) *best_ms = best_t;
  return AERL_OK;
}

}  // extern "C"
