// Serving loop: continuous batching of fitness and prediction requests.
//
// Submitting threads validate and pack a request on the host and queue it.
// One scheduler thread admits queued requests in arrival order while their
// device footprint fits in one free range of the caller's arena, and puts
// every request it can admit into the next launch on a free stream slot:
// one H2D copy (packed populations, prediction rows, work tables), the
// persistent fitness kernel, the batched prediction kernel, one D2H copy of
// the outputs and an event.  While launches run, newly arriving requests
// queue up and leave in the next launch as soon as a slot and arena space
// are free, so batch sizes follow the load.  Completed launches are reaped
// by polling their events; outputs are copied to the callers' buffers and
// the arena range is returned.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <thread>

#include "batch.h"
#include "serve_sched.h"

namespace aerl {

using Clock = std::chrono::steady_clock;

namespace {

const BatchSplit kServeSplit{512, 2, 64 * 1024};  // rule sets, tiles per work item; tile LDS
constexpr size_t kTableSlack = 16 * 256;  // alignment padding of the per-launch tables
constexpr size_t kInitialPinned = 16u << 20;

size_t al(size_t v) { return (v + 255) & ~size_t(255); }

double us_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::micro>(b - a).count();
}

struct Req {
  uint64_t ticket = 0;
  int32_t kind = 0;
  int32_t dataset_id = -1;
  DatasetRec dsv;                       // copy of the dataset's record
  const DatasetRec *ds = nullptr;       // &dsv for fitness requests
  const DatasetRec *ds_reg = nullptr;   // the registry entry it was copied from
  std::vector<char> image;  // packed population (host)
  PackedLayout L{};
  PopRec rec{};
  int32_t nf = 0, nc = 0, set_index = 0;
  std::vector<float> rows;
  int64_t n_rows = 0;
  int32_t *h_correct = nullptr, *h_conf = nullptr, *h_pred = nullptr;
  size_t in_bytes = 0, out_bytes = 0, table_bytes = 0;
  size_t in_off = 0, rows_off = 0, out_off = 0;  // inside the launch's range
  double nominal = 0;
  Clock::time_point t_submit, t_queued, t_launch, t_seen_done, t_done;
  aerl_status status = AERL_OK;
  int32_t batch_size = 0;
  bool done = false;

  size_t dev_bytes() const { return in_bytes + out_bytes + table_bytes; }
  size_t correct_bytes() const { return (size_t)rec.n_sets * 4; }
  size_t conf_bytes() const { return h_conf ? (size_t)rec.n_sets * nc * nc * 4 : 0; }
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  // with a trace: timing events before the upload, after it, after the
  // kernels and after the download
  hipEvent_t span[4] = {nullptr, nullptr, nullptr, nullptr};
  int index = 0;
  void *h_in = nullptr, *h_out = nullptr;
  size_t in_cap = 0, out_cap = 0;
  bool busy = false;
  std::vector<Req *> reqs;
  size_t off = 0, bytes = 0, out_bytes = 0;
};

hipError_t ensure_pinned(void **p, size_t *cap, size_t need) {
  if (*cap >= need) return hipSuccess;
  const size_t n = std::max(need, std::max(kInitialPinned, 2 * *cap));
  if (*p) (void)hipHostFree(*p);
  *p = nullptr;
  *cap = 0;
  hipError_t e = hipHostMalloc(p, n, hipHostMallocDefault);
  if (e == hipSuccess) *cap = n;
  return e;
}

}  // namespace

struct Serve {
  aerl_ctx *ctx = nullptr;
  char *arena = nullptr;
  size_t arena_bytes = 0;
  int32_t max_batch = 256, max_inflight = 4;
  int device = 0, n_cu = 0;

  std::mutex m;
  std::condition_variable cv_work, cv_done;
  std::thread thr;
  bool running = false, stopping = false;
  std::deque<Req *> pending;
  std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
  std::unordered_map<int32_t, int32_t> ds_refs;
  uint64_t next_ticket = 1;
  ArenaAlloc alloc;
  std::vector<Slot> slots;

  // AERL_TRACE span log (JSON lines, one per completed request), or null
  FILE *trace = nullptr;
  Clock::time_point t_start;

  // statistics since start or the last reset
  std::vector<double> lat_us;
  int64_t submitted = 0, completed = 0, launches = 0, launched_reqs = 0;
  double nominal_done = 0;
  bool have_first = false;
  Clock::time_point t_first, t_last;
  size_t arena_peak = 0;

  void run();
  bool launch_one(std::unique_lock<std::mutex> &lk, Slot &slot);
  void reap(std::unique_lock<std::mutex> &lk, Slot &slot, hipError_t status);
  void write_trace(const Slot &slot, const std::vector<Req *> &rs, hipError_t status);
};

// Takes a FIFO prefix of the pending requests that fits in the largest free
// arena range, lays it out and enqueues its copies and kernels on the slot.
bool Serve::launch_one(std::unique_lock<std::mutex> &lk, Slot &slot) {
  size_t need = 0;
  const int32_t n_take = admit_prefix(
      pending,
      [](const Req *r) { return QueuedSize{r->dev_bytes(), r->in_bytes + r->table_bytes, r->out_bytes}; },
      alloc.largest(), max_batch, kTableSlack, slot.in_cap, slot.out_cap, &need);
  if (n_take == 0) return false;
  std::vector<Req *> take(pending.begin(), pending.begin() + n_take);
  pending.erase(pending.begin(), pending.begin() + n_take);
  size_t off = 0;
  alloc.alloc(need, &off);  // cannot fail: need <= the largest free range
  arena_peak = std::max(arena_peak, alloc.used());
  const Clock::time_point now = Clock::now();
  for (Req *r : take) {
    r->t_launch = now;
    r->batch_size = (int32_t)take.size();
  }
  slot.busy = true;
  slot.reqs = take;
  slot.off = off;
  slot.bytes = need;
  ++launches;
  launched_reqs += (int64_t)take.size();
  lk.unlock();

  // Range layout: [outputs][inputs][fitness tables][prediction tasks].
  char *dev = arena + off;
  size_t cur = 0;
  for (Req *r : take) {
    r->out_off = cur;
    cur += r->out_bytes;
  }
  const size_t out_end = cur;
  for (Req *r : take) {
    r->in_off = cur;
    r->rows_off = cur + al(r->L.total);
    cur += r->in_bytes;
  }
  std::vector<BatchSource> src;
  std::vector<PredictTask> ptasks;
  size_t plds = 0;
  for (Req *r : take) {
    const int4 *dsets = reinterpret_cast<const int4 *>(dev + r->in_off + r->L.sets_off);
    const uint4 *dconds = reinterpret_cast<const uint4 *>(dev + r->in_off + r->L.hconds_off);
    const uint4 *dheads = reinterpret_cast<const uint4 *>(dev + r->in_off + r->L.heads_off);
    if (r->kind == AERL_REQ_FITNESS) {
      int32_t *c = reinterpret_cast<int32_t *>(dev + r->out_off);
      int32_t *cf = r->h_conf ? reinterpret_cast<int32_t *>(dev + r->out_off + al(r->correct_bytes()))
                              : nullptr;
      src.push_back({r->ds, r->rec.n_sets, reinterpret_cast<const int4 *>(r->image.data()), dsets,
                     dconds, dheads, c, cf, r->rec.n_cat > 0});
    } else {
      const int S = predict_samples_per_lane(r->nf);
      plds = std::max(plds, (size_t)r->nf * 64 * S * 4);
      for (int64_t row0 = 0; row0 < r->n_rows; row0 += 64 * S) {
        PredictTask t{};
        t.rows = reinterpret_cast<const float *>(dev + r->rows_off);
        t.set = dsets + r->set_index;
        t.conds = dconds;
        t.out = reinterpret_cast<int32_t *>(dev + r->out_off);
        t.n = r->n_rows;
        t.row0 = row0;
        t.nf = r->nf;
        t.S = S;
        ptasks.push_back(t);
      }
    }
  }
  BatchTables bt;
  build_batch_tables(src, kServeSplit, &bt);
  const size_t tables_off = al(cur);
  const size_t ptasks_off = al(tables_off + bt.bytes);
  const size_t in_end = al(ptasks_off + sizeof(PredictTask) * ptasks.size());
  hipError_t e = in_end <= need ? hipSuccess : hipErrorInvalidValue;
  if (e == hipSuccess) e = ensure_pinned(&slot.h_in, &slot.in_cap, in_end - out_end);
  if (e == hipSuccess) e = ensure_pinned(&slot.h_out, &slot.out_cap, std::max<size_t>(out_end, 1));
  BatchLaunch bl{};
  PredictLaunch pl{};
  if (e == hipSuccess) {
    // host image of the range [out_end, in_end)
    auto h = [&](size_t range_off) { return static_cast<char *>(slot.h_in) + (range_off - out_end); };
    for (Req *r : take) {
      std::memcpy(h(r->in_off), r->image.data(), r->L.total);
      if (r->kind == AERL_REQ_PREDICT && r->n_rows > 0)
        std::memcpy(h(r->rows_off), r->rows.data(), r->rows.size() * sizeof(float));
    }
    emit_batch_tables(bt, h(tables_off), dev + tables_off, n_cu, &bl);
    if (!ptasks.empty())
      std::memcpy(h(ptasks_off), ptasks.data(), sizeof(PredictTask) * ptasks.size());
    pl.tasks = reinterpret_cast<const PredictTask *>(dev + ptasks_off);
    pl.n_tasks = (int32_t)ptasks.size();
    pl.lds = plds;
    if (trace) e = hipEventRecord(slot.span[0], slot.stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dev + out_end, slot.h_in, in_end - out_end, hipMemcpyHostToDevice,
                         slot.stream);
  }
  if (e == hipSuccess && trace) e = hipEventRecord(slot.span[1], slot.stream);
  if (e == hipSuccess && !src.empty()) e = launch_batch(bl, slot.stream);
  if (e == hipSuccess && pl.n_tasks > 0) e = launch_predict_batch(pl, slot.stream);
  if (e == hipSuccess && trace) e = hipEventRecord(slot.span[2], slot.stream);
  if (e == hipSuccess && out_end > 0)
    e = hipMemcpyAsync(slot.h_out, dev, out_end, hipMemcpyDeviceToHost, slot.stream);
  if (e == hipSuccess && trace) e = hipEventRecord(slot.span[3], slot.stream);
  slot.out_bytes = out_end;
  if (e == hipSuccess) e = hipEventRecord(slot.done, slot.stream);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(slot.stream);
    lk.lock();
    reap(lk, slot, e);
    return true;
  }
  lk.lock();
  return true;
}

// Finishes a launch: copies outputs to the callers (status == hipSuccess),
// completes its tickets and returns its arena range.  Called with lk held;
// drops it around the copies.
void Serve::reap(std::unique_lock<std::mutex> &lk, Slot &slot, hipError_t status) {
  std::vector<Req *> rs = slot.reqs;
  lk.unlock();
  const Clock::time_point t_seen = Clock::now();
  if (status == hipSuccess) {
    const char *h = static_cast<const char *>(slot.h_out);
    for (Req *r : rs) {
      if (r->kind == AERL_REQ_FITNESS) {
        if (r->rec.n_sets > 0) std::memcpy(r->h_correct, h + r->out_off, r->correct_bytes());
        if (r->h_conf && r->rec.n_sets > 0)
          std::memcpy(r->h_conf, h + r->out_off + al(r->correct_bytes()), r->conf_bytes());
      } else if (r->n_rows > 0) {
        std::memcpy(r->h_pred, h + r->out_off, (size_t)r->n_rows * 4);
      }
    }
  }
  lk.lock();
  const Clock::time_point now = Clock::now();
  for (Req *r : rs) {
    r->status = status == hipSuccess ? AERL_OK : AERL_EDEVICE;
    r->t_seen_done = t_seen;
    r->t_done = now;
    r->done = true;
    if (r->kind == AERL_REQ_FITNESS && --ds_refs[r->dataset_id] == 0) ds_refs.erase(r->dataset_id);
    lat_us.push_back(us_between(r->t_submit, now));
    ++completed;
    nominal_done += r->nominal;
    r->image = std::vector<char>();
    r->rows = std::vector<float>();
  }
  t_last = now;
  if (trace) write_trace(slot, rs, status);
  alloc.release(slot.off, slot.bytes);
  slot.busy = false;
  slot.reqs.clear();
  cv_done.notify_all();
}

// One JSON line per request of a finished launch: the host spans (packing on
// the submitting thread, waiting in the queue, launch to completion seen by
// the scheduler, completion to outputs in the caller's buffers) and the
// launch's device spans from its timing events (upload, kernels, download),
// shared by every request of the launch.  Times in microseconds, the submit
// time from the loop's start.
void Serve::write_trace(const Slot &slot, const std::vector<Req *> &rs, hipError_t status) {
  float dev_ms[3] = {-1.0f, -1.0f, -1.0f};
  if (status == hipSuccess)
    for (int i = 0; i < 3; ++i)
      if (hipEventElapsedTime(&dev_ms[i], slot.span[i], slot.span[i + 1]) != hipSuccess) {
        (void)hipGetLastError();
        dev_ms[i] = -1.0f;
      }
  for (const Req *r : rs) {
    std::fprintf(trace,
                 "{\"ticket\": %llu, \"kind\": \"%s\", \"dataset\": %d, \"sets\": %d, "
                 "\"rows\": %lld, \"batch\": %d, \"slot\": %d, \"status\": %d, "
                 "\"submit_us\": %.1f, \"pack_us\": %.1f, \"queue_us\": %.1f, "
                 "\"launch_us\": %.1f, \"copy_out_us\": %.1f, \"total_us\": %.1f, "
                 "\"h2d_us\": %.1f, \"kernels_us\": %.1f, \"d2h_us\": %.1f}\n",
                 (unsigned long long)r->ticket, r->kind == AERL_REQ_FITNESS ? "fitness" : "predict",
                 r->kind == AERL_REQ_FITNESS ? r->dataset_id : -1, r->rec.n_sets,
                 (long long)r->n_rows, r->batch_size, slot.index, (int)r->status,
                 us_between(t_start, r->t_submit), us_between(r->t_submit, r->t_queued),
                 us_between(r->t_queued, r->t_launch), us_between(r->t_launch, r->t_seen_done),
                 us_between(r->t_seen_done, r->t_done), us_between(r->t_submit, r->t_done),
                 dev_ms[0] * 1e3, dev_ms[1] * 1e3, dev_ms[2] * 1e3);
  }
  std::fflush(trace);
}

void Serve::run() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(m);
  for (;;) {
    bool busy = false;
    for (Slot &s : slots) {
      if (!s.busy) continue;
      lk.unlock();
      const hipError_t q = hipEventQuery(s.done);
      lk.lock();
      if (q == hipErrorNotReady) {
        busy = true;
      } else {
        reap(lk, s, q);
      }
    }
    for (Slot &s : slots) {
      if (pending.empty()) break;
      if (s.busy) continue;
      if (!launch_one(lk, s)) break;  // the head does not fit yet: wait for a launch to end
      busy = busy || s.busy;
    }
    if (stopping && pending.empty() && !busy) break;
    if (busy) {
      cv_work.wait_for(lk, std::chrono::microseconds(20));
    } else {
      cv_work.wait(lk, [&] { return stopping || !pending.empty(); });
    }
  }
}

void serve_shutdown(aerl_ctx *ctx) {
  if (!ctx || !ctx->serve) return;
  if (ctx->serve->running) (void)aerl_serve_stop(ctx);
  delete ctx->serve;
  ctx->serve = nullptr;
}

bool serve_uses_dataset(aerl_ctx *ctx, int32_t dataset_id) {
  Serve *sv = ctx->serve;
  if (!sv) return false;
  std::lock_guard<std::mutex> lk(sv->m);
  return sv->ds_refs.count(dataset_id) > 0;
}

}  // namespace aerl

using namespace aerl;

namespace {

void free_slots(Serve *sv) {
  for (Slot &s : sv->slots) {
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.done) (void)hipEventDestroy(s.done);
    for (hipEvent_t ev : s.span)
      if (ev) (void)hipEventDestroy(ev);
    if (s.h_in) (void)hipHostFree(s.h_in);
    if (s.h_out) (void)hipHostFree(s.h_out);
  }
  sv->slots.clear();
}

void reset_stats(Serve *sv) {
  sv->lat_us.clear();
  sv->submitted = sv->completed = sv->launches = sv->launched_reqs = 0;
  sv->nominal_done = 0;
  sv->have_first = false;
  sv->arena_peak = sv->alloc.used();
}

Serve *running_serve(aerl_ctx *ctx) {
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  return ctx->serve && ctx->serve->running ? ctx->serve : nullptr;
}

}  // namespace

extern "C" {

aerl_status aerl_serve_start(aerl_ctx *ctx, void *arena, size_t arena_bytes,
                             const aerl_serve_cfg *cfg) {
  if (!ctx) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->err.clear();
  if (ctx->serve && ctx->serve->running) return fail(ctx, AERL_ESTATE, "serving loop already running");
  if (!arena || ((uintptr_t)arena & 255)) return fail(ctx, AERL_EINVAL, "arena is NULL or not 256-byte aligned");
  if (arena_bytes < 4096) return fail(ctx, AERL_EINVAL, "arena of %zu bytes is too small", arena_bytes);
  int32_t max_batch = cfg && cfg->max_batch > 0 ? cfg->max_batch : 256;
  int32_t max_inflight = cfg && cfg->max_inflight > 0 ? cfg->max_inflight : 4;
  if (max_inflight > 8) return fail(ctx, AERL_EINVAL, "max_inflight %d above 8", max_inflight);
  if (!ctx->serve) ctx->serve = new Serve();
  Serve *sv = ctx->serve;
  sv->ctx = ctx;
  sv->arena = static_cast<char *>(arena);
  sv->arena_bytes = arena_bytes;
  sv->max_batch = max_batch;
  sv->max_inflight = max_inflight;
  sv->device = ctx->device;
  sv->n_cu = ctx->n_cu;
  sv->alloc.reset(arena_bytes);
  sv->pending.clear();
  sv->reqs.clear();
  sv->ds_refs.clear();
  reset_stats(sv);
  AERL_HIP(ctx, hipSetDevice(ctx->device));
  // AERL_TRACE=<file>: append one JSON line per completed request
  const char *trace_path = std::getenv("AERL_TRACE");
  if (sv->trace) std::fclose(sv->trace);
  sv->trace = nullptr;
  if (trace_path && *trace_path) {
    sv->trace = std::fopen(trace_path, "a");
    if (!sv->trace) return fail(ctx, AERL_EINVAL, "cannot open the trace file %s", trace_path);
  }
  sv->t_start = Clock::now();
  sv->slots.assign(max_inflight, Slot{});
  int index = 0;
  for (Slot &s : sv->slots) {
    s.index = index++;
    hipError_t e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
    for (int i = 0; i < 4 && e == hipSuccess && sv->trace; ++i) e = hipEventCreate(&s.span[i]);
    if (e == hipSuccess) e = ensure_pinned(&s.h_in, &s.in_cap, kInitialPinned);
    if (e == hipSuccess) e = ensure_pinned(&s.h_out, &s.out_cap, kInitialPinned);
    if (e != hipSuccess) {
      free_slots(sv);
      if (sv->trace) std::fclose(sv->trace);
      sv->trace = nullptr;
      return fail(ctx, AERL_EDEVICE, "serving slot setup failed: %s", hipGetErrorString(e));
    }
  }
  sv->stopping = false;
  sv->running = true;
  sv->thr = std::thread([sv] { sv->run(); });
  return AERL_OK;
}

aerl_status aerl_serve_submit(aerl_ctx *ctx, const aerl_request *req, uint64_t *ticket) {
  if (!ctx) return AERL_EINVAL;
  // Checks and the dataset lookup under the context lock; validation and
  // packing (the expensive part) without it, so submitting threads pack in
  // parallel; the lookup is repeated when the request is queued.
  const Clock::time_point t0 = Clock::now();
  auto r = std::make_unique<Req>();
  Serve *sv = nullptr;
  {
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    ctx->err.clear();
    sv = ctx->serve;
    if (!sv || !sv->running) return fail(ctx, AERL_ESTATE, "serving loop is not running");
    if (!req || !ticket || !req->pop) return fail(ctx, AERL_EINVAL, "NULL request, population or ticket");
    r->kind = req->kind;
    if (req->kind == AERL_REQ_FITNESS) {
      auto it = ctx->datasets.find(req->dataset_id);
      if (it == ctx->datasets.end()) return fail(ctx, AERL_ENOENT, "unknown dataset %d", req->dataset_id);
      r->dsv = it->second;
      r->ds = &r->dsv;
      r->ds_reg = &it->second;
      r->dataset_id = req->dataset_id;
      if (req->n_features != r->ds->nf || req->n_classes != r->ds->nc)
        return fail(ctx, AERL_EINVAL, "request shape (%d features, %d classes) differs from the dataset's",
                    req->n_features, req->n_classes);
      if (req->pop->n_sets > 0 && !req->correct) return fail(ctx, AERL_EINVAL, "correct is NULL");
    } else if (req->kind == AERL_REQ_PREDICT) {
      if (req->n_rows < 0) return fail(ctx, AERL_EINVAL, "n_rows < 0");
      if (req->n_rows > 0 && (!req->rows || !req->pred)) return fail(ctx, AERL_EINVAL, "NULL rows or pred");
      if (req->set_index < 0 || req->set_index >= req->pop->n_sets)
        return fail(ctx, AERL_EINVAL, "set_index %d outside the population", req->set_index);
      if ((size_t)req->n_features * 64 * 4 > kDynLdsMax)
        return fail(ctx, AERL_EINVAL, "%d features exceed the prediction tile", req->n_features);
    } else {
      return fail(ctx, AERL_EINVAL, "unknown request kind %d", req->kind);
    }
  }
  r->nf = req->n_features;
  r->nc = req->n_classes;
  int32_t n_rules = 0, n_conds = 0;
  if (validate_population(nullptr, req->pop, r->nf, r->nc, &n_rules, &n_conds) != AERL_OK) {
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);  // again, for the message
    return validate_population(ctx, req->pop, r->nf, r->nc, &n_rules, &n_conds);
  }
  r->L = packed_layout(req->pop->n_sets, n_rules, n_conds);
  r->image.resize(r->L.total);
  pack_population_image(req->pop, r->nf, r->nc, n_rules, n_conds, r->image.data(), &r->rec);
  const int4 *hsets = reinterpret_cast<const int4 *>(r->image.data() + r->L.sets_off);
  if (r->kind == AERL_REQ_FITNESS) {
    r->h_correct = req->correct;
    r->h_conf = req->confusion;
    r->in_bytes = al(r->L.total);
    r->out_bytes = al(r->correct_bytes()) + al(r->conf_bytes());
    const int64_t tasks = batch_task_count(*r->ds, r->rec.n_sets, kServeSplit);
    r->table_bytes = sizeof(BatchItem) + 2 * sizeof(BatchZero) + (size_t)tasks * sizeof(BatchTask);
    r->nominal = (double)r->ds->n * (double)r->rec.nominal_conds;
  } else {
    r->set_index = req->set_index;
    r->n_rows = req->n_rows;
    r->h_pred = req->pred;
    if (r->n_rows > 0) r->rows.assign(req->rows, req->rows + (size_t)r->n_rows * r->nf);
    r->in_bytes = al(r->L.total) + al((size_t)r->n_rows * r->nf * 4);
    r->out_bytes = al((size_t)r->n_rows * 4);
    const int S = predict_samples_per_lane(r->nf);
    r->table_bytes = (size_t)((r->n_rows + 64 * S - 1) / (64 * S)) * sizeof(PredictTask);
    r->nominal = (double)r->n_rows * (double)hsets[r->set_index].w;
  }
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (sv != ctx->serve || !sv->running) return fail(ctx, AERL_ESTATE, "serving loop is not running");
  if (r->dev_bytes() + kTableSlack > sv->arena_bytes)
    return fail(ctx, AERL_ENOMEM, "request needs %zu bytes of the %zu-byte arena",
                r->dev_bytes() + kTableSlack, sv->arena_bytes);
  if (r->kind == AERL_REQ_FITNESS) {
    auto it = ctx->datasets.find(r->dataset_id);
    if (it == ctx->datasets.end() || &it->second != r->ds_reg)
      return fail(ctx, AERL_ENOENT, "dataset %d was released", r->dataset_id);
  }
  std::lock_guard<std::mutex> sl(sv->m);
  if (sv->stopping) return fail(ctx, AERL_ESTATE, "serving loop is stopping");
  r->t_submit = t0;
  r->t_queued = Clock::now();
  r->ticket = sv->next_ticket++;
  if (!sv->have_first) {
    sv->have_first = true;
    sv->t_first = r->t_submit;
  }
  ++sv->submitted;
  if (r->kind == AERL_REQ_FITNESS) ++sv->ds_refs[r->dataset_id];
  *ticket = r->ticket;
  sv->pending.push_back(r.get());
  sv->reqs[r->ticket] = std::move(r);
  sv->cv_work.notify_one();
  return AERL_OK;
}

aerl_status aerl_serve_wait(aerl_ctx *ctx, uint64_t ticket, int64_t timeout_us, aerl_result *res) {
  if (!ctx) return AERL_EINVAL;
  Serve *sv = nullptr;
  {
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    sv = ctx->serve;
  }
  if (!sv) return AERL_ENOENT;
  std::unique_lock<std::mutex> lk(sv->m);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return AERL_ENOENT;
  Req *r = it->second.get();
  if (timeout_us < 0) {
    sv->cv_done.wait(lk, [&] { return r->done; });
  } else if (!sv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return r->done; })) {
    return AERL_ETIMEDOUT;
  }
  if (res) {
    res->status = r->status;
    res->batch_size = r->batch_size;
    res->queue_us = us_between(r->t_submit, r->t_launch);
    res->latency_us = us_between(r->t_submit, r->t_done);
  }
  sv->reqs.erase(it);
  return AERL_OK;
}

aerl_status aerl_serve_stats(aerl_ctx *ctx, struct aerl_serve_stats *out, int32_t reset) {
  if (!ctx) return AERL_EINVAL;
  Serve *sv = running_serve(ctx);
  if (!sv) return fail(ctx, AERL_ESTATE, "serving loop is not running");
  if (!out) return fail(ctx, AERL_EINVAL, "out is NULL");
  std::lock_guard<std::mutex> lk(sv->m);
  struct aerl_serve_stats s{};
  s.submitted = sv->submitted;
  s.completed = sv->completed;
  s.launches = sv->launches;
  s.mean_batch = sv->launches ? (double)sv->launched_reqs / sv->launches : 0.0;
  s.arena_peak = sv->arena_peak;
  if (!sv->lat_us.empty()) {
    std::vector<double> v = sv->lat_us;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {  // nearest-rank percentile
      const double rank = std::max(1.0, std::ceil(p * (double)v.size()));
      return v[std::min(v.size(), (size_t)rank) - 1];
    };
    s.p50_us = pct(0.50);
    s.p99_us = pct(0.99);
    s.max_us = v.back();
    double sum = 0;
    for (double x : v) sum += x;
    s.mean_us = sum / v.size();
    const double span = us_between(sv->t_first, sv->t_last) * 1e-6;
    if (span > 0) {
      s.requests_per_s = sv->completed / span;
      s.cond_evals_per_s = sv->nominal_done / span;
    }
  }
  *out = s;
  if (reset) reset_stats(sv);
  return AERL_OK;
}

aerl_status aerl_serve_stop(aerl_ctx *ctx) {
  if (!ctx) return AERL_EINVAL;
  Serve *sv = running_serve(ctx);
  if (!sv) return fail(ctx, AERL_ESTATE, "serving loop is not running");
  {
    std::lock_guard<std::mutex> lk(sv->m);
    sv->stopping = true;
    sv->cv_work.notify_all();
  }
  sv->thr.join();
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  {
    std::lock_guard<std::mutex> sl(sv->m);
    sv->running = false;
    free_slots(sv);
    if (sv->trace) std::fclose(sv->trace);
    sv->trace = nullptr;
    sv->ds_refs.clear();
    sv->cv_done.notify_all();
  }
  return AERL_OK;
}

}  // extern "C"
