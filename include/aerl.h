/*
 * aerl.h - C ABI of libaerl, a gfx950 (AMD Instinct MI355X) library that
 * evaluates whole populations of tensorized rule sets on a resident dataset.
 *
 * Method: Shahrzad & Miikkulainen, "GPU-Accelerated Rule Evaluation and
 * Evolution" (AERL).  Section 3 describes the tensorized rule form (Fig. 1a:
 * each condition is one row of weights plus a bias, evaluated as
 * w.x + b > 0), the step activation used for inference, the sigmoid
 * relaxation used to fine-tune coefficients by back-propagation, and the
 * split between evolution on the CPU and evaluation on the GPU, which this
 * interface is.
 *
 * Conventions
 * -----------
 * - Every call returns aerl_status: AERL_OK (0) or a negative code.  The
 *   message of the last failure on a context is aerl_last_error(ctx).  No
 *   C++ exception crosses this interface.
 * - Device memory is always owned by the caller (for example PyTorch
 *   tensors).  The library never frees caller memory; it keeps non-owning
 *   references to registered dataset and population buffers until they are
 *   released.  The library owns only host-side state (registries, pinned
 *   staging buffers, events, graphs, threads).
 * - Calls that take a hipStream_t enqueue work on that stream and return
 *   before it finishes unless stated otherwise.  Outputs are valid once the
 *   stream has reached that point.
 * - One context per host thread for the direct calls.  The serving calls
 *   (aerl_serve_*) are thread-safe.
 * - Hard results are bit-exact: conditions compare individually rounded
 *   IEEE fp32 products (no fused multiply-add, subnormals kept), and counts
 *   are integers.
 */
#ifndef AERL_H
#define AERL_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t aerl_status;
enum {
  AERL_OK = 0,
  AERL_EINVAL = -1,    /* invalid argument or input data, nothing enqueued */
  AERL_ENOMEM = -2,    /* a caller-supplied buffer or host allocation is too small */
  AERL_EDEVICE = -3,   /* a HIP runtime call failed; message holds the HIP error */
  AERL_ENOENT = -4,    /* unknown dataset, population or ticket id */
  AERL_EAGAIN = -5,    /* serving: admission budget is full, try again */
  AERL_ETIMEDOUT = -6, /* serving: wait timed out, the ticket stays valid */
  AERL_ESTATE = -7     /* call not valid in the current state */
};

/* Limits of the library. */
#define AERL_MAX_CLASSES 64        /* classes per dataset */
#define AERL_MAX_FEATURES 512      /* features per dataset (one LDS tile row each) */
#define AERL_MAX_RULE_CONDS 255    /* conditions per rule */
#define AERL_TILE 256              /* samples per layout tile (class regions are padded to it) */

/* Condition operators and kinds (Section 3, Fig. 1a/b). */
enum { AERL_OP_LT = 0, AERL_OP_LE = 1, AERL_OP_GT = 2, AERL_OP_GE = 3 };
enum {
  AERL_KIND_THRESHOLD = 0,  /* coef*x[f] op theta            (one non-zero weight)            */
  AERL_KIND_FEATURE = 1,    /* coef*x[f] op coef2*x[g]      (two non-zero weights, zero bias) */
  AERL_KIND_CATEGORICAL = 2 /* x[f] in a set of category codes (Section 5's categorical features) */
};

typedef struct aerl_ctx aerl_ctx;

/* Create a context bound to HIP device `device_ordinal`.  *out receives the
 * context (NULL on failure).  Errors: AERL_EINVAL (bad ordinal or NULL out),
 * AERL_EDEVICE. */
aerl_status aerl_create(aerl_ctx **out, int device_ordinal);

/* Destroy a context: stops serving if running, waits for the library's own
 * host work, releases host state.  Caller device memory is untouched.
 * Accepts NULL. */
void aerl_destroy(aerl_ctx *ctx);

/* Message of the last failed call on ctx.  Library-owned, valid until the
 * next call on ctx.  Never NULL ("" when nothing failed). */
const char *aerl_last_error(const aerl_ctx *ctx);

/* ------------------------------------------------------------------ data */

/* Largest sample count a dataset with n_classes classes may hold: the
 * label-grouped layout pads every class region to a multiple of AERL_TILE
 * samples and indexes the padded samples with int32, so
 * (ceil(n / AERL_TILE) + n_classes) * AERL_TILE must stay below 2^31.
 * Pure host arithmetic; n_classes outside [1, AERL_MAX_CLASSES] gives 0. */
int64_t aerl_max_samples(int32_t n_classes);

/* Bytes of the caller-allocated device buffer that holds a resident dataset
 * of n samples x f features with n_classes classes (feature-major samples,
 * labels, tile table, tau and upload scratch).  Pure host arithmetic.
 * Errors: AERL_EINVAL (n < 0, n > aerl_max_samples(n_classes), f < 1,
 * f > AERL_MAX_FEATURES, n_classes < 1 or > AERL_MAX_CLASSES). */
aerl_status aerl_dataset_bytes(int64_t n, int32_t f, int32_t n_classes, size_t *bytes);

/* Register a labeled dataset (Section 1: fitness is classification
 * accuracy on a labeled dataset; Section 4.1 uses one such table).
 *   x         device, fp32 [n][f] row-major, every value finite
 *   y         device, int32 [n], each in [0, n_classes)
 *   mem       device buffer of aerl_dataset_bytes(n, f, n_classes) bytes,
 *             256-byte aligned, owned by the caller and kept alive until
 *             aerl_release_dataset; x and y may be freed after return.
 * The library stably groups the samples by label, pads each class region
 * to a multiple of AERL_TILE samples, stores the features feature-major
 * (fp32 [f][n_pad], rows 1 KiB-aligned), and computes
 * tau[f] = 0.05 * (population std of feature f), fp64 then rounded to fp32
 * (1 where the std is 0), which scales the soft relaxation.  Permuting the
 * samples never changes a fitness count.
 * Synchronous: returns after the layout is complete on `stream`.
 * *dataset_id receives the id.  Errors: AERL_EINVAL (sizes, non-finite
 * feature, label out of range, misaligned or NULL pointers), AERL_ENOMEM
 * (mem_bytes too small), AERL_EDEVICE. */
aerl_status aerl_upload_dataset(aerl_ctx *ctx, const float *x, const int32_t *y, int64_t n,
                                int32_t f, int32_t n_classes, void *mem, size_t mem_bytes,
                                hipStream_t stream, int32_t *dataset_id);

/* Information about a registered dataset.  Pointers are into its `mem`:
 *   x_fm   fp32 [f][n_pad] (label-grouped order), y_pad int32 [n_pad]
 *          (-1 on padding), perm int32 [n_pad] (original sample index or
 *          -1), tau fp32 [f].
 * Errors: AERL_ENOENT. */
typedef struct {
  int64_t n, n_pad;
  int32_t n_features, n_classes;
  int64_t class_count[AERL_MAX_CLASSES];
  const float *x_fm;
  const int32_t *y_pad;
  const int32_t *perm;
  const float *tau;
} aerl_dataset_info;
aerl_status aerl_dataset_query(aerl_ctx *ctx, int32_t dataset_id, aerl_dataset_info *info);

/* Forget a dataset.  The caller may free its `mem` once every stream that
 * used it has finished.  Errors: AERL_ENOENT, AERL_ESTATE (served requests
 * on it are still in flight). */
aerl_status aerl_release_dataset(aerl_ctx *ctx, int32_t dataset_id);

/* ------------------------------------------------------------ population */

/* A population as produced by the evolution loop (Section 3: evolution
 * runs on the CPU and hands candidates to the GPU).  HOST arrays, structure
 * of arrays.  Rule set s owns rules [set_rule_off[s], set_rule_off[s+1]) in
 * order, then falls back to set_default[s] (first rule that fires decides).
 * Rule r owns conditions [rule_cond_off[r], rule_cond_off[r+1]) (an AND)
 * and predicts rule_class[r].  Condition j is
 *   kind 0: coef[j]*x[f[j]] op[j] theta[j]
 *   kind 1: coef[j]*x[f[j]] op[j] coef2[j]*x[g[j]]
 *   kind 2: x[f[j]] is a category code k in 0..63 (the value is exactly the
 *           integer k) with bit k of cat_mask[j] set; any other value (a
 *           fraction, a negative, 64 or more, an infinity, NaN) is in no
 *           set.  An equality test is a one-code set.  op and coef are
 *           not used.  The soft relaxation takes the condition's truth as
 *           its soft truth (it has nothing to tune): its gradients are 0.
 * with each product rounded to fp32 once.  Empty rule sets and empty rules
 * (an empty AND always fires) are allowed. */
typedef struct {
  int32_t n_sets;
  const int32_t *set_rule_off;  /* [n_sets+1], set_rule_off[0] == 0, non-decreasing */
  const int32_t *set_default;   /* [n_sets] */
  const int32_t *rule_cond_off; /* [n_rules+1], rule_cond_off[0] == 0, non-decreasing */
  const int32_t *rule_class;    /* [n_rules] */
  const uint8_t *op;            /* [n_conds] AERL_OP_* */
  const uint8_t *kind;          /* [n_conds] AERL_KIND_* */
  const int32_t *f;             /* [n_conds] */
  const int32_t *g;             /* [n_conds], read for kind 1 only */
  const float *coef;            /* [n_conds] */
  const float *coef2;           /* [n_conds], read for kind 1 only */
  const float *theta;           /* [n_conds], read for kind 0 only; +-inf allowed */
  const uint64_t *cat_mask;     /* [n_conds], read for kind 2 only; may be NULL without kind 2 */
} aerl_population;

/* Bytes of the device workspace that holds the packed form of `pop`.
 * Validates the structure (offsets, ops, kinds, classes, feature indices
 * against n_features, g != f for kind 1, finite coefficients, non-NaN
 * thresholds, at most AERL_MAX_RULE_CONDS conditions per rule and at most
 * 1022 conditions per rule set, an empty rule counting as one).
 * Errors: AERL_EINVAL with the first offending index in the message. */
aerl_status aerl_population_bytes(const aerl_population *pop, int32_t n_features,
                                  int32_t n_classes, size_t *bytes);

/* Validate and pack `pop` into the caller's device workspace `ws`
 * (ws_bytes >= aerl_population_bytes, 256-byte aligned, kept alive until
 * aerl_release_population).  The host arrays may be reused once the call
 * returns: they are copied into library-owned pinned staging memory and
 * sent with an asynchronous copy on `stream`.  *pop_id receives the id.
 * Errors: AERL_EINVAL, AERL_ENOMEM, AERL_EDEVICE. */
aerl_status aerl_pack_population(aerl_ctx *ctx, const aerl_population *pop, int32_t n_features,
                                 int32_t n_classes, void *ws, size_t ws_bytes, hipStream_t stream,
                                 int32_t *pop_id);

/* Host-only variant of the packing step: validates `pop` and writes its
 * packed image (the bytes aerl_pack_population sends to the device) into
 * host memory `dst` of at least aerl_population_bytes bytes.  Lets tools and
 * tests inspect the exact comparison forms the kernels evaluate.  Errors:
 * AERL_EINVAL, AERL_ENOMEM. */
aerl_status aerl_pack_population_host(const aerl_population *pop, int32_t n_features,
                                      int32_t n_classes, void *dst, size_t dst_bytes);

/* Forget a packed population (waits for its staging copy).  Its pinned
 * host staging buffer stays with the context for later packs of a similar
 * size (at most 8 buffers and 512 MiB kept; aerl_destroy frees them).
 * Errors: AERL_ENOENT. */
aerl_status aerl_release_population(aerl_ctx *ctx, int32_t pop_id);

/* ------------------------------------------------------------------ hard */

/* Fitness of every rule set of pop_id on dataset_id (Section 1: accuracy on
 * labeled data; Section 3: step activation, AND of conditions, first
 * firing rule, else the default class).
 *   correct    device int32 [n_sets]: samples whose prediction equals the label
 *   confusion  device int32 [n_sets][C][C] ([true][predicted]) or NULL
 * Outputs are overwritten (no accumulation).  Bit-exact.  With two to four
 * classes, at least 4 Mi (256-sample tile, rule set) pairs and at most
 * 512 MiB of per-tile counts ((C-1) 10-bit fields per rule set and tile)
 * the call keeps those counts in a device buffer the context owns
 * (allocated or grown on the first call that needs more, freed by
 * aerl_destroy); calls that use it run one after another, also across
 * streams.  Errors:
 * AERL_ENOENT, AERL_EINVAL (feature count or class count of the population
 * and dataset differ, NULL correct), AERL_EDEVICE. */
aerl_status aerl_eval_population(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id,
                                 int32_t *correct, int32_t *confusion, hipStream_t stream);

/* Launch configuration aerl_eval_population picks for a dataset with the
 * given per-class sample counts (class_count[n_classes]) and a population of
 * n_sets rule sets on a GPU with n_cu compute units.  Pure host arithmetic,
 * the same planner the call runs.
 *   samples_per_lane, sets_per_chunk, tiles_per_group  as in
 *                    aerl_eval_population_cfg
 *   workgroups       one per (chunk of rule sets, group of tiles), in a
 *                    one-dimensional grid of 1024-thread workgroups
 * Datasets past 65,535 x 255 tiles take groups of several tiles so that the
 * grid's work-item count fits 32 bits.  Errors: AERL_EINVAL (bad counts,
 * a total above aerl_max_samples, n_sets < 0, n_cu < 1, or a grid that
 * does not fit even with 255-tile groups). */
typedef struct {
  int32_t samples_per_lane, sets_per_chunk, tiles_per_group, pad;
  int64_t workgroups;
} aerl_eval_launch;
aerl_status aerl_eval_plan(const int64_t *class_count, int32_t n_classes, int32_t n_features,
                           int32_t n_sets, int32_t n_cu, aerl_eval_launch *out);

/* aerl_eval_population with an explicit launch configuration (used by the
 * autotuner and by tests that cover every code path):
 *   samples_per_lane  1, 2 or 4 (a wave covers 64*samples_per_lane samples)
 *   sets_per_chunk    rule sets per workgroup, >= 1
 *   tiles_per_group   AERL_TILE-sample tiles per workgroup, 1..255
 * Same outputs, bit for bit, for every valid configuration.  Errors: as
 * aerl_eval_population, plus AERL_EINVAL for a configuration whose LDS
 * footprint does not fit or whose grid exceeds the launch limit. */
aerl_status aerl_eval_population_cfg(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id,
                                     int32_t *correct, int32_t *confusion,
                                     int32_t samples_per_lane, int32_t sets_per_chunk,
                                     int32_t tiles_per_group, hipStream_t stream);

/* Predicted class of rule set `set` of pop_id for n rows (Section 3,
 * inference with the step activation).
 *   rows  device fp32 [n][f] row-major (f = the population's feature count)
 *   pred  device int32 [n]
 * Errors: AERL_ENOENT, AERL_EINVAL (set out of range, n < 0), AERL_EDEVICE. */
aerl_status aerl_predict(aerl_ctx *ctx, int32_t pop_id, int32_t set, const float *rows, int64_t n,
                         int32_t *pred, hipStream_t stream);

/* ----------------------------------------------------------- ragged batch */

/* Many independent evaluations (each its own dataset and population, of any
 * shapes) in ONE persistent launch, the form in which an evolution loop that
 * runs several populations or datasets keeps the whole GPU busy (Section 3:
 * candidates are handed to the GPU for evaluation; Section 4.3 and Fig. 3: the cost
 * varies with the number of rules and conditions per generation).  Results
 * are bit-identical to aerl_eval_population of each item. */
typedef struct {
  int32_t dataset_id;
  int32_t pop_id;
  int32_t *correct;   /* device int32 [n_sets of pop] */
  int32_t *confusion; /* device int32 [n_sets][C][C] or NULL */
} aerl_batch_item;

/* Work split of a batch: rule sets per work item, AERL_TILE-sample tiles per
 * work item (at most 255), and the LDS budget of a block's feature tile in
 * KiB (an item takes 4, 2 or 1 samples per lane, the most whose 64-lane
 * tile of all its features fits the budget; above 80 only one block fits a
 * CU).  0 in a field asks for the library's choice (the tuned one when
 * aerl_autotune has seen a batch of this shape, else 512 sets, 1 tile,
 * 64 KiB). */
typedef struct {
  int32_t sets_per_task;
  int32_t tiles_per_task;
  int32_t tile_kib;
} aerl_batch_cfg;

enum {
  AERL_BATCH_GRAPH = 1 /* capture the launch sequence once in a hipGraph and replay it */
};

/* Device workspace needed by aerl_batch_plan for these items and cfg (NULL
 * cfg = library choice).  Errors: AERL_ENOENT, AERL_EINVAL. */
aerl_status aerl_batch_workspace_bytes(aerl_ctx *ctx, const aerl_batch_item *items,
                                       int32_t n_items, const aerl_batch_cfg *cfg,
                                       size_t *bytes);

/* Build the work list of a batch (one work item = a chunk of rule sets of one
 * item on a group of label-uniform tiles of its dataset, ordered by
 * estimated cost, largest first) and store it in the caller's device
 * workspace `ws` (kept alive until aerl_batch_release); the tables are
 * copied before the call returns (`stream` is synchronized).  With
 * AERL_BATCH_GRAPH the zeroing of the outputs and the persistent kernel are
 * captured once (on a private stream) into a hipGraph that every
 * aerl_batch_run replays on its stream.  ws: 256-byte aligned.
 * The items' datasets, populations and output buffers must stay registered
 * and allocated while the plan exists.  *plan_id receives the id.
 * Errors: AERL_ENOENT, AERL_EINVAL (shape mismatch, NULL outputs),
 * AERL_ENOMEM (ws too small), AERL_EDEVICE. */
aerl_status aerl_batch_plan(aerl_ctx *ctx, const aerl_batch_item *items, int32_t n_items,
                            const aerl_batch_cfg *cfg, void *ws, size_t ws_bytes, uint32_t flags,
                            hipStream_t stream, int32_t *plan_id);

/* Run a plan on `stream`: zero every item's outputs, then one persistent
 * kernel whose workgroups pull work items from a device counter until the
 * list is exhausted.  Asynchronous.  Errors: AERL_ENOENT, AERL_EDEVICE. */
aerl_status aerl_batch_run(aerl_ctx *ctx, int32_t plan_id, hipStream_t stream);

/* Forget a plan (and its graph).  Errors: AERL_ENOENT. */
aerl_status aerl_batch_release(aerl_ctx *ctx, int32_t plan_id);

/* Autotuner: times the batch under candidate work-splits on `stream`
 * (outputs are overwritten), keeps the fastest for batches of this shape
 * (number of items, and per item the feature count, sample tiles, rule sets
 * and conditions, each bucketed by powers of two) and returns it in *best
 * with its time in *best_ms.  Later plans with cfg NULL or zero fields use
 * it.  With AERL_AUTOTUNE_CACHE set in the environment the table is also
 * read from and appended to that file.  ws as for aerl_batch_plan with the
 * largest candidate (aerl_batch_workspace_bytes with cfg {1, 1, 64}).
 * Errors: as aerl_batch_plan. */
aerl_status aerl_autotune(aerl_ctx *ctx, const aerl_batch_item *items, int32_t n_items, void *ws,
                          size_t ws_bytes, hipStream_t stream, aerl_batch_cfg *best,
                          float *best_ms);

/* -------------------------------------------------------------- serving */

/* A request loop over resident datasets: evolution workers (Section 3: the
 * CPU side evolves candidates and hands them to the GPU for scoring) submit
 * fitness and prediction requests of any size from any thread; the loop
 * admits them in arrival order as long as their device footprint fits in
 * the caller's arena (the HBM budget), packs every request admitted while
 * earlier launches are still running into the next launch (one persistent
 * fitness kernel plus one prediction kernel, on one of several streams, so
 * launches overlap), and hands results back per request.  Results are
 * bit-identical to aerl_eval_population / aerl_predict of the same request
 * alone. */
enum { AERL_REQ_FITNESS = 0, AERL_REQ_PREDICT = 1 };

typedef struct {
  int32_t max_batch;    /* most requests per launch; 0 = 256 */
  int32_t max_inflight; /* launches that may be on the device at once, 1..8; 0 = 4 */
} aerl_serve_cfg;

typedef struct {
  int32_t kind;                /* AERL_REQ_FITNESS or AERL_REQ_PREDICT */
  int32_t dataset_id;          /* fitness: a resident dataset (its shape must match) */
  const aerl_population *pop;  /* host; copied and packed during submit */
  int32_t n_features, n_classes;
  int32_t set_index;           /* predict: the rule set of pop to apply */
  const float *rows;           /* predict: host fp32 [n_rows][n_features], copied during submit */
  int64_t n_rows;
  int32_t *correct;            /* fitness: host int32 [n_sets] */
  int32_t *confusion;          /* fitness: host int32 [n_sets][C][C] or NULL */
  int32_t *pred;               /* predict: host int32 [n_rows] */
} aerl_request;

typedef struct {
  aerl_status status;  /* AERL_OK, or the device error that ended the launch */
  int32_t batch_size;  /* requests in the launch that carried this one */
  double queue_us;     /* submit -> launch */
  double latency_us;   /* submit -> outputs written to the caller's buffers */
} aerl_result;

struct aerl_serve_stats {
  int64_t submitted, completed, launches;
  double p50_us, p99_us, mean_us, max_us; /* latency of completed requests */
  double requests_per_s;   /* completed / (last completion - first submit) */
  double cond_evals_per_s; /* nominal condition evaluations over the same span */
  double mean_batch;       /* requests per launch */
  size_t arena_peak;       /* most arena bytes in use at once */
};

/* Start the loop on ctx's device.  arena: caller-allocated device memory
 * (256-byte aligned) whose size is the admission budget; it must outlive
 * aerl_serve_stop.  cfg may be NULL.  When the environment variable
 * AERL_TRACE names a file at start, the loop appends one JSON line per
 * completed request: ticket, kind, dataset, sets, rows, batch, slot,
 * status, submit_us (from start), the host spans pack_us (validation and
 * packing), queue_us, launch_us (launch to completion seen), copy_out_us
 * (outputs to the caller's buffers), total_us, and its launch's device spans
 * h2d_us, kernels_us, d2h_us (-1 when the launch failed).  Errors:
 * AERL_ESTATE (already running), AERL_EINVAL (bad arena or configuration,
 * a trace file that cannot be opened), AERL_EDEVICE. */
aerl_status aerl_serve_start(aerl_ctx *ctx, void *arena, size_t arena_bytes,
                             const aerl_serve_cfg *cfg);

/* Submit one request; returns at once with *ticket.  Inputs are copied, so
 * the caller may reuse them; output buffers must stay valid until the
 * ticket completes.  Errors: AERL_ESTATE (not running), AERL_ENOENT (unknown
 * dataset), AERL_EINVAL (invalid population, shape mismatch, bad set_index,
 * NULL outputs), AERL_ENOMEM (the request alone exceeds the arena). */
aerl_status aerl_serve_submit(aerl_ctx *ctx, const aerl_request *req, uint64_t *ticket);

/* Wait for a ticket (timeout_us < 0: no limit) and collect it: its outputs
 * are in the caller's buffers and *res (may be NULL) tells how it went.  A
 * collected ticket is forgotten.  Errors: AERL_ENOENT (unknown or already
 * collected), AERL_ETIMEDOUT (not done yet; the ticket stays). */
aerl_status aerl_serve_wait(aerl_ctx *ctx, uint64_t ticket, int64_t timeout_us, aerl_result *res);

/* Latency and throughput since start (or the last reset).  reset != 0
 * clears the counters after reading them.  Errors: AERL_ESTATE. */
aerl_status aerl_serve_stats(aerl_ctx *ctx, struct aerl_serve_stats *out, int32_t reset);

/* Finish every accepted request (outputs written), then stop the loop and
 * free its streams and host buffers.  Completed tickets stay collectable by
 * aerl_serve_wait until the next aerl_serve_start or aerl_destroy, which
 * must not race with a waiting thread.  Errors: AERL_ESTATE (not running). */
aerl_status aerl_serve_stop(aerl_ctx *ctx);

/* ------------------------------------------------------------------ soft */

/* Device scratch needed by aerl_soft_forward / aerl_soft_backward for this
 * dataset and population (per-block partial sums that are reduced in a
 * fixed order, which keeps results bit-identical from run to run, and one
 * 16-byte record per condition gathered at each call).
 * Errors: AERL_ENOENT, AERL_EINVAL. */
aerl_status aerl_soft_workspace_bytes(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id,
                                      size_t *forward_bytes, size_t *backward_bytes);

/* Soft loss of every rule set (Section 3: a sigmoid replaces the step so
 * that coefficients can be tuned by back-propagation).  Condition j has soft
 * truth sigmoid(z_j), z_j = s_j*(coef[j]*x[f] - theta[j])/tau[f] (kind 0) or
 * s_j*(coef[j]*x[f] - coef2[j]*x[g])/tau[f] (kind 1), s_j = +1 for > and >=,
 * -1 for < and <=.  A rule's soft truth is the product over its
 * conditions; rule k fires first with probability r_k*prod_{i<k}(1-r_i);
 * the rest goes to the default class.  loss[s] = mean over samples of
 * min(-log P(label), 100).  Computed in log space in fp32; the parameter
 * arrays (device fp32 [n_conds], the population's condition order) are
 * live values and may differ from the packed ones; the population's
 * structure (ops, kinds, features, classes) is used.
 *   loss  device fp32 [n_sets]
 *   ws    device scratch of at least forward_bytes (aerl_soft_workspace_bytes)
 * Deterministic (fixed reduction order).  Errors: AERL_ENOENT, AERL_EINVAL,
 * AERL_EDEVICE. */
aerl_status aerl_soft_forward(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id, const float *coef,
                              const float *coef2, const float *theta, float *loss, void *ws,
                              size_t ws_bytes, hipStream_t stream);

/* Gradient of sum_s dloss[s]*loss[s] with respect to coef, coef2 and theta
 * (device fp32 [n_conds] each; coef2 entries of kind-0 conditions and
 * theta entries of kind-1 conditions are written as 0).  The adjoint
 * recomputes every sigmoid instead of storing activations.  dloss is
 * device fp32 [n_sets]; ws holds at least backward_bytes.  Deterministic.
 * Rule sets of up to 32 rules run with the per-rule state in per-lane
 * memory; longer ones keep it in LDS with fewer waves per workgroup as they
 * grow, which bounds them (about 300 rules with few features).  Errors:
 * AERL_ENOENT, AERL_EINVAL (also: rule sets too long for the adjoint
 * kernel), AERL_EDEVICE. */
aerl_status aerl_soft_backward(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id,
                               const float *coef, const float *coef2, const float *theta,
                               const float *dloss, float *dcoef, float *dcoef2, float *dtheta,
                               void *ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------- softmax head */

/* Soft loss of every rule set under the softmax head (Section 5: a softmax
 * activation gives probabilistic, finer-grained class outputs).  Condition
 * soft truths as in aerl_soft_forward; every rule votes for its class with
 * its soft truth r_k, the default class receives the probability that no
 * rule fires, D = prod_k (1 - r_k):
 *   v_c = sum_{k: class_k = c} r_k + [c = default] * D,
 *   P_c = exp(beta * v_c) / sum_c' exp(beta * v_c'),
 * loss[s] = mean over samples of min(-log P(label), 100).  The order of the
 * rules does not matter under this head.  beta: finite, >= 0 (the
 * sharpness).  At most 16 classes.  ws: forward_bytes of
 * aerl_soft_workspace_bytes.  Deterministic.  Errors: as aerl_soft_forward,
 * plus AERL_EINVAL (more than 16 classes, bad beta). */
aerl_status aerl_softmax_forward(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id,
                                 const float *coef, const float *coef2, const float *theta,
                                 float beta, float *loss, void *ws, size_t ws_bytes,
                                 hipStream_t stream);

/* Gradient of sum_s dloss[s] * loss[s] under the softmax head (outputs as
 * aerl_soft_backward): dL/dv_c = beta (P_c - [c = y]),
 * dL/dr_k = dL/dv_{class_k} - dL/dv_default * prod_{i != k} (1 - r_i),
 * dL/dz = dL/dr_k * r_k * sigmoid(-z).  Every sigmoid is recomputed.
 * ws: backward_bytes.  Deterministic.  Errors: as aerl_soft_backward, plus
 * AERL_EINVAL (more than 16 classes, rule sets too long for the kernel's
 * LDS, bad beta). */
aerl_status aerl_softmax_backward(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id,
                                  const float *coef, const float *coef2, const float *theta,
                                  float beta, const float *dloss, float *dcoef, float *dcoef2,
                                  float *dtheta, void *ws, size_t ws_bytes, hipStream_t stream);

/* Class probabilities P_c (the softmax head) of rule set `set` for n
 * request rows: rows device fp32 [n][f] row-major, probs device fp32
 * [n][C]; tau comes from dataset_id (the table the rule sets were tuned
 * on).  Non-finite rows give non-finite probabilities.  ws: forward_bytes.
 * Errors: AERL_ENOENT, AERL_EINVAL, AERL_EDEVICE. */
aerl_status aerl_softmax_proba(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id, int32_t set,
                               const float *coef, const float *coef2, const float *theta,
                               float beta, const float *rows, int64_t n, float *probs, void *ws,
                               size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------ fine-tuning */

/* Optimizers of aerl_finetune.  The paper tunes the coefficients by
 * back-propagation for 50 epochs (Sections 3 and 4.1) without naming the
 * update rule; both common ones are offered. */
#define AERL_OPT_ADAM 0 /* Adam with bias correction (beta1, beta2, eps) */
#define AERL_OPT_SGD 1  /* plain gradient descent, p -= lr * g */
typedef struct {
  int32_t epochs;    /* full-batch steps, >= 0 */
  int32_t optimizer; /* AERL_OPT_ADAM or AERL_OPT_SGD */
  float lr;          /* > 0, finite */
  float beta1, beta2, eps; /* Adam: in [0, 1), [0, 1), > 0; ignored by SGD */
} aerl_finetune_cfg;

/* Device scratch of aerl_finetune for this dataset and population (the
 * adjoint's partial sums, the gradients, the optimizer moments).  Errors:
 * AERL_ENOENT. */
aerl_status aerl_finetune_workspace_bytes(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id,
                                          size_t *bytes);

/* Fine-tune every rule set of pop_id on dataset_id (Section 3: gradients of
 * the sigmoid relaxation adjust the rule coefficients without changing the
 * logical structure; Section 4.1: 50 epochs of gradient updates).  Each
 * epoch is one full-batch step: the adjoint of aerl_soft_backward over the
 * whole dataset with dloss = 1 for every rule set (each rule set is its own
 * model), then one fused optimizer update, on the device, of each
 * condition's coefficient and of its threshold (threshold condition) or
 * second coefficient (feature-vs-feature condition).  The other entry of the
 * pair is never written, and the population's structure (features, ops,
 * rules, classes) is unchanged.
 *   coef, coef2, theta  device fp32 [n_conds], the starting values, updated
 *                       in place
 *   loss_hist           device fp32 [epochs + 1][n_sets]: row e is the soft
 *                       loss after e updates; NULL skips these forward passes
 *   ws                  device scratch of aerl_finetune_workspace_bytes
 * Asynchronous on stream; deterministic.  The tuned parameters are scored
 * with the step activation by packing them (aerl_pack_population) and
 * calling aerl_eval_population.  Errors: AERL_ENOENT, AERL_EINVAL (bad cfg,
 * NULL arrays, shapes, rule sets too long for the adjoint), AERL_ENOMEM (ws
 * too small), AERL_EDEVICE. */
aerl_status aerl_finetune(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id,
                          const aerl_finetune_cfg *cfg, float *coef, float *coef2, float *theta,
                          float *loss_hist, void *ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------ evolution */

/* The evolution loop that feeds the library (Section 3: evolution on the
 * CPU by tournament selection and offspring with randomized coefficients,
 * candidates evaluated on the GPU, optional back-propagation every
 * generation whose tuned fitness steers selection, the Baldwin effect;
 * Section 4.1: a pool of 100 candidate rule sets).  The paper names no
 * operator details; the ones below are this library's reading.
 *
 * Random stream: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), state s:
 *   next(): s += 0x9e3779b97f4a7c15; z = s; z = (z ^ z >> 30) * 0xbf58476d1ce4e5b9;
 *           z = (z ^ z >> 27) * 0x94d049bb133111eb; return z ^ z >> 31
 *   below(n) = ((next() >> 32) * n) >> 32;  unit() = (next() >> 40) * 2^-24
 * Random condition: feature-vs-feature if unit() < ff_frac (and F >= 2);
 *   f = below(F); g = (f + 1 + below(F - 1)) % F (feature-vs-feature);
 *   op = below(4); coef = unit(); then coef2 = unit() (feature-vs-feature)
 *   or theta = (float)(lo[f] + unit() * (hi[f] - lo[f])) in double.
 * Random rule: class = below(C), one random condition.  Random pool: per
 *   rule set R = 1 + below(max_rules), default = below(C); per rule
 *   K = 1 + below(max_conds), class = below(C), K random conditions.
 * Next generation from pool P with fitness F: the elite best (fitness
 *   descending, ties by index) pass unchanged; each other slot: child = copy
 *   of tournament() (tournament draws i = below(pool) that many times and
 *   keeps the fittest, ties to the lower index); if unit() < p_crossover,
 *   B = tournament(), ca = below(R_child + 1), cb = below(R_B + 1), rules =
 *   child[0, ca) + B[cb, R_B) (child[0, 1) if empty), cut to max_rules; each
 *   condition in order: if unit() < p_coef, coef = unit() then coef2 or
 *   theta redrawn as for a random condition; if unit() < p_struct, t =
 *   below(4): 0 add a random condition to rule below(R) if it has fewer
 *   than max_conds; 1 drop condition below(K_r) of rule r = below(R) if
 *   K_r >= 2; 2 insert a random rule at below(R + 1) if R < max_rules;
 *   3 drop rule below(R) if R >= 2.  Draws guarded by a condition happen
 *   only when it holds. */
typedef struct {
  int32_t pool;        /* rule sets per generation, >= 2 (the paper: 100) */
  int32_t tournament;  /* tournament size, >= 1 */
  int32_t elite;       /* best rule sets kept unchanged, 0 .. pool - 1 */
  int32_t max_rules;   /* rules per rule set, 1 .. 64 */
  int32_t max_conds;   /* conditions per rule, 1 .. AERL_MAX_RULE_CONDS,
                          max_rules * max_conds <= 1022 */
  float ff_frac;       /* probability that a new condition compares two features */
  float p_crossover, p_coef, p_struct; /* probabilities, in [0, 1] */
  int32_t tune_epochs; /* fine-tuning epochs per generation, 0 = none */
  aerl_finetune_cfg tune; /* its optimizer (the epochs field is ignored) */
  uint64_t seed;       /* initial SplitMix64 state */
} aerl_evolve_cfg;

/* A pool written by the library into caller arrays of capacity
 * pool + 1, pool, pool * max_rules + 1, pool * max_rules and
 * pool * max_rules * max_conds. */
typedef struct {
  int32_t n_sets, n_rules, n_conds; /* written */
  int32_t *set_rule_off, *set_default, *rule_cond_off, *rule_class;
  uint8_t *op, *kind;
  int32_t *f, *g;
  float *coef, *coef2, *theta;
} aerl_population_out;

/* Host-only steps of the loop (no GPU): a random initial pool, and the next
 * generation from a pool and its fitness (correct counts), as specified
 * above.  lo, hi: per-feature ranges [F] for drawn thresholds; *rng_state is
 * the SplitMix64 state, advanced.  Errors: AERL_EINVAL (cfg, ranges, pool
 * not of cfg->pool rule sets or outside max_rules / max_conds). */
aerl_status aerl_random_pool(const aerl_evolve_cfg *cfg, int32_t n_features, int32_t n_classes,
                             const float *lo, const float *hi, uint64_t *rng_state,
                             aerl_population_out *out);
aerl_status aerl_breed(const aerl_population *pool, const int32_t *fitness,
                       const aerl_evolve_cfg *cfg, int32_t n_features, int32_t n_classes,
                       const float *lo, const float *hi, uint64_t *rng_state,
                       aerl_population_out *out);

/* Device bytes of the arena a run on dataset_id needs (packed pools,
 * fitness, and with fine-tuning the parameters and the tuning workspace).
 * Errors: AERL_ENOENT. */
aerl_status aerl_evolve_arena_bytes(aerl_ctx *ctx, int32_t dataset_id, const aerl_evolve_cfg *cfg,
                                    size_t *bytes);

/* Start a run on dataset_id: generation 0 is `initial` (cfg->pool rule sets
 * within max_rules / max_conds) or, when NULL, a random pool drawn from the
 * seed; it is evaluated before the call returns.  Each evaluation packs the
 * pool, scores it with aerl_eval_population and copies the counts to the
 * host; with tune_epochs > 0 the pool is first fine-tuned on the device
 * (aerl_finetune), and the tuned rule sets are scored (Baldwinian: the pool
 * itself keeps its untuned coefficients).  arena: device memory of
 * aerl_evolve_arena_bytes, 256-byte aligned, the caller's, used until
 * aerl_evolve_release.  Synchronous on stream.  Errors: AERL_ENOENT,
 * AERL_EINVAL, AERL_ENOMEM (arena too small), AERL_EDEVICE. */
aerl_status aerl_evolve_create(aerl_ctx *ctx, int32_t dataset_id, const aerl_evolve_cfg *cfg,
                               const float *lo, const float *hi, const aerl_population *initial,
                               void *arena, size_t arena_bytes, hipStream_t stream,
                               int32_t *evo_id);

/* Breed and evaluate `generations` more generations.  Synchronous.  Errors:
 * AERL_ENOENT, AERL_EINVAL, AERL_EDEVICE. */
aerl_status aerl_evolve_run(aerl_ctx *ctx, int32_t evo_id, int32_t generations, hipStream_t stream);

/* The current generation: its pool, its fitness (of the tuned rule sets when
 * fine-tuning), the tuned parameters (NULL without fine-tuning), the random
 * state and host wall-clock seconds spent so far evaluating, tuning and
 * breeding.  Library-owned arrays, valid until the next call on evo_id. */
typedef struct {
  int32_t generation, pad;
  aerl_population pool;
  const int32_t *fitness;
  const float *tuned_coef, *tuned_coef2, *tuned_theta;
  uint64_t rng_state;
  double seconds_eval, seconds_tune, seconds_breed;
} aerl_evolve_info;
aerl_status aerl_evolve_state(aerl_ctx *ctx, int32_t evo_id, aerl_evolve_info *out);

/* Checkpoint a run to a file (configuration, ranges, generation, random
 * state, pool, fitness, tuned parameters) and resume one on a dataset of the
 * same shape: the resumed run continues exactly as the saved one would.
 * Errors: AERL_ENOENT, AERL_EINVAL (unreadable or inconsistent file),
 * AERL_ENOMEM, AERL_EDEVICE. */
aerl_status aerl_evolve_save(aerl_ctx *ctx, int32_t evo_id, const char *path);
aerl_status aerl_evolve_load(aerl_ctx *ctx, int32_t dataset_id, const char *path, void *arena,
                             size_t arena_bytes, int32_t *evo_id);
aerl_status aerl_evolve_release(aerl_ctx *ctx, int32_t evo_id);

/* ---------------------------------------------------------- measurement */

/* Issue rates of the VALU instruction classes a roofline of the soft path
 * weights (Section 4.3 measures cost against the amount of rule and
 * condition work; this prices that work on the device).  Runs, on `stream`,
 * a kernel of fp32 multiply chains and one of chains alternating v_exp_f32
 * and v_log_f32, each filling every SIMD, and writes out[0] = multiply
 * lane-ops per second, out[1] = transcendental lane-ops per second (their
 * ratio is the issue cost of a transcendental in multiply slots).  Blocks
 * until both kernels finish; allocates about 4 MiB of device memory for the
 * call.  Errors: AERL_EINVAL (null argument), AERL_EDEVICE. */
aerl_status aerl_probe_valu_rates(aerl_ctx *ctx, double *out, hipStream_t stream);

/* aerl_soft_forward for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and the same results, bit for bit, with the
 * per-block partial sums and condition records kept in a scratch array the
 * library holds in device memory, one per GPU, AERL_NOALLOC_SCRATCH_BYTES
 * long, from the GPU's first aerl_create until the process ends.  The
 * caller passes inputs and outputs only.  The call allocates nothing
 * (no hipMalloc, no library allocation).  Every call on a GPU shares that
 * GPU's array: calls that overlap on one GPU (concurrent streams, threads
 * or contexts) race and must be serialized by the caller; a call's
 * partial sums are overwritten by the next call.  Errors: AERL_ENOMEM when
 * the call would need more than AERL_NOALLOC_SCRATCH_BYTES of scratch
 * (aerl_soft_workspace_bytes' forward_bytes), otherwise as
 * aerl_soft_forward. */
#define AERL_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
aerl_status aerl_soft_forward_noalloc(aerl_ctx *ctx, int32_t dataset_id, int32_t pop_id,
                                      const float *coef, const float *coef2, const float *theta,
                                      float *loss, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* AERL_H */
