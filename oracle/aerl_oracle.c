/*
 * Plain CPU oracle for tensorized rule-set evaluation (AERL, Shahrzad &
 * Miikkulainen, "GPU-Accelerated Rule Evaluation and Evolution").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liborc and is called
 * by the test suite, by the smoke check and by the benchmark's CPU-baseline
 * leg.  The product library never links, loads or calls it, and it shares no
 * source with the library.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 * On x86-64 float arithmetic is IEEE single (SSE), denormals are kept (no
 * fast-math startup code sets FTZ/DAZ) and contraction is off, so every
 * float product below is one correctly rounded IEEE product.
 *
 * What is computed
 * ----------------
 * Hard path (Section 3, Fig. 1): a condition row of the paper's rule tensor
 * with weights w and bias b fires when w.x + b > 0 (the step activation maps
 * non-positive sums to false and positive sums to true).  With one weight
 * this is  c*x[f] > theta  (theta = -b); with two weights and zero bias it is
 * c*x[f] > c2*x[g]  (Fig. 1a, second row of rule 1).  A rule fires when all
 * of its conditions hold (the "&" of Fig. 1b); rules are numbered and each
 * maps to a class.  Resolution: the first rule that fires gives the class,
 * otherwise the rule set's default class.  Fitness is classification
 * accuracy (Section 1): the count of samples whose predicted class equals
 * the label, plus the confusion matrix [true][predicted].
 * The operators <, <=, >, >= are all allowed; the paper writes "<" as a
 * negated feature, and -c*x > -t is the same test as c*x < t.
 *
 * Soft path (Section 3, the sigmoid relaxation used for back-propagation):
 * the paper names only "a differentiable activation (e.g. sigmoid)".  The
 * reading used here: a condition's soft truth is sigmoid(z) with
 *   z = s*(c*x[f] - theta)/tau_f          (threshold condition)
 *   z = s*(c*x[f] - c2*x[g])/tau_f        (feature-vs-feature)
 * s = +1 for > and >=, -1 for < and <=, tau_f = 0.05 * std_f (population
 * std over the dataset, fp64, stored as float32; 1 if std_f = 0).  A rule's
 * soft truth r_k is the product of its conditions' soft truths; rule k is the
 * first to fire with probability r_k * prod_{i<k} (1 - r_i); nobody fires
 * with probability prod_i (1 - r_i), which goes to the default class.  The
 * class probability P_c sums these over rules of class c (and the default).
 * Per-sample loss L = min(-log P_y, 100); a rule set's loss is the mean over
 * samples.  Everything is done in log space in fp64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int32_t n_sets;
  const int32_t *set_rule_off;  /* [n_sets+1] */
  const int32_t *set_default;   /* [n_sets] */
  const int32_t *rule_cond_off; /* [n_rules+1] */
  const int32_t *rule_class;    /* [n_rules] */
  const uint8_t *op;            /* [n_conds] 0 <, 1 <=, 2 >, 3 >= */
  const uint8_t *kind;          /* [n_conds] 0 threshold, 1 feature-vs-feature, 2 categorical */
  const int32_t *f, *g;         /* [n_conds] */
  const float *coef, *coef2, *theta; /* [n_conds] */
  const uint64_t *cat_mask;     /* [n_conds], categorical conditions only (may be NULL) */
} orc_population;

/* Categorical condition (Section 5 names categorical features as an
 * extension).  Reading: the feature holds category codes 0..63 as floats;
 * the condition holds when x[f] is exactly one of the codes in the set
 * (bit k of cat_mask for code k).  Any other value (a fraction, a negative,
 * 64 and above, an infinity, NaN) is in no set.  Equality is a one-code set. */
static int category_member(uint64_t mask, float v) {
  if (!(v >= 0.0f && v <= 63.0f)) return 0;
  if (v != floorf(v)) return 0;
  return (int)((mask >> (int)v) & 1u);
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of one call's parallel region: nthreads when positive, else the
 * OpenMP default.  Passed as a num_threads clause, so a call never changes
 * the thread count of later calls. */
static int pick_threads(int nthreads) {
#ifdef _OPENMP
  return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

/* ------------------------------------------------------------------ hard */

/* One IEEE comparison; the operands are never NaN for finite inputs. */
static int compare(int op, float lhs, float rhs) {
  switch (op) {
    case 0: return lhs < rhs;
    case 1: return lhs <= rhs;
    case 2: return lhs > rhs;
    default: return lhs >= rhs;
  }
}

/* Truth of condition j on sample row xr (Section 3: one row of the rule
 * tensor against one sample).  Each product is rounded to float once. */
static int condition_holds(const orc_population *p, int64_t j, const float *xr) {
  if (p->kind[j] == 2) return category_member(p->cat_mask[j], xr[p->f[j]]);
  float lhs = p->coef[j] * xr[p->f[j]];
  float rhs = p->kind[j] ? p->coef2[j] * xr[p->g[j]] : p->theta[j];
  return compare(p->op[j], lhs, rhs);
}

/* Class predicted by rule set s for sample row xr: the first rule whose
 * conditions all hold, else the default class (Fig. 1b decision list). */
static int32_t predict_one(const orc_population *p, int32_t s, const float *xr) {
  for (int32_t k = p->set_rule_off[s]; k < p->set_rule_off[s + 1]; ++k) {
    int fires = 1;
    for (int32_t j = p->rule_cond_off[k]; j < p->rule_cond_off[k + 1]; ++j) {
      if (!condition_holds(p, j, xr)) { fires = 0; break; }
    }
    if (fires) return p->rule_class[k];
  }
  return p->set_default[s];
}

/* correct[s] = #samples with predicted class == label;
 * confusion[s][true][pred] (optional, may be NULL).  x is [n][nf] row-major. */
int orc_hard_eval(int64_t n, int32_t nf, const float *x, const int32_t *y, int32_t nc,
                  const orc_population *p, int32_t *correct, int32_t *confusion, int nthreads) {
  const int nt = pick_threads(nthreads);
  (void)nt;
  int64_t cc = (int64_t)nc * nc;
  if (confusion) memset(confusion, 0, sizeof(int32_t) * (size_t)(p->n_sets * cc));
#pragma omp parallel for schedule(static) num_threads(nt)
  for (int32_t s = 0; s < p->n_sets; ++s) {
    int32_t good = 0;
    for (int64_t i = 0; i < n; ++i) {
      int32_t pred = predict_one(p, s, x + i * nf);
      if (pred == y[i]) ++good;
      if (confusion) confusion[s * cc + (int64_t)y[i] * nc + pred] += 1;
    }
    correct[s] = good;
  }
  (void)nf;
  return 0;
}

/* pred[i] = class rule set s predicts for row i of x ([n][nf]). */
int orc_predict(int64_t n, int32_t nf, const float *x, const orc_population *p, int32_t s,
                int32_t *pred) {
  for (int64_t i = 0; i < n; ++i) pred[i] = predict_one(p, s, x + i * nf);
  return 0;
}

/* Work a 64-lane wave must do under wave-uniform early exit.  For every rule
 * set and every tile (a list of sample indices): walk the rules in order
 * while some sample of the tile is still undecided; within a rule walk the
 * conditions in order while some undecided sample still passes all
 * conditions seen so far; every condition visited counts once (threshold and
 * feature-vs-feature separately).  The samples that pass a whole rule become
 * decided.  Output: work_t[s], work_ff[s] summed over tiles. */
int orc_workcount(int64_t n_tiles, const int64_t *tile_ptr, const int64_t *tile_idx, int32_t nf,
                  const float *x, const orc_population *p, int64_t *work_t, int64_t *work_ff,
                  int nthreads) {
  const int nt = pick_threads(nthreads);
  (void)nt;
  int64_t max_tile = 0;
  for (int64_t t = 0; t < n_tiles; ++t)
    if (tile_ptr[t + 1] - tile_ptr[t] > max_tile) max_tile = tile_ptr[t + 1] - tile_ptr[t];
  int bad = 0;
#pragma omp parallel num_threads(nt)
  {
    unsigned char *undecided = (unsigned char *)malloc((size_t)max_tile + 1);
    unsigned char *alive = (unsigned char *)malloc((size_t)max_tile + 1);
    if (!undecided || !alive) {
#pragma omp atomic write
      bad = 1;
    }
#pragma omp for schedule(static)
    for (int32_t s = 0; s < p->n_sets; ++s) {
      int64_t wt = 0, wf = 0;
      if (undecided && alive) {
        for (int64_t t = 0; t < n_tiles; ++t) {
          int64_t a = tile_ptr[t], m = tile_ptr[t + 1] - a;
          int64_t n_und = m;
          for (int64_t i = 0; i < m; ++i) undecided[i] = 1;
          for (int32_t k = p->set_rule_off[s]; k < p->set_rule_off[s + 1] && n_und > 0; ++k) {
            int64_t n_alive = 0;
            for (int64_t i = 0; i < m; ++i) { alive[i] = undecided[i]; n_alive += alive[i]; }
            for (int32_t j = p->rule_cond_off[k]; j < p->rule_cond_off[k + 1] && n_alive > 0; ++j) {
              if (p->kind[j] == 1) ++wf; else ++wt;
              n_alive = 0;
              for (int64_t i = 0; i < m; ++i) {
                if (alive[i]) {
                  alive[i] = (unsigned char)condition_holds(p, j, x + tile_idx[a + i] * nf);
                  n_alive += alive[i];
                }
              }
            }
            for (int64_t i = 0; i < m; ++i)
              if (alive[i]) { undecided[i] = 0; --n_und; }
          }
        }
      }
      work_t[s] = wt;
      work_ff[s] = wf;
    }
    free(undecided);
    free(alive);
  }
  return bad ? -2 : 0;
}

/* ------------------------------------------------------------------ soft */

/* tau_f = 0.05 * std_f over all n samples (population std, fp64 two-pass),
 * rounded to float; 1 where the std is 0. */
int orc_tau(int64_t n, int32_t nf, const float *x, float *tau) {
  for (int32_t f = 0; f < nf; ++f) {
    double sum = 0.0;
    for (int64_t i = 0; i < n; ++i) sum += (double)x[i * nf + f];
    double mean = n > 0 ? sum / (double)n : 0.0;
    double ss = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double d = (double)x[i * nf + f] - mean;
      ss += d * d;
    }
    double sd = n > 0 ? sqrt(ss / (double)n) : 0.0;
    tau[f] = sd > 0.0 ? (float)(0.05 * sd) : 1.0f;
  }
  return 0;
}

/* log(sigmoid(z)) = -softplus(-z), softplus(t) = max(t,0) + log1p(exp(-|t|)). */
static double log_sigmoid(double z) {
  double t = -z;
  return -((t > 0 ? t : 0.0) + log1p(exp(-fabs(t))));
}

/* log(1 - exp(a)) for a <= 0 (Maechler 2012: expm1 branch above -ln 2,
 * log1p branch below).  a = 0 gives -inf. */
static double log1mexp(double a) {
  if (a >= 0.0) return -INFINITY;
  return a > -M_LN2 ? log(-expm1(a)) : log1p(-exp(a));
}

/* log(exp(a) + exp(b)) with -inf handled. */
static double lse2(double a, double b) {
  double m = a > b ? a : b;
  if (m == -INFINITY) return -INFINITY;
  return m + log1p(exp(-fabs(a - b)));
}

static double cond_sign(int op) { return op >= 2 ? 1.0 : -1.0; }

/* z of condition j for sample row xr (soft reading above), fp64. */
static double cond_z(const orc_population *p, const double *coef, const double *coef2,
                     const double *theta, int64_t j, const float *xr, const float *tau) {
  int f = p->f[j];
  /* a categorical condition has no parameter to relax: its soft truth is
   * its truth, sigmoid(+inf) = 1 or sigmoid(-inf) = 0 */
  if (p->kind[j] == 2) return category_member(p->cat_mask[j], xr[f]) ? INFINITY : -INFINITY;
  double lhs = coef[j] * (double)xr[f];
  double rhs = p->kind[j] ? coef2[j] * (double)xr[p->g[j]] : theta[j];
  return cond_sign(p->op[j]) * (lhs - rhs) / (double)tau[f];
}

/* Per-sample log class probabilities of rule set s (logp[nc]); fills
 * a[k], b[k] (log r_k, log(1-r_k)) for the rules of s when not NULL. */
static void soft_sample(const orc_population *p, const double *coef, const double *coef2,
                        const double *theta, int32_t s, const float *xr, const float *tau,
                        int32_t nc, double *logp, double *a, double *b) {
  for (int c = 0; c < nc; ++c) logp[c] = -INFINITY;
  double surv = 0.0; /* log prod_{i<k} (1 - r_i) */
  int32_t k0 = p->set_rule_off[s];
  for (int32_t k = k0; k < p->set_rule_off[s + 1]; ++k) {
    double ak = 0.0;
    for (int32_t j = p->rule_cond_off[k]; j < p->rule_cond_off[k + 1]; ++j)
      ak += log_sigmoid(cond_z(p, coef, coef2, theta, j, xr, tau));
    double bk = log1mexp(ak);
    int c = p->rule_class[k];
    logp[c] = lse2(logp[c], ak + surv);
    surv += bk;
    if (a) { a[k - k0] = ak; b[k - k0] = bk; }
  }
  int d = p->set_default[s];
  logp[d] = lse2(logp[d], surv);
}

/* Per-sample class log-probabilities of one rule set: logp[n][nc]. */
int orc_soft_logprobs(int64_t n, int32_t nf, const float *x, const float *tau, int32_t nc,
                      const orc_population *p, const double *coef, const double *coef2,
                      const double *theta, int32_t s, double *logp) {
  for (int64_t i = 0; i < n; ++i)
    soft_sample(p, coef, coef2, theta, s, x + i * nf, tau, nc, logp + i * nc, NULL, NULL);
  return 0;
}

#define LOSS_CAP 100.0
#define MAX_CLASSES 256

/* loss[s] = mean over samples of min(-log P_y, 100). */
int orc_soft_forward(int64_t n, int32_t nf, const float *x, const int32_t *y, const float *tau,
                     int32_t nc, const orc_population *p, const double *coef, const double *coef2,
                     const double *theta, double *loss, int nthreads) {
  if (nc > MAX_CLASSES) return -1;
  const int nt = pick_threads(nthreads);
  (void)nt;
#pragma omp parallel for schedule(static) num_threads(nt)
  for (int32_t s = 0; s < p->n_sets; ++s) {
    double logp[MAX_CLASSES];
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      soft_sample(p, coef, coef2, theta, s, x + i * nf, tau, nc, logp, NULL, NULL);
      double L = -logp[y[i]];
      acc += L > LOSS_CAP ? LOSS_CAP : L;
    }
    loss[s] = n > 0 ? acc / (double)n : 0.0;
  }
  return 0;
}

/* Same loss, evaluated naively in probability space (no logs until the
 * end).  Only meaningful where nothing saturates; a cross-check of the
 * log-space form. */
int orc_soft_forward_naive(int64_t n, int32_t nf, const float *x, const int32_t *y,
                           const float *tau, int32_t nc, const orc_population *p,
                           const double *coef, const double *coef2, const double *theta,
                           double *loss) {
  for (int32_t s = 0; s < p->n_sets; ++s) {
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      const float *xr = x + i * nf;
      double none = 1.0, py = 0.0;
      for (int32_t k = p->set_rule_off[s]; k < p->set_rule_off[s + 1]; ++k) {
        double r = 1.0;
        for (int32_t j = p->rule_cond_off[k]; j < p->rule_cond_off[k + 1]; ++j)
          r *= 1.0 / (1.0 + exp(-cond_z(p, coef, coef2, theta, j, xr, tau)));
        if (p->rule_class[k] == y[i]) py += r * none;
        none *= 1.0 - r;
      }
      if (p->set_default[s] == y[i]) py += none;
      double L = -log(py);
      acc += L > LOSS_CAP ? LOSS_CAP : L;
    }
    loss[s] = n > 0 ? acc / (double)n : 0.0;
  }
  (void)nc;
  return 0;
}

/* Gradient of loss[s] (weighted by dloss[s]) with respect to every coef,
 * coef2 and theta.  Derivation (one sample, label y, rules k = 0..R-1):
 *   V_k = P(class y | rules 0..k did not fire): V_{R-1} = [default == y],
 *         V_{k-1} = [class_k == y] r_k + (1 - r_k) V_k,   P_y = V_{-1};
 *   dP_y/dr_k = prod_{m<k}(1 - r_m) ([class_k == y] - V_k);
 *   dL/da_k  = -(r_k/P_y) prod_{m<k}(1 - r_m) ([class_k == y] - V_k),
 * with a_k = log r_k = sum_j log sigmoid(z_kj), so dL/dz_kj = dL/da_k *
 * sigmoid(-z_kj).  All in log space: U_k = log V_k, l_k = a_k + sum_{m<k}
 * b_m.  A clamped sample (-log P_y > 100) contributes nothing.
 * dz/dc = s x_f / tau_f, dz/dtheta = -s / tau_f, dz/dc2 = -s x_g / tau_f. */
int orc_soft_backward(int64_t n, int32_t nf, const float *x, const int32_t *y, const float *tau,
                      int32_t nc, const orc_population *p, const double *coef,
                      const double *coef2, const double *theta, const double *dloss,
                      double *dcoef, double *dcoef2, double *dtheta, int nthreads) {
  int32_t n_conds = p->rule_cond_off[p->set_rule_off[p->n_sets]];
  memset(dcoef, 0, sizeof(double) * (size_t)n_conds);
  memset(dcoef2, 0, sizeof(double) * (size_t)n_conds);
  memset(dtheta, 0, sizeof(double) * (size_t)n_conds);
  int32_t max_r = 0;
  for (int32_t s = 0; s < p->n_sets; ++s) {
    int32_t r = p->set_rule_off[s + 1] - p->set_rule_off[s];
    if (r > max_r) max_r = r;
  }
  const int nt = pick_threads(nthreads);
  (void)nt;
  int bad = 0;
#pragma omp parallel num_threads(nt)
  {
    double *a = (double *)malloc(sizeof(double) * (size_t)(max_r + 1));
    double *b = (double *)malloc(sizeof(double) * (size_t)(max_r + 1));
    double *U = (double *)malloc(sizeof(double) * (size_t)(max_r + 1));
    double logp[MAX_CLASSES];
    if (!a || !b || !U) {
#pragma omp atomic write
      bad = 1;
    }
#pragma omp for schedule(static)
    for (int32_t s = 0; s < p->n_sets; ++s) {
      if (!a || !b || !U) continue;
      int32_t k0 = p->set_rule_off[s], R = p->set_rule_off[s + 1] - k0;
      double scale = n > 0 ? dloss[s] / (double)n : 0.0;
      for (int64_t i = 0; i < n; ++i) {
        const float *xr = x + i * nf;
        int32_t yi = y[i];
        soft_sample(p, coef, coef2, theta, s, xr, tau, nc, logp, a, b);
        double logpy = logp[yi];
        if (-logpy > LOSS_CAP) continue;
        /* reverse sweep: U[k] = log V_k */
        double u = p->set_default[s] == yi ? 0.0 : -INFINITY;
        for (int32_t k = R - 1; k >= 0; --k) {
          U[k] = u;
          double hit = p->rule_class[k0 + k] == yi ? a[k] : -INFINITY;
          u = lse2(hit, b[k] + u);
        }
        /* forward sweep: dL/da_k, then per condition */
        double surv = 0.0;
        for (int32_t k = 0; k < R; ++k) {
          double lk = a[k] + surv;
          double g;
          if (p->rule_class[k0 + k] == yi)
            g = -exp(lk - logpy) * (-expm1(U[k]));
          else
            g = exp(lk + U[k] - logpy);
          surv += b[k];
          if (g == 0.0) continue;
          int32_t kk = k0 + k;
          for (int32_t j = p->rule_cond_off[kk]; j < p->rule_cond_off[kk + 1]; ++j) {
            if (p->kind[j] == 2) continue; /* no parameters */
            double z = cond_z(p, coef, coef2, theta, j, xr, tau);
            double dz = g * exp(log_sigmoid(-z)); /* dL/dz = dL/da * sigmoid(-z) */
            int f = p->f[j];
            double st = cond_sign(p->op[j]) / (double)tau[f];
            double tc = scale * dz * st * (double)xr[f];
            double t2 = -scale * dz * st * (p->kind[j] == 1 ? (double)xr[p->g[j]] : 1.0);
            dcoef[j] += tc;
            if (p->kind[j] == 1)
              dcoef2[j] += t2;
            else
              dtheta[j] += t2;
          }
        }
      }
    }
    free(a);
    free(b);
    free(U);
  }
  return bad ? -2 : 0;
}

/* ------------------------------------------------------------ softmax head
 * Section 5 names probabilistic outputs through a softmax activation as a
 * variant.  Reading: every rule votes for its class with its soft truth
 * r_k = prod_j sigmoid(z_kj), the default class receives the probability
 * that no rule fires, D = prod_k (1 - r_k):
 *   v_c = sum_{k: class_k = c} r_k + [c = default] * D,
 *   P_c = exp(beta * v_c) / sum_c' exp(beta * v_c'),
 * L = min(-log P_y, 100), loss = mean over samples.  Unlike the first-firing
 * relaxation, the order of the rules does not matter. */

static void smax_votes(const orc_population *p, const double *coef, const double *coef2,
                       const double *theta, int32_t s, const float *xr, const float *tau,
                       int32_t nc, double *v, double *r) {
  for (int c = 0; c < nc; ++c) v[c] = 0.0;
  double none = 1.0;
  int32_t k0 = p->set_rule_off[s];
  for (int32_t k = k0; k < p->set_rule_off[s + 1]; ++k) {
    double lr = 0.0;
    for (int32_t j = p->rule_cond_off[k]; j < p->rule_cond_off[k + 1]; ++j)
      lr += log_sigmoid(cond_z(p, coef, coef2, theta, j, xr, tau));
    double rk = exp(lr);
    v[p->rule_class[k]] += rk;
    none *= 1.0 - rk;
    if (r) r[k - k0] = rk;
  }
  v[p->set_default[s]] += none;
}

/* log P_c for every class from the votes. */
static void smax_logp(const double *v, int32_t nc, double beta, double *logp) {
  double m = -INFINITY;
  for (int c = 0; c < nc; ++c)
    if (beta * v[c] > m) m = beta * v[c];
  double sum = 0.0;
  for (int c = 0; c < nc; ++c) sum += exp(beta * v[c] - m);
  for (int c = 0; c < nc; ++c) logp[c] = beta * v[c] - m - log(sum);
}

/* Class probabilities of rule set s for every sample: probs[n][nc]. */
int orc_smax_probs(int64_t n, int32_t nf, const float *x, const float *tau, int32_t nc,
                   const orc_population *p, const double *coef, const double *coef2,
                   const double *theta, int32_t s, double beta, double *probs) {
  if (nc > MAX_CLASSES) return -1;
  double v[MAX_CLASSES], lp[MAX_CLASSES];
  for (int64_t i = 0; i < n; ++i) {
    smax_votes(p, coef, coef2, theta, s, x + i * nf, tau, nc, v, NULL);
    smax_logp(v, nc, beta, lp);
    for (int c = 0; c < nc; ++c) probs[i * nc + c] = exp(lp[c]);
  }
  return 0;
}

int orc_smax_forward(int64_t n, int32_t nf, const float *x, const int32_t *y, const float *tau,
                     int32_t nc, const orc_population *p, const double *coef, const double *coef2,
                     const double *theta, double beta, double *loss, int nthreads) {
  if (nc > MAX_CLASSES) return -1;
  const int nt = pick_threads(nthreads);
  (void)nt;
#pragma omp parallel for schedule(static) num_threads(nt)
  for (int32_t s = 0; s < p->n_sets; ++s) {
    double v[MAX_CLASSES], lp[MAX_CLASSES];
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      smax_votes(p, coef, coef2, theta, s, x + i * nf, tau, nc, v, NULL);
      smax_logp(v, nc, beta, lp);
      double L = -lp[y[i]];
      acc += L > LOSS_CAP ? LOSS_CAP : L;
    }
    loss[s] = n > 0 ? acc / (double)n : 0.0;
  }
  return 0;
}

/* Gradient of sum_s dloss[s] * loss[s] under the softmax head, by the chain
 * rule written out: dL/dv_c = beta (P_c - [c = y]);
 * dL/dr_k = dL/dv_{class_k} - dL/dv_default * prod_{i != k} (1 - r_i);
 * dL/dz_kj = dL/dr_k * r_k * sigmoid(-z_kj); clamped samples contribute
 * nothing. */
int orc_smax_backward(int64_t n, int32_t nf, const float *x, const int32_t *y, const float *tau,
                      int32_t nc, const orc_population *p, const double *coef,
                      const double *coef2, const double *theta, double beta, const double *dloss,
                      double *dcoef, double *dcoef2, double *dtheta, int nthreads) {
  if (nc > MAX_CLASSES) return -1;
  int32_t n_conds = p->rule_cond_off[p->set_rule_off[p->n_sets]];
  memset(dcoef, 0, sizeof(double) * (size_t)n_conds);
  memset(dcoef2, 0, sizeof(double) * (size_t)n_conds);
  memset(dtheta, 0, sizeof(double) * (size_t)n_conds);
  int32_t max_r = 0;
  for (int32_t s = 0; s < p->n_sets; ++s) {
    int32_t r = p->set_rule_off[s + 1] - p->set_rule_off[s];
    if (r > max_r) max_r = r;
  }
  const int nt = pick_threads(nthreads);
  (void)nt;
  int bad = 0;
#pragma omp parallel num_threads(nt)
  {
    double *r = (double *)malloc(sizeof(double) * (size_t)(max_r + 1));
    double v[MAX_CLASSES], lp[MAX_CLASSES], g[MAX_CLASSES];
    if (!r) {
#pragma omp atomic write
      bad = 1;
    }
#pragma omp for schedule(static)
    for (int32_t s = 0; s < p->n_sets; ++s) {
      if (!r) continue;
      int32_t k0 = p->set_rule_off[s], R = p->set_rule_off[s + 1] - k0;
      double scale = n > 0 ? dloss[s] / (double)n : 0.0;
      for (int64_t i = 0; i < n; ++i) {
        const float *xr = x + i * nf;
        smax_votes(p, coef, coef2, theta, s, xr, tau, nc, v, r);
        smax_logp(v, nc, beta, lp);
        if (-lp[y[i]] > LOSS_CAP) continue;
        for (int c = 0; c < nc; ++c) g[c] = beta * (exp(lp[c]) - (c == y[i] ? 1.0 : 0.0));
        for (int32_t k = 0; k < R; ++k) {
          double others = 1.0;
          for (int32_t m = 0; m < R; ++m)
            if (m != k) others *= 1.0 - r[m];
          double dr = g[p->rule_class[k0 + k]] - g[p->set_default[s]] * others;
          if (dr == 0.0 || r[k] == 0.0) continue;
          int32_t kk = k0 + k;
          for (int32_t j = p->rule_cond_off[kk]; j < p->rule_cond_off[kk + 1]; ++j) {
            if (p->kind[j] == 2) continue; /* no parameters */
            double z = cond_z(p, coef, coef2, theta, j, xr, tau);
            double dz = dr * r[k] * exp(log_sigmoid(-z));
            int f = p->f[j];
            double st = cond_sign(p->op[j]) / (double)tau[f];
            dcoef[j] += scale * dz * st * (double)xr[f];
            double t2 = -scale * dz * st * (p->kind[j] == 1 ? (double)xr[p->g[j]] : 1.0);
            if (p->kind[j] == 1)
              dcoef2[j] += t2;
            else
              dtheta[j] += t2;
          }
        }
      }
    }
    free(r);
  }
  return bad ? -2 : 0;
}
