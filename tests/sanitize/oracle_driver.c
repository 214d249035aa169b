/* Exercise of the C oracle for an AddressSanitizer + UndefinedBehaviorSanitizer
 * build: every entry point on a small random table and population of every
 * condition kind (empty rule sets and rules included).  Exits non-zero on
 * any unexpected status; the sanitizers abort on any finding. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
  int32_t n_sets;
  const int32_t *set_rule_off, *set_default, *rule_cond_off, *rule_class;
  const uint8_t *op, *kind;
  const int32_t *f, *g;
  const float *coef, *coef2, *theta;
  const uint64_t *cat_mask;
} orc_population;

int orc_hard_eval(int64_t, int32_t, const float *, const int32_t *, int32_t, const orc_population *,
                  int32_t *, int32_t *, int);
int orc_predict(int64_t, int32_t, const float *, const orc_population *, int32_t, int32_t *);
int orc_workcount(int64_t, const int64_t *, const int64_t *, int32_t, const float *,
                  const orc_population *, int64_t *, int64_t *, int);
int orc_tau(int64_t, int32_t, const float *, float *);
int orc_soft_forward(int64_t, int32_t, const float *, const int32_t *, const float *, int32_t,
                     const orc_population *, const double *, const double *, const double *, double *,
                     int);
int orc_soft_backward(int64_t, int32_t, const float *, const int32_t *, const float *, int32_t,
                      const orc_population *, const double *, const double *, const double *,
                      const double *, double *, double *, double *, int);
int orc_smax_forward(int64_t, int32_t, const float *, const int32_t *, const float *, int32_t,
                     const orc_population *, const double *, const double *, const double *, double,
                     double *, int);
int orc_smax_backward(int64_t, int32_t, const float *, const int32_t *, const float *, int32_t,
                      const orc_population *, const double *, const double *, const double *, double,
                      const double *, double *, double *, double *, int);
int orc_smax_probs(int64_t, int32_t, const float *, const float *, int32_t, const orc_population *,
                   const double *, const double *, const double *, int32_t, double, double *);

#define NS 40
#define NF 5
#define NC 3
#define N 300

static uint64_t st = 88172645463325252ull;
static uint64_t rnd(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return st; }
static int below(int n) { return (int)(rnd() % (uint64_t)n); }

int main(void) {
  static int32_t sro[NS + 1], sd[NS], rco[NS * 6 + 1], rc[NS * 6], f[NS * 30], g[NS * 30];
  static uint8_t op[NS * 30], kind[NS * 30];
  static float c1[NS * 30], c2[NS * 30], th[NS * 30], x[N * NF], tau[NF];
  static uint64_t mk[NS * 30];
  static int32_t y[N];
  int nr = 0, nk = 0;
  for (int s = 0; s < NS; ++s) {
    sro[s] = nr;
    sd[s] = below(NC);
    int R = below(6);
    for (int r = 0; r < R; ++r) {
      rco[nr] = nk;
      rc[nr++] = below(NC);
      int K = below(5);
      for (int k = 0; k < K; ++k) {
        kind[nk] = (uint8_t)below(3);
        op[nk] = (uint8_t)below(4);
        f[nk] = below(NF);
        g[nk] = (f[nk] + 1 + below(NF - 1)) % NF;
        c1[nk] = (float)below(1000) / 500.0f - 1.0f;
        c2[nk] = (float)below(1000) / 700.0f;
        th[nk] = (float)below(1000) / 200.0f;
        mk[nk] = rnd();
        ++nk;
      }
    }
  }
  sro[NS] = nr;
  rco[nr] = nk;
  for (int i = 0; i < N * NF; ++i) x[i] = (i % NF == NF - 1) ? (float)below(70) : (float)below(1000) / 100.0f;
  for (int i = 0; i < N; ++i) y[i] = below(NC);
  orc_population p = {NS, sro, sd, rco, rc, op, kind, f, g, c1, c2, th, mk};
  static int32_t correct[NS], conf[NS * NC * NC], pred[N];
  static double d1[NS * 30], d2[NS * 30], d3[NS * 30], dl[NS], loss[NS], probs[N * NC];
  for (int j = 0; j < nk; ++j) { d1[j] = c1[j]; d2[j] = c2[j]; d3[j] = th[j]; }
  for (int s = 0; s < NS; ++s) dl[s] = 1.0;
  int bad = 0;
  bad |= orc_hard_eval(N, NF, x, y, NC, &p, correct, conf, 0);
  bad |= orc_predict(N, NF, x, &p, NS - 1, pred);
  int64_t ptr[N / 64 + 2], idx[N], wt[NS], wf[NS];
  int nt = 0;
  for (int i = 0; i < N; ++i) idx[i] = i;
  for (int t = 0; t * 64 < N; ++t) ptr[nt++] = t * 64;
  ptr[nt] = N;
  bad |= orc_workcount(nt, ptr, idx, NF, x, &p, wt, wf, 0);
  bad |= orc_tau(N, NF, x, tau);
  bad |= orc_soft_forward(N, NF, x, y, tau, NC, &p, d1, d2, d3, loss, 0);
  static double g1[NS * 30], g2[NS * 30], g3[NS * 30];
  bad |= orc_soft_backward(N, NF, x, y, tau, NC, &p, d1, d2, d3, dl, g1, g2, g3, 0);
  bad |= orc_smax_forward(N, NF, x, y, tau, NC, &p, d1, d2, d3, 2.0, loss, 0);
  bad |= orc_smax_backward(N, NF, x, y, tau, NC, &p, d1, d2, d3, 2.0, dl, g1, g2, g3, 0);
  bad |= orc_smax_probs(N, NF, x, tau, NC, &p, d1, d2, d3, 0, 2.0, probs);
  if (bad) { fprintf(stderr, "an oracle call failed\n"); return 1; }
  printf("oracle driver: all calls returned 0\n");
  return 0;
}
