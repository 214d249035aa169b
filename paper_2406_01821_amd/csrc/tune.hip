// On-device fine-tuning of a population's coefficients and thresholds.
//
// Section 3: back-propagation through the sigmoid relaxation adjusts the
// coefficients of every rule without changing its logical structure; the
// paper applies 50 epochs of gradient updates to each candidate rule set
// (Section 4.1, the fine-tuning example of Fig. 1).  Every rule set is its
// own model: the gradient of sum_s loss[s] with respect to a condition's
// parameters is the gradient of its own rule set's loss.  One epoch here is
// one full-batch step: the adjoint over the whole resident dataset, then a
// fused optimizer update of every parameter in place.  The parameters of a
// condition are its coefficient, plus its threshold (threshold condition)
// or its second coefficient (feature-vs-feature condition); the unused one
// of the two is never written, so the structure stays exactly as packed.
#include "internal.h"

namespace aerl {

namespace {

constexpr int kTuneBlock = 256;

// Adam with bias correction (c1 = 1/(1 - beta1^t), c2 = 1/(1 - beta2^t)):
//   m = b1*m + (1-b1)*g;  v = b2*v + (1-b2)*g^2;
//   p -= lr * (m*c1) / (sqrt(v*c2) + eps)
// on (coef, rhs) of each condition, rhs = theta or coef2 by kind.
__global__ __launch_bounds__(kTuneBlock) void k_adam_step(
    const uint32_t *__restrict__ sconds, int32_t n_conds, float *__restrict__ coef,
    float *__restrict__ coef2, float *__restrict__ theta, const float *__restrict__ dcoef,
    const float *__restrict__ dcoef2, const float *__restrict__ dtheta, float *__restrict__ m,
    float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_conds) return;
  if (sconds[j] & kSoftCat) return;  // a code set: nothing to tune
  const bool ff = (sconds[j] & kSoftFF) != 0;
  float *rhs = ff ? coef2 : theta;
  const float g[2] = {dcoef[j], ff ? dcoef2[j] : dtheta[j]};
  float *p[2] = {coef + j, rhs + j};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int64_t i = (int64_t)k * n_conds + j;
    const float mk = b1 * m[i] + (1.0f - b1) * g[k];
    const float vk = b2 * v[i] + (1.0f - b2) * (g[k] * g[k]);
    m[i] = mk;
    v[i] = vk;
    *p[k] -= lr * (mk * c1) / (sqrtf(vk * c2) + eps);
  }
}

// Plain gradient descent: p -= lr * g on the same parameters.
__global__ __launch_bounds__(kTuneBlock) void k_sgd_step(
    const uint32_t *__restrict__ sconds, int32_t n_conds, float *__restrict__ coef,
    float *__restrict__ coef2, float *__restrict__ theta, const float *__restrict__ dcoef,
    const float *__restrict__ dcoef2, const float *__restrict__ dtheta, float lr) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_conds) return;
  if (sconds[j] & kSoftCat) return;  // a code set: nothing to tune
  const bool ff = (sconds[j] & kSoftFF) != 0;
  coef[j] -= lr * dcoef[j];
  if (ff)
    coef2[j] -= lr * dcoef2[j];
  else
    theta[j] -= lr * dtheta[j];
}

__global__ void k_fill_f32(float *__restrict__ p, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t fill_f32(float *p, int64_t n, float v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace

TuneLayout tune_layout(const DatasetRec &ds, const PopRec &pop) {
  TuneLayout L{};
  const size_t nc = (size_t)std::max(pop.n_conds, 1);
  const size_t ns = (size_t)std::max(pop.n_sets, 1);
  size_t off = 0;
  L.soft_off = off;  off = align256(off + std::max(soft_ws_bytes(ds, pop, false), soft_ws_bytes(ds, pop, true)));
  L.grad_off = off;  off = align256(off + 3 * nc * sizeof(float));
  L.mom_off = off;   off = align256(off + 4 * nc * sizeof(float));
  L.dloss_off = off; off = align256(off + ns * sizeof(float));
  L.total = off;
  return L;
}

hipError_t run_finetune(const TuneLaunch &t, hipStream_t st) {
  const DatasetRec &ds = *t.ds;
  const PopRec &pop = *t.pop;
  const TuneLayout L = tune_layout(ds, pop);
  char *w = static_cast<char *>(t.ws);
  float *grad = reinterpret_cast<float *>(w + L.grad_off);
  float *mom = reinterpret_cast<float *>(w + L.mom_off);
  float *ones = reinterpret_cast<float *>(w + L.dloss_off);
  const int64_t nc = pop.n_conds;
  SoftLaunch s{};
  s.ds = &ds;
  s.pop = &pop;
  s.coef = t.coef;
  s.coef2 = t.coef2;
  s.theta = t.theta;
  s.ws = w + L.soft_off;
  s.ws_bytes = L.grad_off - L.soft_off;
  s.dloss = ones;
  s.dcoef = grad;
  s.dcoef2 = grad + nc;
  s.dtheta = grad + 2 * nc;
  hipError_t e = fill_f32(ones, pop.n_sets, 1.0f, st);
  if (e == hipSuccess) e = fill_f32(mom, 4 * nc, 0.0f, st);
  const unsigned blocks = (unsigned)((nc + kTuneBlock - 1) / kTuneBlock);
  double b1t = 1.0, b2t = 1.0;
  for (int32_t ep = 0; e == hipSuccess && ep <= t.epochs; ++ep) {
    if (t.loss_hist) {
      s.loss = t.loss_hist + (int64_t)ep * pop.n_sets;
      e = launch_soft_forward(s, st);
      if (e != hipSuccess) break;
    }
    if (ep == t.epochs || nc == 0) continue;
    e = launch_soft_backward(s, st);
    if (e != hipSuccess) break;
    if (t.optimizer == AERL_OPT_ADAM) {
      b1t *= (double)t.beta1;
      b2t *= (double)t.beta2;
      const float c1 = (float)(1.0 / (1.0 - b1t)), c2 = (float)(1.0 / (1.0 - b2t));
      hipLaunchKernelGGL(k_adam_step, dim3(blocks), dim3(kTuneBlock), 0, st, pop.sconds,
                         (int32_t)nc, t.coef, t.coef2, t.theta, s.dcoef, s.dcoef2, s.dtheta, mom,
                         mom + 2 * nc, t.lr, t.beta1, t.beta2, t.eps, c1, c2);
    } else {
      hipLaunchKernelGGL(k_sgd_step, dim3(blocks), dim3(kTuneBlock), 0, st, pop.sconds,
                         (int32_t)nc, t.coef, t.coef2, t.theta, s.dcoef, s.dcoef2, s.dtheta, t.lr);
    }
    e = hipGetLastError();
  }
  return e;
}

}  // namespace aerl
