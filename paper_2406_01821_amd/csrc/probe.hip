// Issue-rate probe: how many lane-operations per second the VALU sustains
// for fp32 multiplies and for the transcendentals (v_exp_f32, v_log_f32)
// the soft path is built on, so that a roofline can weight transcendental
// instructions by a measured cost instead of an assumed one.
//
// Each thread runs 8 independent dependency chains (enough in flight to
// cover the VALU latency) for `iters` rounds; every round issues 16
// instructions of the probed class per thread.  The chains start from
// values read from memory and their sums are written out, so nothing is
// folded away; values stay in [-1, 0] (transcendental chain x -> 2^x in
// [0.5, 1], then log2) or unchanged (multiplies by 1.0 read from memory).
#include "internal.h"

namespace aerl {

namespace {

constexpr int kProbeBlock = 256;
constexpr int kProbeChains = 8;

template <bool TRANS>
__global__ __launch_bounds__(kProbeBlock) void k_probe(const float *__restrict__ in,
                                                       float *__restrict__ out, int iters) {
  float a[kProbeChains];
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) a[k] = in[(threadIdx.x + 37 * k) % kProbeBlock];
  const float one = in[kProbeBlock];
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) {
      if constexpr (TRANS) {
        a[k] = __builtin_amdgcn_exp2f(a[k]);
        a[k] = __builtin_amdgcn_logf(a[k]);
      } else {
        a[k] = a[k] * one;
        a[k] = a[k] * one;
      }
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) s += a[k];
  out[(int64_t)blockIdx.x * kProbeBlock + threadIdx.x] = s;
}

}  // namespace

}  // namespace aerl

extern "C" aerl_status aerl_probe_valu_rates(aerl_ctx *ctx, double *out, hipStream_t stream) {
  using namespace aerl;
  if (!ctx || !out) return AERL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->err.clear();
  AERL_HIP(ctx, hipSetDevice(ctx->device));
  // 16 blocks of 256 threads per CU: four waves per SIMD, each with eight
  // independent chains
  const int blocks = 16 * std::max(ctx->n_cu, 1);
  const int iters = 2048;
  float *buf = nullptr;
  const size_t in_floats = kProbeBlock + 1, out_floats = (size_t)blocks * kProbeBlock;
  AERL_HIP(ctx, hipMalloc(&buf, (in_floats + out_floats) * sizeof(float)));
  struct Free {
    float *p;
    ~Free() { (void)hipFree(p); }
  } guard{buf};
  float host[kProbeBlock + 1];
  for (int i = 0; i < kProbeBlock; ++i) host[i] = -(float)i / kProbeBlock;
  host[kProbeBlock] = 1.0f;
  AERL_HIP(ctx, hipMemcpyAsync(buf, host, sizeof(host), hipMemcpyHostToDevice, stream));
  AERL_HIP(ctx, hipStreamSynchronize(stream));  // host[] is on this frame
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  struct Ev {
    hipEvent_t *e;
    ~Ev() {
      for (int i = 0; i < 3; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } evg{ev};
  for (auto &e : ev) AERL_HIP(ctx, hipEventCreate(&e));
  // one untimed launch of each, then the timed pair
  hipLaunchKernelGGL(k_probe<false>, dim3(blocks), dim3(kProbeBlock), 0, stream, buf,
                     buf + in_floats, iters);
  hipLaunchKernelGGL(k_probe<true>, dim3(blocks), dim3(kProbeBlock), 0, stream, buf,
                     buf + in_floats, iters);
  AERL_HIP(ctx, hipEventRecord(ev[0], stream));
  hipLaunchKernelGGL(k_probe<false>, dim3(blocks), dim3(kProbeBlock), 0, stream, buf,
                     buf + in_floats, iters);
  AERL_HIP(ctx, hipEventRecord(ev[1], stream));
  hipLaunchKernelGGL(k_probe<true>, dim3(blocks), dim3(kProbeBlock), 0, stream, buf,
                     buf + in_floats, iters);
  AERL_HIP(ctx, hipEventRecord(ev[2], stream));
  AERL_HIP(ctx, hipGetLastError());
  AERL_HIP(ctx, hipEventSynchronize(ev[2]));
  float ms_mul = 0.0f, ms_trans = 0.0f;
  AERL_HIP(ctx, hipEventElapsedTime(&ms_mul, ev[0], ev[1]));
  AERL_HIP(ctx, hipEventElapsedTime(&ms_trans, ev[1], ev[2]));
  const double lane_ops = (double)blocks * kProbeBlock * iters * (2.0 * kProbeChains);
  out[0] = lane_ops / (ms_mul * 1e-3);
  out[1] = lane_ops / (ms_trans * 1e-3);
  return AERL_OK;
}
