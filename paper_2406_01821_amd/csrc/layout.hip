// Dataset upload: validation, label grouping, feature-major transpose, tau.
//
// The resident layout stores the samples feature-major (x_fm[f][n_pad]) so
// that a wave reads one feature of 64..256 consecutive samples with one
// coalesced access.  Samples are stably grouped by label and every class
// region is padded to a multiple of AERL_TILE samples, so every tile holds a
// single label; fitness counts do not depend on the sample order (accuracy
// is a sum over samples, Section 1).
#include "internal.h"

namespace aerl {

namespace {

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

// Per block of kUploadBlock samples: flags non-finite features / bad labels
// and counts labels per class.
__global__ __launch_bounds__(kUploadBlock) void k_validate_count(
    const float *__restrict__ x, const int32_t *__restrict__ y, int64_t n, int32_t nf,
    int32_t nc, int32_t *__restrict__ block_counts, int32_t *__restrict__ flags) {
  __shared__ int32_t hist[AERL_MAX_CLASSES];
  const int t = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * kUploadBlock;
  const int64_t rows = min((int64_t)kUploadBlock, n - i0);
  if (t < AERL_MAX_CLASSES) hist[t] = 0;
  __syncthreads();
  int bad_x = 0;
  const int64_t total = rows * nf;
  const float *xb = x + i0 * nf;
  for (int64_t k = t; k < total; k += kUploadBlock) {
    float v = xb[k];
    if (!__builtin_isfinite(v)) bad_x = 1;
  }
  int bad_y = 0;
  if (t < rows) {
    int32_t c = y[i0 + t];
    if (c < 0 || c >= nc) bad_y = 1;
    else atomicAdd(&hist[c], 1);
  }
  if (bad_x) atomicOr(&flags[0], 1);
  if (bad_y) atomicOr(&flags[1], 1);
  __syncthreads();
  if (t < nc) block_counts[(int64_t)blockIdx.x * nc + t] = hist[t];
}

// Stable scatter of a block's samples to their label-grouped slots and
// transpose into x_fm.  block_base[b][c] is the first slot of class c for
// block b.  The rank of a sample among its class inside the block comes from
// per-wave ballots, so the order inside each class is the original order.
constexpr int kChunkF = 32;
__global__ __launch_bounds__(kUploadBlock) void k_scatter_transpose(
    const float *__restrict__ x, const int32_t *__restrict__ y, int64_t n, int32_t nf,
    int32_t nc, const int32_t *__restrict__ block_base, float *__restrict__ x_fm,
    int32_t *__restrict__ y_pad, int32_t *__restrict__ perm, int64_t n_pad) {
  constexpr int kWaves = kUploadBlock / 64;
  __shared__ int32_t wave_count[kWaves][AERL_MAX_CLASSES];
  __shared__ float tile[kUploadBlock][kChunkF + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * kUploadBlock;
  const int64_t rows = min((int64_t)kUploadBlock, n - i0);
  const bool valid = t < rows;
  const int32_t c_me = valid ? y[i0 + t] : -1;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int32_t rank = 0;
  for (int c = 0; c < nc; ++c) {
    uint64_t m = __builtin_amdgcn_ballot_w64(c_me == c);
    if (c_me == c) rank = __builtin_popcountll(m & below);
    if (lane == 0) wave_count[w][c] = __builtin_popcountll(m);
  }
  __syncthreads();
  int64_t dest = -1;
  if (valid) {
    int32_t before = 0;
    for (int ww = 0; ww < w; ++ww) before += wave_count[ww][c_me];
    dest = (int64_t)block_base[(int64_t)blockIdx.x * nc + c_me] + before + rank;
    y_pad[dest] = c_me;
    perm[dest] = (int32_t)(i0 + t);
  }
  for (int f0 = 0; f0 < nf; f0 += kChunkF) {
    const int fc = min(kChunkF, nf - f0);
    __syncthreads();
    for (int k = t; k < kUploadBlock * kChunkF; k += kUploadBlock) {
      int r = k / kChunkF, ff = k % kChunkF;
      if (r < rows && ff < fc) tile[r][ff] = x[(i0 + r) * nf + f0 + ff];
    }
    __syncthreads();
    if (valid)
      for (int ff = 0; ff < fc; ++ff) x_fm[(int64_t)(f0 + ff) * n_pad + dest] = tile[t][ff];
  }
}

// tau[f] = 0.05 * population std over the real samples (1 if the std is 0),
// fp64 two-pass, rounded to float.  Each pass splits every feature row into
// kTauParts slices of whole layout tiles, one 256-thread block per (slice,
// feature); a sample counts when its tile's valid count says it is real
// (the tile table, not a per-sample label read).  Block sums use a fixed
// tree and the slice partials are added in slice order, so tau is the same
// from run to run.  Pass 1 writes the slices' sums, pass 2 the slices' sums
// of squared deviations from the mean (which every block forms from the
// pass-1 partials in the same order), and the last kernel finishes tau.
constexpr int kTauBlock = 256;

__device__ __forceinline__ double block_sum(double v, double *red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int h = kTauBlock / 2; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

__device__ __forceinline__ double tau_mean(const double *__restrict__ part, int f, int64_t n) {
  double s = 0.0;
  for (int b = 0; b < kTauParts; ++b) s += part[(int64_t)f * kTauParts + b];
  return n > 0 ? s / (double)n : 0.0;
}

// PASS 1: part1[f][b] = sum of the slice's real x; PASS 2: part2[f][b] = sum
// of (x - mean)^2.
template <int PASS>
__global__ __launch_bounds__(kTauBlock) void k_tau_part(const float *__restrict__ x_fm,
                                                        const int32_t *__restrict__ tile_info,
                                                        int64_t n_pad, int64_t n,
                                                        double *__restrict__ part1,
                                                        double *__restrict__ part2) {
  __shared__ double red[kTauBlock];
  const int f = blockIdx.y, b = blockIdx.x;
  const int64_t tiles = n_pad / AERL_TILE;
  const int64_t t0 = tiles * b / kTauParts, t1 = tiles * (b + 1) / kTauParts;
  const float *row = x_fm + (int64_t)f * n_pad;
  const double mean = PASS == 2 ? tau_mean(part1, f, n) : 0.0;
  double s = 0.0;
  for (int64_t t = t0; t < t1; ++t) {
    const int valid = tile_info[t] >> 8;
    const int i = threadIdx.x;  // one sample of the tile per thread
    if (i < valid) {
      const double v = (double)row[t * AERL_TILE + i];
      s += PASS == 1 ? v : (v - mean) * (v - mean);
    }
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) (PASS == 1 ? part1 : part2)[(int64_t)f * kTauParts + b] = s;
}

__global__ void k_tau_final(const double *__restrict__ part2, int32_t nf, int64_t n,
                            float *__restrict__ tau) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  double q = 0.0;
  for (int b = 0; b < kTauParts; ++b) q += part2[(int64_t)f * kTauParts + b];
  const double sd = n > 0 ? sqrt(q / (double)n) : 0.0;
  const float tf = sd > 0.0 ? (float)(0.05 * sd) : 1.0f;
  tau[f] = tf;
  tau[nf + f] = (float)(1.0 / (double)tf);  // 1/tau follows tau
}

}  // namespace

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_validate_count(const float *x, const int32_t *y, int64_t n, int32_t nf,
                                 int32_t nc, int32_t *block_counts, int32_t *flags,
                                 int64_t n_blocks, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate_count, dim3((unsigned)n_blocks), dim3(kUploadBlock), 0, s, x, y,
                     n, nf, nc, block_counts, flags);
  return hipGetLastError();
}

hipError_t launch_scatter_transpose(const float *x, const int32_t *y, int64_t n, int32_t nf,
                                    int32_t nc, const int32_t *block_base, float *x_fm,
                                    int32_t *y_pad, int32_t *perm, int64_t n_pad,
                                    int64_t n_blocks, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_transpose, dim3((unsigned)n_blocks), dim3(kUploadBlock), 0, s, x,
                     y, n, nf, nc, block_base, x_fm, y_pad, perm, n_pad);
  return hipGetLastError();
}

hipError_t launch_tau(const float *x_fm, const int32_t *tile_info, int64_t n_pad, int32_t nf,
                      int64_t n, double *part, float *tau, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  double *part1 = part, *part2 = part + (int64_t)nf * kTauParts;
  const dim3 grid(kTauParts, (unsigned)nf);
  hipLaunchKernelGGL(k_tau_part<1>, grid, dim3(kTauBlock), 0, s, x_fm, tile_info, n_pad, n, part1,
                     part2);
  hipLaunchKernelGGL(k_tau_part<2>, grid, dim3(kTauBlock), 0, s, x_fm, tile_info, n_pad, n, part1,
                     part2);
  hipLaunchKernelGGL(k_tau_final, dim3((unsigned)((nf + 63) / 64)), dim3(64), 0, s, part2, nf, n,
                     tau);
  return hipGetLastError();
}

}  // namespace aerl
