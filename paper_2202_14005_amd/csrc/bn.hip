// Batch normalisation of the denoiser's hidden layers (the MoDL
// subsection's conv + BN + ReLU), training-mode statistics over every pixel
// of the batch, on NHWC bf16 activations with 64 channels.  The layer's
// convolution runs twice: once summing y and y^2 per channel in fp32 from
// its accumulators (CONV_STATS), once writing the normalised value
// yhat = (y - mu) istd (CONV_NORM), so y itself is never rounded (y - mu
// would lose the bf16 rounding of y to cancellation when the mean is large
// against the spread).  Here:
//   forward:  mu, istd = 1 / sqrt(var + eps) from the sums (in double);
//             a = ReLU(gamma yhat + beta) rounded to bf16;
//   reverse:  with g_z the gradient after the ReLU derivative,
//             g_beta = sum g_z, g_gamma = sum g_z yhat,
//             g_y = gamma istd (g_z - sum g_z / N - yhat sum(g_z yhat) / N).
// Every sum is taken in a fixed order: per thread over its pixels, then per
// workgroup over its 32 pixel lanes, then over the workgroups in order.
#include "bn.h"

namespace mrx {

namespace {

constexpr int BN_TPB = 256;  // 32 pixel lanes x 8 chunks of 8 channels

__device__ __forceinline__ float bf2f(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }
__device__ __forceinline__ uint16_t f2bf_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// The pixel range of workgroup blk: [p0, p1).
__device__ __forceinline__ void bn_range(int64_t npix, int blk, int64_t& p0, int64_t& p1) {
  const int64_t per = (npix + BN_BLOCKS - 1) / BN_BLOCKS;
  p0 = (int64_t)blk * per;
  p1 = p0 + per < npix ? p0 + per : npix;
}

// The 32 pixel lanes' 8-channel sums v (per thread) into part[blk][64].
__device__ __forceinline__ void bn_block_store(const float (&v)[8], float* part) {
  __shared__ float red[32][CNN_F + 1];
  const int chunk = threadIdx.x & 7, pl = threadIdx.x >> 3;
#pragma unroll
  for (int e = 0; e < 8; ++e) red[pl][chunk * 8 + e] = v[e];
  __syncthreads();
  if (threadIdx.x < CNN_F) {
    float s = 0.f;
    for (int i = 0; i < 32; ++i) s += red[i][threadIdx.x];
    part[(int64_t)blockIdx.x * CNN_F + threadIdx.x] = s;
  }
}

// sum over the workgroup's pixels of g_z yhat (both bf16), per channel
__global__ void __launch_bounds__(BN_TPB) k_bn_gyhat(const uint16_t* yhat, const uint16_t* g, int64_t npix,
                                                    float* part) {
  int64_t p0, p1;
  bn_range(npix, blockIdx.x, p0, p1);
  const int chunk = threadIdx.x & 7, pl = threadIdx.x >> 3;
  float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int64_t p = p0 + pl; p < p1; p += 32) {
    const uint4 raw = *(const uint4*)(yhat + p * CNN_F + chunk * 8);
    const uint4 graw = *(const uint4*)(g + p * CNN_F + chunk * 8);
    const uint16_t* h = (const uint16_t*)&raw;
    const uint16_t* gh = (const uint16_t*)&graw;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] += bf2f(gh[e]) * bf2f(h[e]);
  }
  bn_block_store(v, part);
}

// mean and 1 / sqrt(var + eps) per channel from the convolution's
// per-workgroup sums of y and y^2 (fp32 slots, added in order in double)
__global__ void __launch_bounds__(CNN_F) k_bn_finish_stats(const float* slots, int nslots, int64_t npix,
                                                          float* stats) {
  const int c = threadIdx.x;
  double s1 = 0.0, s2 = 0.0;
  for (int k = 0; k < nslots; ++k) {
    s1 += (double)slots[(int64_t)k * 2 * CNN_F + c];
    s2 += (double)slots[(int64_t)k * 2 * CNN_F + CNN_F + c];
  }
  const double mean = s1 / (double)npix;
  double var = s2 / (double)npix - mean * mean;
  if (var < 0.0) var = 0.0;
  stats[BN_MEAN + c] = (float)mean;
  stats[BN_ISTD + c] = (float)(1.0 / sqrt(var + (double)BN_EPS));
}

// sum g_z yhat over the workgroup partials (fixed order): kept for the
// apply pass; g_gamma (+)=
__global__ void __launch_bounds__(CNN_F) k_bn_finish_sgy(const float* part, float* stats, float* g_gamma,
                                                        int accumulate) {
  const int c = threadIdx.x;
  float s = 0.f;
  for (int b = 0; b < BN_BLOCKS; ++b) s += part[(int64_t)b * CNN_F + c];
  stats[BN_SGY + c] = s;
  if (g_gamma) g_gamma[c] = accumulate ? g_gamma[c] + s : s;
}

// forward: out = ReLU(gamma yhat + beta) rounded to bf16; reverse (in place
// on out = g_z): g_y = gamma istd (g_z - sgz / N - yhat sgy / N)
__global__ void __launch_bounds__(BN_TPB) k_bn_apply(const uint16_t* yhat, uint16_t* out, int64_t npix,
                                                    const float* stats, const float* gamma, const float* beta,
                                                    int reverse) {
  const int64_t q = (int64_t)blockIdx.x * BN_TPB + threadIdx.x;  // chunk index
  if (q >= npix * 8) return;
  const int chunk = (int)(q & 7);
  const uint4 raw = *(const uint4*)(yhat + q * 8);
  const uint16_t* h = (const uint16_t*)&raw;
  uint4 res;
  uint16_t* r = (uint16_t*)&res;
  if (!reverse) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = chunk * 8 + e;
      const float z = gamma[c] * bf2f(h[e]) + beta[c];
      r[e] = f2bf_rne(z > 0.f ? z : 0.f);
    }
  } else {
    const uint4 graw = *(const uint4*)(out + q * 8);
    const uint16_t* gh = (const uint16_t*)&graw;
    const float inv_n = 1.0f / (float)npix;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = chunk * 8 + e;
      const float gy = gamma[c] * stats[BN_ISTD + c] *
                       (bf2f(gh[e]) - stats[BN_SGZ + c] * inv_n - bf2f(h[e]) * stats[BN_SGY + c] * inv_n);
      r[e] = f2bf_rne(gy);
    }
  }
  *(uint4*)(out + q * 8) = res;
}

// stats[BN_SGZ] = sgz; g_beta (+)= sgz
__global__ void k_bn_take_sgz(const float* sgz, float* stats, float* g_beta, int accumulate) {
  const int c = threadIdx.x;
  if (c >= CNN_F) return;
  stats[BN_SGZ + c] = sgz[c];
  if (g_beta) g_beta[c] = accumulate ? g_beta[c] + sgz[c] : sgz[c];
}

}  // namespace

hipError_t bn_finish_stats(const float* slots, int nslots, int64_t npix, float* stats, hipStream_t s) {
  hipLaunchKernelGGL(k_bn_finish_stats, dim3(1), dim3(CNN_F), 0, s, slots, nslots, npix, stats);
  return hipGetLastError();
}

hipError_t bn_apply_forward(const uint16_t* yhat, uint16_t* a, int64_t npix, const float* gamma, const float* beta,
                            const float* stats, hipStream_t s) {
  const int64_t chunks = npix * 8;
  hipLaunchKernelGGL(k_bn_apply, dim3((unsigned)((chunks + BN_TPB - 1) / BN_TPB)), dim3(BN_TPB), 0, s, yhat, a,
                     npix, stats, gamma, beta, 0);
  return hipGetLastError();
}

hipError_t bn_backward(const uint16_t* yhat, uint16_t* g, int64_t npix, const float* gamma, float* stats,
                       const float* sgz, float* part, float* g_gamma, float* g_beta, int accumulate,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_bn_take_sgz, dim3(1), dim3(CNN_F), 0, s, sgz, stats, g_beta, accumulate);
  hipLaunchKernelGGL(k_bn_gyhat, dim3(BN_BLOCKS), dim3(BN_TPB), 0, s, yhat, g, npix, part);
  hipLaunchKernelGGL(k_bn_finish_sgy, dim3(1), dim3(CNN_F), 0, s, part, stats, g_gamma, accumulate);
  const int64_t chunks = npix * 8;
  hipLaunchKernelGGL(k_bn_apply, dim3((unsigned)((chunks + BN_TPB - 1) / BN_TPB)), dim3(BN_TPB), 0, s, yhat, g,
                     npix, stats, gamma, gamma, 1);
  return hipGetLastError();
}

}  // namespace mrx
