// iPALM, the training algorithm the paper names for VarNet (Iterative
// Training Algorithms; Variational Network subsection): inertial
// extrapolation, a gradient step at the extrapolated point and a proximal
// step, here the projection onto the original VarNet's constraints (filters
// of zero mean and unit norm, non-negative step sizes); and the data
// normalisation max|x^0| = 1 of the VarNet training option.  Reductions run
// in a fixed order (deterministic).
#include "../../include/mrx.h"
#include "api_internal.h"

namespace mrx {

__global__ void k_ipalm_extrapolate(const float* th, const float* prev, float* y, int64_t n, float alpha) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = __builtin_fmaf(alpha, th[i] - prev[i], th[i]);
}

__global__ void k_ipalm_update(float* th, float* prev, const float* y, const float* g, int64_t n, float tau) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    prev[i] = th[i];
    th[i] = __builtin_fmaf(-tau, g[i], y[i]);
  }
}

constexpr int PRJ_THREADS = 256;

// Fixed-order block sum of two values per thread (the 4 wavefronts' sums
// added in order).
__device__ __forceinline__ float2 prj_sum2(float a, float b, float2* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  __syncthreads();
  if (lane == 0) red[wv] = make_float2(a, b);
  __syncthreads();
  float2 s = red[0];
#pragma unroll
  for (int w = 1; w < PRJ_THREADS / 64; ++w) s = make_float2(s.x + red[w].x, s.y + red[w].y);
  return s;
}

// One workgroup per complex filter of `taps` taps (taps <= PRJ_THREADS):
// subtract the mean, scale to unit Euclidean norm (a filter that is zero
// after removing its mean stays zero).
__global__ void __launch_bounds__(PRJ_THREADS) k_vn_project_filters(float2* k, int taps) {
  __shared__ float2 red[PRJ_THREADS / 64];
  float2* f = k + (int64_t)blockIdx.x * taps;
  const int t = threadIdx.x;
  const float2 v = t < taps ? f[t] : make_float2(0.f, 0.f);
  const float2 s = prj_sum2(v.x, v.y, red);
  const float2 u = make_float2(v.x - s.x / taps, v.y - s.y / taps);
  const float2 nn = prj_sum2(t < taps ? u.x * u.x + u.y * u.y : 0.f, 0.f, red);
  const float inv = nn.x > 0.f ? 1.0f / sqrtf(nn.x) : 0.f;
  if (t < taps) f[t] = make_float2(u.x * inv, u.y * inv);
}

__global__ void k_clamp_nonneg(float* a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = fmaxf(a[i], 0.f);
}

// Per-slice max |x|: block partial maxima of CG_EPB-pixel blocks (part
// [B][nblk]), then one value per slice (max is exact, so order is free).
__global__ void __launch_bounds__(256) k_slice_absmax(const SliceDesc* desc, const float2* x, float* part, int nblk) {
  __shared__ float red[4];
  const int b = blockIdx.y;
  const SliceDesc d = desc[b];
  const int64_t n = (int64_t)d.H * d.W;
  float m = 0.f;
  const int64_t base = (int64_t)blockIdx.x * CG_EPB;
  for (int k = threadIdx.x; k < CG_EPB; k += 256) {
    const int64_t i = base + k;
    if (i >= n) break;
    const float2 v = x[d.xoff + i];
    m = fmaxf(m, sqrtf(v.x * v.x + v.y * v.y));
  }
  for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)b * nblk + blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

__global__ void k_slice_scale_factor(const float* part, int nblk, int B, float* scale) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float m = 0.f;
  for (int i = 0; i < nblk; ++i) m = fmaxf(m, part[(int64_t)b * nblk + i]);
  scale[b] = m > 0.f ? 1.0f / m : 1.0f;
}

// x_b (image sized), y_b (coil sized) and ref_b (image sized) *= scale[b].
__global__ void k_slice_scale(const SliceDesc* desc, const float* scale, float2* x, float2* y, float2* ref) {
  const int b = blockIdx.y;
  const SliceDesc d = desc[b];
  const int64_t n = (int64_t)d.H * d.W, nc = n * d.C;
  const float s = scale[b];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += (int64_t)gridDim.x * blockDim.x) {
    if (i < n) {
      if (x) x[d.xoff + i] = cscale(x[d.xoff + i], s);
      if (ref) ref[d.xoff + i] = cscale(ref[d.xoff + i], s);
    }
    if (y) y[d.soff + i] = cscale(y[d.soff + i], s);
  }
}

}  // namespace mrx

using namespace mrx;

extern "C" {

mrx_status mrx_ipalm_extrapolate(const float* theta, const float* theta_prev, float* y, int64_t n, float alpha,
                                 void* stream) {
  if (!theta || !theta_prev || !y) return fail(MRX_EINVAL, "ipalm_extrapolate: null pointer");
  if (n < 0) return fail(MRX_EINVAL, "ipalm_extrapolate: negative size");
  if (n == 0) return MRX_OK;
  hipLaunchKernelGGL(k_ipalm_extrapolate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     theta, theta_prev, y, n, alpha);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MRX_OK : hip_fail(e, "ipalm_extrapolate");
}

mrx_status mrx_ipalm_update(float* theta, float* theta_prev, const float* y, const float* g, int64_t n, float tau,
                            void* stream) {
  if (!theta || !theta_prev || !y || !g) return fail(MRX_EINVAL, "ipalm_update: null pointer");
  if (n < 0) return fail(MRX_EINVAL, "ipalm_update: negative size");
  if (n == 0) return MRX_OK;
  hipLaunchKernelGGL(k_ipalm_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, theta,
                     theta_prev, y, g, n, tau);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MRX_OK : hip_fail(e, "ipalm_update");
}

mrx_status mrx_vn_project(float* k, int32_t n_filters, int32_t taps, float* lam, int32_t n_lam, void* stream) {
  if ((n_filters > 0 && !k) || (n_lam > 0 && !lam)) return fail(MRX_EINVAL, "vn_project: null pointer");
  if (n_filters < 0 || n_lam < 0 || taps < 1 || taps > PRJ_THREADS)
    return fail(MRX_EINVAL, "vn_project: counts out of range (taps must be in [1, 256])");
  hipStream_t s = (hipStream_t)stream;
  if (n_filters > 0) hipLaunchKernelGGL(k_vn_project_filters, dim3(n_filters), dim3(PRJ_THREADS), 0, s, (float2*)k, taps);
  if (n_lam > 0) hipLaunchKernelGGL(k_clamp_nonneg, dim3((n_lam + 255) / 256), dim3(256), 0, s, lam, n_lam);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MRX_OK : hip_fail(e, "vn_project");
}

mrx_status mrx_normalize_max(mrx_plan p, float* x, float* y, float* ref, float* scale_out, void* stream) {
  if (!p) return fail(MRX_EINVAL, "normalize_max: null plan");
  if (!x || !scale_out) return fail(MRX_EINVAL, "normalize_max: null data pointer");
  if (!p->ws) return fail(MRX_ENOWORKSPACE, "normalize_max: workspace not set");
  hipStream_t s = (hipStream_t)stream;
  float* part = (float*)(p->ws + p->ws_part);  // B x nrr floats
  const int nblk = (int)((p->maxHW + CG_EPB - 1) / CG_EPB);
  hipLaunchKernelGGL(k_slice_absmax, dim3(nblk, p->B), dim3(256), 0, s, p->d_desc, (const float2*)x, part, nblk);
  hipLaunchKernelGGL(k_slice_scale_factor, dim3((p->B + 255) / 256), dim3(256), 0, s, part, nblk, p->B, scale_out);
  hipLaunchKernelGGL(k_slice_scale, dim3(64, p->B), dim3(256), 0, s, p->d_desc, scale_out, (float2*)x, (float2*)y,
                     (float2*)ref);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MRX_OK : hip_fail(e, "normalize_max");
}

}  // extern "C"
