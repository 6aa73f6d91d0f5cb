// The one-off steps of non-Cartesian SENSE that the Extensions to the
// SENSE-Model subsection precomputes for a whole dataset: the adjoint
// reconstruction A^H y and the point spread function of the trajectory;
// plus the forward model that simulates the k-space data.  All three are
// exact sums over the samples (the non-uniform DFT by its definition, no
// gridding), deterministic, with each phase formed in double precision and
// reduced to one turn before the single-precision sine and cosine.
//
// Conventions (as the header states): sample j of slice b is
// traj[(b M + j) 2 + {0, 1}] = (ky, kx) in cycles per field of view; pixel
// (r, s) sits at (r - H/2, s - W/2); y is [C][M] per slice, slices packed in
// order (offset M x the coils of the slices before).
#include <cmath>

#include "../../include/mrx.h"
#include "api_internal.h"

namespace mrx {

namespace {

constexpr int NU_TPB = 256;     // threads a workgroup
constexpr int NU_CHUNK = 256;   // samples / pixels staged a step
constexpr int NU_CG = 16;       // coils accumulated together

__device__ __forceinline__ int64_t coil_prefix(const SliceDesc* desc, int b) {
  int64_t c = 0;
  for (int i = 0; i < b; ++i) c += desc[i].C;
  return c;
}

// exp(sign 2 pi i t) for t given in turns (double), reduced to [-1/2, 1/2]
__device__ __forceinline__ float2 cis_turns(double t, float sign) {
  const float f = (float)(t - rint(t));
  float sn, cs;
  sincospif(2.0f * f, &sn, &cs);
  return make_float2(cs, sign * sn);
}

// x[pixel] = (HW)^{-1/2} sum_c conj(S_c) sum_j y_cj exp(+2 pi i phi_j(pixel))
__global__ void __launch_bounds__(NU_TPB) k_nudft_adj(const SliceDesc* desc, int M, const float* traj,
                                                     const float2* y, const float2* S, float2* x) {
  __shared__ float2 ky[NU_CHUNK];
  __shared__ float2 yy[NU_CG][NU_CHUNK];
  const int b = blockIdx.y;
  const SliceDesc d = desc[b];
  const int H = d.H, W = d.W;
  const int64_t npx = (int64_t)H * W;
  const int64_t pix = (int64_t)blockIdx.x * NU_TPB + threadIdx.x;
  if ((int64_t)blockIdx.x * NU_TPB >= npx) return;
  const bool valid = pix < npx;
  const int r = valid ? (int)(pix / W) : 0, s = valid ? (int)(pix % W) : 0;
  const double ry = (double)(r - H / 2) / H, sx = (double)(s - W / 2) / W;
  const float* tb = traj + (int64_t)b * M * 2;
  const float2* yb = y + coil_prefix(desc, b) * M;
  float2 out = make_float2(0.f, 0.f);
  for (int c0 = 0; c0 < d.C; c0 += NU_CG) {
    const int nc = min(NU_CG, d.C - c0);
    float2 u[NU_CG];
#pragma unroll
    for (int c = 0; c < NU_CG; ++c) u[c] = make_float2(0.f, 0.f);
    for (int j0 = 0; j0 < M; j0 += NU_CHUNK) {
      const int nj = min(NU_CHUNK, M - j0);
      __syncthreads();
      for (int i = threadIdx.x; i < nj; i += NU_TPB) ky[i] = make_float2(tb[2 * (j0 + i)], tb[2 * (j0 + i) + 1]);
      for (int i = threadIdx.x; i < NU_CG * NU_CHUNK; i += NU_TPB) {
        const int c = i / NU_CHUNK, j = i % NU_CHUNK;
        yy[c][j] = (c < nc && j < nj) ? yb[(int64_t)(c0 + c) * M + j0 + j] : make_float2(0.f, 0.f);
      }
      __syncthreads();
      for (int j = 0; j < nj; ++j) {
        const float2 k = ky[j];
        const float2 e = cis_turns((double)k.x * ry + (double)k.y * sx, 1.f);
#pragma unroll
        for (int c = 0; c < NU_CG; ++c) u[c] = cadd(u[c], cmul(yy[c][j], e));
      }
    }
    if (valid)
      for (int c = 0; c < nc; ++c) out = cadd(out, cmulc(S[d.soff + (int64_t)(c0 + c) * npx + pix], u[c]));
  }
  if (valid) x[d.xoff + pix] = cscale(out, rsqrtf((float)npx));
}

// y_cj = (HW)^{-1/2} sum_pixels S_c x exp(-2 pi i phi_j(pixel)) (+ noise)
__global__ void __launch_bounds__(NU_TPB) k_nudft_fwd(const SliceDesc* desc, int M, const float* traj,
                                                     const float2* x, const float2* S, const float2* noise,
                                                     float2* y) {
  __shared__ float2 sx_[NU_CG][NU_CHUNK];
  const int b = blockIdx.y;
  const SliceDesc d = desc[b];
  const int H = d.H, W = d.W;
  const int64_t npx = (int64_t)H * W;
  const int j = blockIdx.x * NU_TPB + threadIdx.x;
  if (blockIdx.x * NU_TPB >= M) return;
  const bool valid = j < M;
  const float* tb = traj + (int64_t)b * M * 2;
  const double ky = valid ? (double)tb[2 * j] : 0.0, kx = valid ? (double)tb[2 * j + 1] : 0.0;
  const int64_t yoff = coil_prefix(desc, b) * M;
  const float sc = rsqrtf((float)npx);
  for (int c0 = 0; c0 < d.C; c0 += NU_CG) {
    const int nc = min(NU_CG, d.C - c0);
    float2 u[NU_CG];
#pragma unroll
    for (int c = 0; c < NU_CG; ++c) u[c] = make_float2(0.f, 0.f);
    for (int64_t p0 = 0; p0 < npx; p0 += NU_CHUNK) {
      const int np = (int)min<int64_t>(NU_CHUNK, npx - p0);
      __syncthreads();
      for (int i = threadIdx.x; i < NU_CG * NU_CHUNK; i += NU_TPB) {
        const int c = i / NU_CHUNK, q = i % NU_CHUNK;
        sx_[c][q] = (c < nc && q < np)
                        ? cmul(S[d.soff + (int64_t)(c0 + c) * npx + p0 + q], x[d.xoff + p0 + q])
                        : make_float2(0.f, 0.f);
      }
      __syncthreads();
      for (int q = 0; q < np; ++q) {
        const int64_t pix = p0 + q;
        const int r = (int)(pix / W), s = (int)(pix % W);
        const float2 e = cis_turns(ky * ((double)(r - H / 2) / H) + kx * ((double)(s - W / 2) / W), -1.f);
#pragma unroll
        for (int c = 0; c < NU_CG; ++c) u[c] = cadd(u[c], cmul(sx_[c][q], e));
      }
    }
    if (valid)
      for (int c = 0; c < nc; ++c) {
        const int64_t o = yoff + (int64_t)(c0 + c) * M + j;
        float2 v = cscale(u[c], sc);
        if (noise) v = cadd(v, noise[o]);
        y[o] = v;
      }
  }
}

// Dirichlet kernel sum_{|d| < n} exp(2 pi i d u / n) = sin(pi a (2n - 1)) / sin(pi a),
// a = u / n (its limit 2n - 1 at integer a).
__device__ __forceinline__ double dirichlet(double u, int n) {
  const double a = u / n;
  if (a == rint(a)) return 2.0 * n - 1.0;
  return sinpi(a * (2.0 * n - 1.0)) / sinpi(a);
}

constexpr int PSF_T = 16;  // output tile PSF_T x PSF_T a workgroup
constexpr int PSF_J = 64;  // samples a step

// psf[ky][kx] (2H x 2W, ky, kx the cyclic frequency indices) =
//   (HW)^{-1} sum_j D_H(ky_j - ky / 2) D_W(kx_j - kx / 2),
// the 2-D DFT of the cyclically laid out point spread function, which
// separates per sample into two Dirichlet kernels.  Accumulated in double.
__global__ void __launch_bounds__(PSF_T * PSF_T) k_psf(const SliceDesc* desc, int M, const float* traj, float* psf) {
  __shared__ double dy[PSF_J][PSF_T];
  __shared__ double dx[PSF_J][PSF_T];
  const int b = blockIdx.z;
  const SliceDesc d = desc[b];
  const int H2 = 2 * d.H, W2 = 2 * d.W;
  const int ty0 = blockIdx.y * PSF_T, tx0 = blockIdx.x * PSF_T;
  if (ty0 >= H2 || tx0 >= W2) return;
  const int ly = threadIdx.x / PSF_T, lx = threadIdx.x % PSF_T;
  const float* tb = traj + (int64_t)b * M * 2;
  double acc = 0.0;
  for (int j0 = 0; j0 < M; j0 += PSF_J) {
    const int nj = min(PSF_J, M - j0);
    __syncthreads();
    for (int i = threadIdx.x; i < PSF_J * PSF_T; i += PSF_T * PSF_T) {
      const int j = i / PSF_T, k = i % PSF_T;
      double vy = 0.0, vx = 0.0;
      if (j < nj) {
        vy = dirichlet((double)tb[2 * (j0 + j)] - 0.5 * (ty0 + k), d.H);
        vx = dirichlet((double)tb[2 * (j0 + j) + 1] - 0.5 * (tx0 + k), d.W);
      }
      dy[j][k] = vy;
      dx[j][k] = vx;
    }
    __syncthreads();
    for (int j = 0; j < nj; ++j) acc = fma(dy[j][ly], dx[j][lx], acc);
  }
  const int ky = ty0 + ly, kx = tx0 + lx;
  if (ky < H2 && kx < W2) psf[4 * d.xoff + (int64_t)ky * W2 + kx] = (float)(acc / ((double)d.H * d.W));
}

mrx_status check_traj(mrx_plan p, int32_t M, const void* traj, const char* what) {
  if (!p) return fail(MRX_EINVAL, std::string(what) + ": null plan");
  if (!traj) return fail(MRX_EINVAL, std::string(what) + ": null trajectory");
  if (M <= 0 || M > (1 << 26)) return fail(MRX_EINVAL, std::string(what) + ": sample count must be in [1, 2^26]");
  return MRX_OK;
}

}  // namespace
}  // namespace mrx

using namespace mrx;

extern "C" {

mrx_status mrx_nufft_adj(mrx_plan p, const float* traj, int32_t M, const float* y, const float* S, float* x,
                         void* stream) {
  mrx_status st = check_traj(p, M, traj, "nufft_adj");
  if (st != MRX_OK) return st;
  if (!y || !S || !x) return fail(MRX_EINVAL, "nufft_adj: null data pointer");
  dim3 grid((unsigned)((p->maxHW + NU_TPB - 1) / NU_TPB), (unsigned)p->B);
  hipLaunchKernelGGL(k_nudft_adj, grid, dim3(NU_TPB), 0, (hipStream_t)stream, p->d_desc, (int)M, traj,
                     (const float2*)y, (const float2*)S, (float2*)x);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MRX_OK : hip_fail(e, "nufft_adj");
}

mrx_status mrx_nufft_fwd(mrx_plan p, const float* traj, int32_t M, const float* x, const float* S,
                         const float* noise, float* y, void* stream) {
  mrx_status st = check_traj(p, M, traj, "nufft_fwd");
  if (st != MRX_OK) return st;
  if (!x || !S || !y) return fail(MRX_EINVAL, "nufft_fwd: null data pointer");
  dim3 grid((unsigned)((M + NU_TPB - 1) / NU_TPB), (unsigned)p->B);
  hipLaunchKernelGGL(k_nudft_fwd, grid, dim3(NU_TPB), 0, (hipStream_t)stream, p->d_desc, (int)M, traj,
                     (const float2*)x, (const float2*)S, (const float2*)noise, (float2*)y);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MRX_OK : hip_fail(e, "nufft_fwd");
}

mrx_status mrx_toeplitz_psf(mrx_plan p, const float* traj, int32_t M, float* psf, void* stream) {
  mrx_status st = check_traj(p, M, traj, "toeplitz_psf");
  if (st != MRX_OK) return st;
  if (!psf) return fail(MRX_EINVAL, "toeplitz_psf: null output");
  dim3 grid((unsigned)((2 * p->maxW + PSF_T - 1) / PSF_T), (unsigned)((2 * p->maxH + PSF_T - 1) / PSF_T),
            (unsigned)p->B);
  hipLaunchKernelGGL(k_psf, grid, dim3(PSF_T * PSF_T), 0, (hipStream_t)stream, p->d_desc, (int)M, traj, psf);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MRX_OK : hip_fail(e, "toeplitz_psf");
}

}  // extern "C"
