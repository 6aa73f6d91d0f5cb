// Fallback and judge: per slice, keep the network result unless it is not
// finite, a status bit was raised while computing it, or its data-consistency
// residual ||A^H A x - A^H y|| exceeds `ratio` times the residual of the plain
// Tikhonov CG-SENSE solution; otherwise take the CG-SENSE result and raise
// the judge bit.  Deterministic fixed-order reductions.
#include "../../include/mrx.h"
#include "api_internal.h"

namespace mrx {

// per (slice, block) partials of ||q - aHy||^2 and, when `bad_part` is given,
// the count of non-finite entries of x
__global__ void __launch_bounds__(CG_THREADS) k_dc_resid(const SliceDesc* desc, const int* slices, const float2* q,
                                                         const float2* aHy, const float2* x, float* part,
                                                         float* bad_part, int nrr) {
  __shared__ float red[CG_THREADS / 64];
  __shared__ float redn[CG_THREADS / 64];
  const int b = slices[blockIdx.y];
  const SliceDesc d = desc[b];
  const int64_t n = (int64_t)d.H * d.W;
  float acc = 0.f, bad = 0.f;
  const int64_t base = (int64_t)blockIdx.x * CG_EPB;
  for (int k = threadIdx.x; k < CG_EPB; k += CG_THREADS) {
    const int64_t i = base + k;
    if (i >= n) break;
    const int64_t o = d.xoff + i;
    const float2 a = q[o], y = aHy[o], xv = x[o];
    const float dx = a.x - y.x, dy = a.y - y.y;
    acc += dx * dx + dy * dy;
    if (!isfinite(xv.x) || !isfinite(xv.y)) bad += 1.f;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int off = 32; off >= 1; off >>= 1) {
    acc += __shfl_xor(acc, off, 64);
    bad += __shfl_xor(bad, off, 64);
  }
  if (lane == 0) { red[wv] = acc; redn[wv] = bad; }
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f, t = 0.f;
    for (int i = 0; i < CG_THREADS / 64; ++i) { s += red[i]; t += redn[i]; }
    part[(int64_t)b * nrr + blockIdx.x] = s;
    if (bad_part) bad_part[(int64_t)b * nrr + blockIdx.x] = t;
  }
}

// choice[b] = 1 when the fallback is taken
__global__ void k_dc_decide(const SliceDesc* desc, const float* pc, const float* pn, const float* pf, int nrr,
                            int B, float ratio, uint32_t* status, uint32_t* choice) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int nb = (int)(((int64_t)desc[b].H * desc[b].W + CG_EPB - 1) / CG_EPB);
  float rc = 0.f, nc = 0.f, rf = 0.f;
  for (int i = 0; i < nb; ++i) {
    rc += pc[(int64_t)b * nrr + i];
    nc += pn[(int64_t)b * nrr + i];
    rf += pf[(int64_t)b * nrr + i];
  }
  const uint32_t st = status[b];
  const bool take = nc > 0.f || !isfinite(rc) || (st & (FLAG_NONFINITE | FLAG_CG_BREAKDOWN | FLAG_CNN_NONFINITE)) ||
                    sqrtf(rc) > ratio * sqrtf(rf);
  if (take) status[b] = st | FLAG_DC_JUDGE;
  choice[b] = take ? 1u : 0u;
}

__global__ void k_dc_select(const SliceDesc* desc, const float2* xc, const float2* xf, const uint32_t* choice,
                            float2* out) {
  const int b = blockIdx.y;
  const SliceDesc d = desc[b];
  const int64_t n = (int64_t)d.H * d.W;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[d.xoff + i] = choice[b] ? xf[d.xoff + i] : xc[d.xoff + i];
}

}  // namespace mrx

using namespace mrx;

extern "C" mrx_status mrx_dc_judge(mrx_plan p, const float* x_net, const float* x_cg, const float* aHy,
                                   const float* S, const float* mask, float ratio, float* out,
                                   uint32_t* dev_choice, void* stream) {
  if (!p) return fail(MRX_EINVAL, "dc_judge: null plan");
  if (!x_net || !x_cg || !aHy || !S || !mask || !out || !dev_choice)
    return fail(MRX_EINVAL, "dc_judge: null data pointer");
  if (!(ratio > 0.f)) return fail(MRX_EINVAL, "dc_judge: ratio must be positive");
  if (!p->ws) return fail(MRX_ENOWORKSPACE, "dc_judge: workspace not set");
  hipStream_t s = (hipStream_t)stream;
  float2* q = (float2*)(p->ws + p->ws_q);
  // [B][nrr] partials: residual of x_net, its non-finite count, residual of x_cg
  float* pc = (float*)(p->ws + p->ws_rr0);
  float* pn = (float*)(p->ws + p->ws_rr1);
  float* pf = (float*)(p->ws + p->ws_part);
  const dim3 grid(p->nrr, p->B);
  mrx_status st = normal_impl(p, (const float2*)x_net, (const float2*)S, mask, nullptr, q, s);
  if (st != MRX_OK) return st;
  hipLaunchKernelGGL(k_dc_resid, grid, dim3(CG_THREADS), 0, s, p->d_desc, p->d_all, q, (const float2*)aHy,
                     (const float2*)x_net, pc, pn, p->nrr);
  st = normal_impl(p, (const float2*)x_cg, (const float2*)S, mask, nullptr, q, s);
  if (st != MRX_OK) return st;
  hipLaunchKernelGGL(k_dc_resid, grid, dim3(CG_THREADS), 0, s, p->d_desc, p->d_all, q, (const float2*)aHy,
                     (const float2*)x_cg, pf, nullptr, p->nrr);
  hipLaunchKernelGGL(k_dc_decide, dim3((p->B + 63) / 64), dim3(64), 0, s, p->d_desc, pc, pn, pf, p->nrr, p->B, ratio,
                     (uint32_t*)(p->ws + p->ws_status), dev_choice);
  hipLaunchKernelGGL(k_dc_select, dim3((unsigned)((p->maxHW + 255) / 256), p->B), dim3(256), 0, s, p->d_desc,
                     (const float2*)x_net, (const float2*)x_cg, dev_choice, (float2*)out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MRX_OK : hip_fail(e, "dc_judge");
}
