// Conjugate-gradient vector kernels with per-slice device scalars and
// deterministic fixed-order reductions (CG as used for the MoDL inversion
// S_lambda^{-1}, MoDL subsection).
//
// Each slice's vectors are split into blocks of EPB elements; a block writes
// one partial sum per reduction and every consumer re-sums the partials of a
// slice in the same fixed order, so results are bitwise reproducible and no
// float atomics are used.
#include "cg_kernels.h"

namespace mrx {

__device__ __forceinline__ float bsum(float v, float* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < CG_THREADS / 64; ++i) s += red[i];
  return s;
}

__device__ __forceinline__ float psum(const float* a, int n) {
  // fixed-order sum, returned to every thread of the block: thread t adds
  // a[t], a[t + CG_THREADS], ...; then a fixed butterfly in each wavefront
  // and the wavefront sums in order
  __shared__ float tmp[CG_THREADS / 64];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += CG_THREADS) s += a[i];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) tmp[threadIdx.x >> 6] = s;
  __syncthreads();
  float t = 0.f;
#pragma unroll
  for (int w = 0; w < CG_THREADS / 64; ++w) t += tmp[w];
  return t;
}

// psum of two arrays at once (one pass of loads and barriers for both).
__device__ __forceinline__ float2 psum2(const float* a, int na, const float* b, int nb) {
  __shared__ float tmp[2][CG_THREADS / 64];
  float s = 0.f, t = 0.f;
  for (int i = threadIdx.x; i < na; i += CG_THREADS) s += a[i];
  for (int i = threadIdx.x; i < nb; i += CG_THREADS) t += b[i];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    s += __shfl_xor(s, off, 64);
    t += __shfl_xor(t, off, 64);
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    tmp[0][threadIdx.x >> 6] = s;
    tmp[1][threadIdx.x >> 6] = t;
  }
  __syncthreads();
  float u = 0.f, v = 0.f;
#pragma unroll
  for (int w = 0; w < CG_THREADS / 64; ++w) {
    u += tmp[0][w];
    v += tmp[1][w];
  }
  return make_float2(u, v);
}

// r = aHy + lambda z, p = r, x = 0; partials of <r, r>.
__global__ void __launch_bounds__(CG_THREADS) k_cg_init(CgElemArgs a) {
  __shared__ float red[CG_THREADS / 64];
  const int b = a.slices[blockIdx.y];
  const SliceDesc d = a.desc[b];
  const int64_t n = (int64_t)d.H * d.W;
  const float lam = a.lam ? a.lam[b] : 0.f;
  float rr = 0.f;
  const int64_t base = (int64_t)blockIdx.x * CG_EPB;
  for (int k = threadIdx.x; k < CG_EPB; k += CG_THREADS) {
    const int64_t i = base + k;
    if (i >= n) break;
    const int64_t o = d.xoff + i;
    float2 r = a.aHy[o];
    if (a.z) { const float2 z = a.z[o]; r.x += lam * z.x; r.y += lam * z.y; }
    a.r[o] = r;
    a.p[o] = r;
    a.x[o] = make_float2(0.f, 0.f);
    rr += r.x * r.x + r.y * r.y;
  }
  // the <p, q> partials of tiles that a schedule never writes must read as zero
  if (a.pq_clear && blockIdx.x == 0)
    for (int i = threadIdx.x; i < a.npq; i += CG_THREADS) a.pq_clear[(int64_t)b * a.npq + i] = 0.f;
  const float s = bsum(rr, red);
  if (threadIdx.x == 0) {
    a.rr_next[(int64_t)b * a.nrr + blockIdx.x] = s;
    if (blockIdx.x == 0) { a.stopped[b] = 0; }
  }
}

// alpha = rho / Re<p, q>; x += alpha p; r -= alpha q; partials of <r, r>.
__global__ void __launch_bounds__(CG_THREADS) k_cg_update(CgElemArgs a) {
  __shared__ float red[CG_THREADS / 64];
  const int b = a.slices[blockIdx.y];
  const SliceDesc d = a.desc[b];
  const int64_t n = (int64_t)d.H * d.W;
  const int64_t base = (int64_t)blockIdx.x * CG_EPB;
  // all of a thread's loads are issued first (one memory latency per block,
  // overlapping the reductions that give alpha)
  // (the further partial planes of a coil split included: the bound on
  // their count makes every load a straight-line one)
  constexpr int PER = CG_EPB / CG_THREADS;
  float2 rv[PER], pv[PER], qv[PER], xv[PER], qe[CG_QPARTS_MAX - 1][PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int64_t i = base + threadIdx.x + j * CG_THREADS;
    const int64_t o = d.xoff + (i < n ? i : 0);
    rv[j] = a.r[o];
    pv[j] = a.p[o];
    qv[j] = a.q[o];
    xv[j] = a.x[o];
#pragma unroll
    for (int k = 1; k < CG_QPARTS_MAX; ++k)
      if (k < d.nq) qe[k - 1][j] = a.q[k * a.qstride + o];
  }
#pragma unroll
  for (int k = 1; k < CG_QPARTS_MAX; ++k)
    if (k < d.nq) {
#pragma unroll
      for (int j = 0; j < PER; ++j) qv[j] = cadd(qv[j], qe[k - 1][j]);
    }
  const float2 rp = psum2(a.rr_cur + (int64_t)b * a.nrr, a.nrr, a.pq + (int64_t)b * a.npq, a.npq);
  const float rho = rp.x, pq = rp.y;
  bool stop = a.stopped[b] != 0;
  const bool bad = !(pq > 0.f) || !(rho > 0.f) || !isfinite(rho / pq);
  if (!stop && bad) {
    stop = true;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.stopped[b] = 1;
      uint32_t f = 0;
      if (!isfinite(pq) || !isfinite(rho)) f |= FLAG_NONFINITE;
      else if (rho > 0.f) f |= FLAG_CG_BREAKDOWN;
      if (f) a.status[b] |= f;
    }
  }
  const float alpha = stop ? 0.f : rho / pq;
  float rr = 0.f;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int64_t i = base + threadIdx.x + j * CG_THREADS;
    if (i >= n) break;
    const int64_t o = d.xoff + i;
    float2 r = rv[j];
    if (!stop) {
      float2 x = xv[j];
      x.x += alpha * pv[j].x; x.y += alpha * pv[j].y;
      r.x -= alpha * qv[j].x; r.y -= alpha * qv[j].y;
      a.x[o] = x;
      a.r[o] = r;
    }
    rr += r.x * r.x + r.y * r.y;
  }
  const float s = bsum(rr, red);
  if (threadIdx.x == 0) a.rr_next[(int64_t)b * a.nrr + blockIdx.x] = s;
}

// The search direction of a CG step, formed once for an operator that
// then reads it as given (p_out = r + beta p_in; see cg_kernels.h).
__global__ void __launch_bounds__(CG_THREADS) k_cg_form_p(CgElemArgs a) {
  const int b = a.slices[blockIdx.y];
  const SliceDesc d = a.desc[b];
  const int64_t n = (int64_t)d.H * d.W;
  const int64_t base = (int64_t)blockIdx.x * CG_EPB;
  // the thread's loads first, then both rho sums in one pass (their memory
  // latency overlaps the reductions, as in k_cg_update)
  constexpr int PER = CG_EPB / CG_THREADS;
  float2 rv[PER], pv[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int64_t i = base + threadIdx.x + j * CG_THREADS;
    const int64_t o = d.xoff + (i < n ? i : 0);
    rv[j] = a.r[o];
    pv[j] = a.p[o];
  }
  const float2 rr = psum2(a.rr_cur + (int64_t)b * a.nrr, a.nrr, a.rr_next + (int64_t)b * a.nrr, a.nrr);
  if (a.stopped[b]) return;
  const float beta = rr.y > 0.f ? rr.x / rr.y : 0.f;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int64_t i = base + threadIdx.x + j * CG_THREADS;
    if (i < n) a.x[d.xoff + i] = make_float2(rv[j].x + beta * pv[j].x, rv[j].y + beta * pv[j].y);
  }
}

// hist[b][k] = rho_k (sum of the current partials).
__global__ void __launch_bounds__(CG_THREADS) k_cg_hist(CgElemArgs a, int k, int stride) {
  const int b = a.slices[blockIdx.y];
  const float rho = psum(a.rr_cur + (int64_t)b * a.nrr, a.nrr);
  if (threadIdx.x == 0) a.hist[(int64_t)b * stride + k] = rho;
}

// Backward helpers: g_z = lambda v; partials of Re<v, z - x>.
__global__ void __launch_bounds__(CG_THREADS) k_cg_bwd_tail(CgElemArgs a, float2* gz, float* part) {
  __shared__ float red[CG_THREADS / 64];
  const int b = a.slices[blockIdx.y];
  const SliceDesc d = a.desc[b];
  const int64_t n = (int64_t)d.H * d.W;
  const float lam = a.lam ? a.lam[b] : 0.f;
  float acc = 0.f;
  const int64_t base = (int64_t)blockIdx.x * CG_EPB;
  for (int k = threadIdx.x; k < CG_EPB; k += CG_THREADS) {
    const int64_t i = base + k;
    if (i >= n) break;
    const int64_t o = d.xoff + i;
    const float2 v = a.x[o];
    if (gz) gz[o] = make_float2(lam * v.x, lam * v.y);
    if (part) {
      float2 zx = a.z ? a.z[o] : make_float2(0.f, 0.f);
      const float2 xf = a.aHy[o];  // forward solution
      zx.x -= xf.x; zx.y -= xf.y;
      acc += v.x * zx.x + v.y * zx.y;
    }
  }
  if (part) {
    const float s = bsum(acc, red);
    if (threadIdx.x == 0) part[(int64_t)b * a.nrr + blockIdx.x] = s;
  }
}

__global__ void __launch_bounds__(CG_THREADS) k_slice_sum(CgElemArgs a, const float* part, float* out, int accumulate) {
  const int b = a.slices[blockIdx.y];
  const float s = psum(part + (int64_t)b * a.nrr, a.nrr);
  if (threadIdx.x == 0) out[b] = accumulate ? out[b] + s : s;
}

hipError_t cg_init(const CgElemArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_init, dim3(a.nrr, a.nslices), dim3(CG_THREADS), 0, s, a);
  return hipGetLastError();
}
hipError_t cg_form_p(const CgElemArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_form_p, dim3(a.nrr, a.nslices), dim3(CG_THREADS), 0, s, a);
  return hipGetLastError();
}
hipError_t cg_update(const CgElemArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_update, dim3(a.nrr, a.nslices), dim3(CG_THREADS), 0, s, a);
  return hipGetLastError();
}
hipError_t cg_hist(const CgElemArgs& a, int k, int stride, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_hist, dim3(1, a.nslices), dim3(CG_THREADS), 0, s, a, k, stride);
  return hipGetLastError();
}
hipError_t cg_bwd_tail(const CgElemArgs& a, float2* gz, float* part, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_bwd_tail, dim3(a.nrr, a.nslices), dim3(CG_THREADS), 0, s, a, gz, part);
  return hipGetLastError();
}
hipError_t slice_sum(const CgElemArgs& a, const float* part, float* out, int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(k_slice_sum, dim3(1, a.nslices), dim3(CG_THREADS), 0, s, a, part, out, accumulate);
  return hipGetLastError();
}

}  // namespace mrx
