// Soft-SENSE operator kernels: the SENSE model with two sets of coil maps
// (Extensions to the SENSE-Model subsection),
//   y_c = P F (S_{0,c} x_0 + S_{1,c} x_1),   (A^H y)_m = sum_c conj(S_{m,c}) F^H P^H y_c.
// Layout of slice b (offsets from the plan's descriptor d): image sets
// [2][H][W] at 2 d.xoff, coil maps [2][C][H][W] at 2 d.soff, k-space
// [C][H][W] at d.soff (as for SENSE), mask [H] at d.moff.  The kernels are
// the SENSE column passes and the fused normal operator with the two sets
// combined before the transform and separated after it; the row passes
// (along W) are the SENSE ones.
#pragma once
#include "sense_impl.h"

namespace mrx {

// Forward column pass: v = S_{0,c} x_0 + S_{1,c} x_1, transform along H,
// keep sampled rows (signs and centering as k_fwd_col).  Loads address a
// wave-uniform plane base plus one 32-bit lane offset (lanes past the last
// column of a ragged tile read column W - 1 and store nothing).
template <class Sd, int WT>
__global__ void __launch_bounds__(Sd::T * WT, 2)
k_fwd_col_soft(SenseColArgs a) {
  constexpr int N = Sd::N, P = Sd::P, T = Sd::T;
  using L = LdsInterleaved<N, WT>;
  __shared__ float2 lds[L::SIZE];
  __shared__ float2 tw[N];
  __shared__ float mk[N];
  const int unit = col_pass_unit<WT>(blockIdx.x), si = unit / a.tiles, tile = unit % a.tiles;
  if (si >= a.nslices) return;
  const int b = a.slices[si];
  const SliceDesc d = a.desc[b];
  if (d.H != N) return;
  const int W = d.W;
  if (tile * WT >= W) return;
  const int lid = threadIdx.x, c = lid % WT, tc = lid / WT, col = tile * WT + c;
  const bool valid = col < W;
  for (int i = lid; i < N; i += T * WT) {
    tw[i] = a.tw[i];
    mk[i] = a.mask[d.moff + i];
  }
  __syncthreads();
  const float scale = rsqrtf((float)N);
  const int64_t plane = (int64_t)N * W;
  const uint32_t voff = (uint32_t)(tc * W + (valid ? col : W - 1)) * 8u;
  auto so = [&](int i, int r) { return (uint32_t)((T * i + r * Sd::M1) * W) * 8u; };
  const uint32_t pbytes = (uint32_t)N * (uint32_t)W * 8u;
  const float2* xin = a.in + 2 * d.xoff;
  const BufPlane xp0(xin, pbytes), xp1(xin + plane, pbytes);
  float2 x0[P], x1[P];
#pragma unroll
  for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
    for (int r = 0; r < Sd::N1; ++r) {
      x0[i * Sd::N1 + r] = xp0.ld(voff, so(i, r));
      x1[i * Sd::N1 + r] = xp1.ld(voff, so(i, r));
    }
  const float2* Sb = a.S + 2 * d.soff;
  for (int coil = 0; coil < d.C; ++coil) {
    const BufPlane S0(Sb + coil * plane, pbytes), S1(Sb + (d.C + coil) * plane, pbytes);
    float2 v[P];
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
      for (int r = 0; r < Sd::N1; ++r) {
        const int k = i * Sd::N1 + r;
        v[k] = cadd(cmul(S0.ld_nt(voff, so(i, r)), x0[k]), cmul(S1.ld_nt(voff, so(i, r)), x1[k]));
      }
    fft_forward<Sd, L>(v, lds, tw, tc, c);
    const BufPlane oc(a.out + d.soff + coil * plane, pbytes);
#pragma unroll
    for (int i = 0; i < Sd::GFIN; ++i)
#pragma unroll
      for (int r = 0; r < Sd::NFIN; ++r) {
        const int j = Sd::freq(tc, i, r);
        const int k = (j + N / 2) % N;
        const float sg = (j & 1) ? -scale : scale;
        if (valid && mk[k] != 0.f) oc.st(cscale(v[i * Sd::NFIN + r], sg), (uint32_t)(k * W + col) * 8u, 0);
      }
  }
}

// Adjoint column pass: per coil, the sampled rows of the row-pass output in
// frequency order with the centering sign, inverse transform along H, then
// x_m += conj(S_{m,c}) v for both sets (addressing as the forward pass).
template <class Sd, int WT>
__global__ void __launch_bounds__(Sd::T * WT, 2)
k_adj_col_soft(SenseColArgs a) {
  constexpr int N = Sd::N, P = Sd::P, T = Sd::T;
  using L = LdsInterleaved<N, WT>;
  __shared__ float2 lds[L::SIZE];
  __shared__ float2 tw[N];
  __shared__ float mk[N];
  const int unit = col_pass_unit<WT>(blockIdx.x), si = unit / a.tiles, tile = unit % a.tiles;
  if (si >= a.nslices) return;
  const int b = a.slices[si];
  const SliceDesc d = a.desc[b];
  if (d.H != N) return;
  const int W = d.W;
  if (tile * WT >= W) return;
  const int lid = threadIdx.x, c = lid % WT, tc = lid / WT, col = tile * WT + c;
  const bool valid = col < W;
  for (int i = lid; i < N; i += T * WT) {
    tw[i] = a.tw[i];
    mk[i] = a.mask[d.moff + i];
  }
  __syncthreads();
  const float scale = rsqrtf((float)N);
  const int64_t plane = (int64_t)N * W;
  const int ccol = valid ? col : W - 1;
  const uint32_t voff = (uint32_t)(tc * W + ccol) * 8u;
  auto so = [&](int i, int r) { return (uint32_t)((T * i + r * Sd::M1) * W) * 8u; };
  const uint32_t pbytes = (uint32_t)N * (uint32_t)W * 8u;
  const float2* Sb = a.S + 2 * d.soff;
  float2 acc0[P], acc1[P];
#pragma unroll
  for (int k = 0; k < P; ++k) acc0[k] = acc1[k] = make_float2(0.f, 0.f);
  for (int coil = 0; coil < d.C; ++coil) {
    const BufPlane ic(a.in + d.soff + coil * plane, pbytes);
    float2 v[P];
#pragma unroll
    for (int i = 0; i < Sd::GFIN; ++i)
#pragma unroll
      for (int r = 0; r < Sd::NFIN; ++r) {
        const int j = Sd::freq(tc, i, r);
        const int k = (j + N / 2) % N;
        const float sg = (j & 1) ? -scale : scale;
        float2 u = make_float2(0.f, 0.f);
        if (mk[k] != 0.f) u = cscale(ic.ld((uint32_t)(k * W + ccol) * 8u, 0), sg);
        v[i * Sd::NFIN + r] = u;
      }
    fft_inverse<Sd, L>(v, lds, tw, tc, c);
    const BufPlane S0(Sb + coil * plane, pbytes), S1(Sb + (d.C + coil) * plane, pbytes);
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
      for (int r = 0; r < Sd::N1; ++r) {
        const int k = i * Sd::N1 + r;
        acc0[k] = cadd(acc0[k], cmulc(S0.ld_nt(voff, so(i, r)), v[k]));
        acc1[k] = cadd(acc1[k], cmulc(S1.ld_nt(voff, so(i, r)), v[k]));
      }
  }
  if (!valid) return;
  const float2* xo = a.out + 2 * d.xoff;
  const BufPlane q0(xo, pbytes), q1(xo + plane, pbytes);
#pragma unroll
  for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
    for (int r = 0; r < Sd::N1; ++r) {
      const int k = i * Sd::N1 + r;
      q0.st(acc0[k], voff, so(i, r));
      q1.st(acc1[k], voff, so(i, r));
    }
}

// Normal operator (A^H A + lambda I) p on both sets, one pass over the coil
// maps: per coil v = S_{0,c} p_0 + S_{1,c} p_1, transform along H, mask,
// inverse transform, q_m += conj(S_{m,c}) v; q_m += lambda p_m.  One
// workgroup = WT columns of one slice.  Mode 1 (CG step): p is given as pin (the CG step forms
// p = r + beta p beforehand, once for both sets) and the tile's Re<p, q>
// partial goes to pq_part.  The operand is re-read for every coil (it is
// L2-resident) so that only the two accumulators and the transform stay in
// registers.  KSPL > 1 (CG steps): a column tile's coils are split over
// KSPL workgroups, each writing its partial planes (both sets) at
// qout + k qstride and its own Re<p, q> partial; the first adds lambda p;
// the CG update adds the planes.
template <class Sd, int WT, int KSPL>
__global__ void __launch_bounds__(Sd::T * WT, 2)
k_normal_soft(NormalArgs a) {
  constexpr int N = Sd::N, P = Sd::P, T = Sd::T, NT = T * WT;
  static_assert(NT % 64 == 0, "the tile's dot product reduces over whole wavefronts");
  using L = LdsInterleaved<N, WT>;
  __shared__ float2 lds[L::SIZE];
  __shared__ float2 tw[N];
  __shared__ float mk[N];
  __shared__ float red[NT / 64];
  // workgroup -> (slice, column tile, coil split): consecutive workgroups
  // go to the 8 XCDs in turn, so the KSPL splits of a (slice, tile) unit,
  // 8 workgroups apart, run on one XCD and share the operand in its L2
  const int Lb = blockIdx.x;
  const int unit = (Lb / (8 * KSPL)) * 8 + (Lb & 7), ks = (Lb >> 3) % KSPL;
  const int si = unit / a.tiles, tile = unit % a.tiles;
  if (si >= a.nslices) return;
  const int b = a.slices[si];
  const SliceDesc d = a.desc[b];
  if (d.H != N) return;
  const int W = d.W;
  if (tile * WT >= W) return;
  const int c_begin = (ks * d.C) / KSPL, c_end = ((ks + 1) * d.C) / KSPL;
  const int lid = threadIdx.x, c = lid % WT, tc = lid / WT, col = tile * WT + c;
  const bool valid = col < W;
  const uint32_t voff = (uint32_t)(tc * W + (valid ? col : W - 1)) * 8u;
  auto so = [&](int i, int r) { return (uint32_t)((T * i + r * Sd::M1) * W) * 8u; };
  const uint32_t pbytes = (uint32_t)N * (uint32_t)W * 8u;
  const bool cg = a.mode == 1;
  if (cg && a.stopped[b]) return;
  for (int i = lid; i < N; i += NT) {
    tw[i] = a.tw[i];
    mk[i] = a.mask[d.moff + (i + N / 2) % N] * (1.0f / N);
  }
  __syncthreads();
  const int64_t plane = (int64_t)N * W;
  const int64_t xo = 2 * d.xoff;
  const BufPlane pin0(a.pin + xo, pbytes), pin1(a.pin + xo + plane, pbytes);
  float2 acc0[P], acc1[P];
#pragma unroll
  for (int k = 0; k < P; ++k) acc0[k] = acc1[k] = make_float2(0.f, 0.f);
  const float2* Sb = a.S + 2 * d.soff;
  for (int coil = c_begin; coil < c_end; ++coil) {
    const BufPlane S0(Sb + coil * plane, pbytes), S1(Sb + (d.C + coil) * plane, pbytes);
    float2 v[P];
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
      for (int r = 0; r < Sd::N1; ++r) {
        const uint32_t s = so(i, r);
        // the maps stream (non-temporal); the operand stays in L2 for the
        // tile's other coils
        v[i * Sd::N1 + r] = cadd(cmul(S0.ld_nt(voff, s), pin0.ld(voff, s)), cmul(S1.ld_nt(voff, s), pin1.ld(voff, s)));
      }
    // the tile region sees only alternating forward and inverse transforms
    fft_forward<Sd, L, BlockSyncPost>(v, lds, tw, tc, c);
    fft_inverse<Sd, L, BlockSyncPost, FreqScale>(v, lds, tw, tc, c, FreqScale{mk});
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
      for (int r = 0; r < Sd::N1; ++r) {
        const int k = i * Sd::N1 + r;
        acc0[k] = cadd(acc0[k], cmulc(S0.ld_nt(voff, so(i, r)), v[k]));
        acc1[k] = cadd(acc1[k], cmulc(S1.ld_nt(voff, so(i, r)), v[k]));
      }
  }
  const float lam = (a.lam && ks == 0) ? a.lam[b] : 0.f;
  float2* qo = a.qout + (int64_t)ks * a.qstride;
  const BufPlane q0(qo + xo, pbytes), q1(qo + xo + plane, pbytes);
  float dot = 0.f;
#pragma unroll
  for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
    for (int r = 0; r < Sd::N1; ++r) {
      const int k = i * Sd::N1 + r;
      const uint32_t s = so(i, r);
      const float2 p0 = pin0.ld(voff, s), p1 = pin1.ld(voff, s);
      const float2 u0 = make_float2(acc0[k].x + lam * p0.x, acc0[k].y + lam * p0.y);
      const float2 u1 = make_float2(acc1[k].x + lam * p1.x, acc1[k].y + lam * p1.y);
      dot += p0.x * u0.x + p0.y * u0.y + p1.x * u1.x + p1.y * u1.y;
      if (valid) {
        q0.st(u0, voff, s);
        q1.st(u1, voff, s);
      }
    }
  if (!valid) dot = 0.f;
  if (cg) {
    const float s = block_sum_fixed(dot, red);
    if (lid == 0) a.pq_part[(int64_t)b * a.npq + tile * KSPL + ks] = s;
  }
}

// CG steps split each column tile's coils over SOFT_KSPL workgroups (partial
// planes a.qstride apart; p given, so iter 0 and no pout); operator
// applications too when split_plain is set (the caller adds the planes),
// else unsplit.
template <class Sd, int WT>
hipError_t launch_normal_soft(const NormalArgs& a0, int maxW, hipStream_t s) {
  NormalArgs a = a0;
  a.tiles = (maxW + WT - 1) / WT;
  if (a.mode == 1 || a.split_plain) {
    if (a.qstride <= 0) return hipErrorInvalidValue;
    // p is given (pin): the kernel neither forms nor writes it
    if (a.mode == 1 && (a.tiles * SOFT_KSPL > a.npq || a.iter != 0 || a.pout)) return hipErrorInvalidValue;
    const int total = a.tiles * a.nslices * SOFT_KSPL, per = 8 * SOFT_KSPL;
    hipLaunchKernelGGL((k_normal_soft<Sd, WT, SOFT_KSPL>), dim3((unsigned)(((total + per - 1) / per) * per)),
                       dim3(Sd::T * WT), 0, s, a);
  } else {
    const int total = a.tiles * a.nslices;
    hipLaunchKernelGGL((k_normal_soft<Sd, WT, 1>), dim3((unsigned)(((total + 7) / 8) * 8)), dim3(Sd::T * WT), 0,
                       s, a);
  }
  return hipGetLastError();
}
template <class Sd, int WT>
hipError_t launch_fwd_col_soft(const SenseColArgs& a, int maxW, hipStream_t s) {
  SenseColArgs c = a;
  c.tiles = (maxW + WT - 1) / WT;
  hipLaunchKernelGGL((k_fwd_col_soft<Sd, WT>), col_pass_grid(c.tiles, c.nslices), dim3(Sd::T * WT), 0, s, c);
  return hipGetLastError();
}
template <class Sd, int WT>
hipError_t launch_adj_col_soft(const SenseColArgs& a, int maxW, hipStream_t s) {
  SenseColArgs c = a;
  c.tiles = (maxW + WT - 1) / WT;
  hipLaunchKernelGGL((k_adj_col_soft<Sd, WT>), col_pass_grid(c.tiles, c.nslices), dim3(Sd::T * WT), 0, s, c);
  return hipGetLastError();
}

// Registers the soft-SENSE kernels of one length (built on the length's
// default decomposition): the normal operator on WTN-column tiles, the
// column passes on WTC-column tiles.
template <class Sd, int WTN, int WTC>
struct RegistrarSoft {
  RegistrarSoft(const char* name) {
    SoftVariant v{Sd::N, &launch_normal_soft<Sd, WTN>, &launch_fwd_col_soft<Sd, WTC>, &launch_adj_col_soft<Sd, WTC>,
                  name};
    register_soft_variant(v);
  }
};

}  // namespace mrx
