// Normal operator of non-Cartesian SENSE through its Toeplitz form (the
// PSF convolution of the Extensions to the SENSE-Model subsection):
//
//   (A^H A + lambda I) p = sum_c conj(S_c) crop(IDFT_2(psf * DFT_2(pad(S_c p)))) + lambda p,
//
// pad: zero-extension of an H x W image to 2H x 2W (top-left corner), DFT_2
// the unnormalised 2H x 2W DFT, crop the top-left H x W of the result, psf
// the real spectrum of the sampling's point spread function on that grid.
// Three passes, each a kernel over the batch:
//   rows:    t_c = DFT_2W(pad_W(S_c p)) row by row -> buffer [C][H][2W]
//   columns: t_c <- IDFT_2H(psf / (4HW) * DFT_2H(pad_H t_c)), rows < H kept
//   rows:    q = sum_c conj(S_c) IDFT_2W(t_c)[< W] + lambda p
// The transforms of length 2N use a decomposition whose first radix is 2
// (N1 = 2, M1 = N): a thread's slots of digit 0 are the points n < N and
// those of digit 1 the points n >= N, so the zero half of a padded input is
// a compile-time zero (the first radix-2 level folds it away) and the crop
// keeps the digit-0 slots.  In CG steps the first pass forms p = r + beta p
// as the Cartesian operator does and the last one splits its coils over
// workgroups writing partial output planes, which the CG update adds.
#pragma once
#include "sense_impl.h"

namespace mrx {


// CG steps: beta = rho_k / rho_{k-1} from the partial sums (wave 0), in
// the Cartesian operator's order.
__device__ __forceinline__ float toep_beta(const ToepArgs& a, int b, int lid) {
  const float rc = wave_sum_fixed(a.rr_cur + (int64_t)b * a.nrr, a.nrr, lid);
  const float rp = wave_sum_fixed(a.rr_prev + (int64_t)b * a.nrr, a.nrr, lid);
  return rp > 0.f ? rc / rp : 0.f;
}

// ------------------------------------------------------------ first pass
// WT rows a workgroup, T threads a row; grid.x = row blocks x coil groups,
// grid.y = slices of the launch.
template <class Sd, int WT>
__global__ void __launch_bounds__(Sd::T * WT)
k_toep_rows_fwd(ToepArgs a) {
  constexpr int N = Sd::N, P = Sd::P, T = Sd::T, W = N / 2;
  static_assert(Sd::N1 == 2 && Sd::M1 == W, "padded transforms need a first radix of 2");
  using L = LdsContig<N, WT>;
  __shared__ float2 lds[L::SIZE];
  __shared__ float2 tw[N];
  __shared__ float sc[1];
  const int b = a.slices[blockIdx.y];
  const SliceDesc d = a.desc[b];
  if (2 * d.W != N) return;
  const int H = d.H, C = d.C;
  const int rblocks = (H + WT - 1) / WT;
  const int rb = blockIdx.x % rblocks, grp = blockIdx.x / rblocks;
  if (grp >= a.split) return;
  const bool cg = a.mode == 1;
  if (cg && a.stopped[b]) return;
  const int c_begin = grp * C / a.split, c_end = (grp + 1) * C / a.split;
  const int lid = threadIdx.x, tc = lid % T, c = lid / T;
  const int row = rb * WT + c;
  const bool valid = row < H;
  const int rowc = valid ? row : H - 1;  // ragged block: transform a real row, store nothing
  for (int i = lid; i < N; i += T * WT) tw[i] = a.tw[i];
  if (cg && a.iter > 0 && lid < 64) {
    const float beta = toep_beta(a, b, lid);
    if (lid == 0) sc[0] = beta;
  }
  __syncthreads();
  const int64_t prow = d.xoff + (int64_t)rowc * W;
  float2 pv[Sd::G1];
  if (cg && a.iter > 0) {
    const float beta = sc[0];
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i) {
      const int n = tc + T * i;
      const float2 o = a.pin[prow + n], rv = a.r[prow + n];
      pv[i] = make_float2(rv.x + beta * o.x, rv.y + beta * o.y);
    }
    // pout differs from pin in CG steps; the first coil group writes p
    if (valid && grp == 0)
#pragma unroll
      for (int i = 0; i < Sd::G1; ++i) a.pout[prow + tc + T * i] = pv[i];
  } else {
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i) pv[i] = a.pin[prow + tc + T * i];
  }
  for (int coil = c_begin; coil < c_end; ++coil) {
    const float2* Sr = a.S + d.soff + ((int64_t)coil * H + rowc) * W;
    float2 v[P];
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i) {
      v[2 * i] = cmul(Sr[tc + T * i], pv[i]);
      v[2 * i + 1] = make_float2(0.f, 0.f);
    }
    fft_forward<Sd, L>(v, lds, tw, tc, c);
    if (valid) {
      float2* o = a.tbuf + 2 * d.soff + ((int64_t)coil * H + row) * N;
#pragma unroll
      for (int i = 0; i < Sd::GFIN; ++i)
#pragma unroll
        for (int r = 0; r < Sd::NFIN; ++r) o[Sd::freq(tc, i, r)] = v[i * Sd::NFIN + r];
    }
  }
}

// ----------------------------------------------------------- middle pass
// WT frequency columns a workgroup (of the 2W), T threads a column, the
// column's PSF values in registers for all the group's coils; grid.x =
// column tiles x coil groups (rounded up to a multiple of 16), grid.y =
// slices.  Tiles 2k and 2k + 1 (the two halves of a 128-byte row segment
// for WT = 8) get block ids 8 apart, so that they run on the same XCD
// (workgroups go to the 8 XCDs in turn) and share its L2.  The transform
// chain forward, inverse, forward, ... allows the post-write-only barriers
// of the Cartesian operator.
template <class Sd, int WT>
__global__ void __launch_bounds__(Sd::T * WT, 2)
k_toep_cols(ToepArgs a) {
  constexpr int N = Sd::N, P = Sd::P, T = Sd::T, H = N / 2;
  static_assert(Sd::N1 == 2 && Sd::M1 == H, "padded transforms need a first radix of 2");
  using L = LdsInterleaved<N, WT>;
  __shared__ float2 lds[L::SIZE];
  __shared__ float2 tw[N];
  const int b = a.slices[blockIdx.y];
  const SliceDesc d = a.desc[b];
  if (2 * d.H != N) return;
  const int W2 = 2 * d.W, C = d.C;
  const int tiles = (W2 + WT - 1) / WT;
  const int Lb = blockIdx.x;
  const int ug = (((Lb >> 4) * 8 + (Lb & 7)) << 1) + ((Lb >> 3) & 1);
  const int tile = ug % tiles, grp = ug / tiles;
  if (grp >= a.split) return;
  if (a.mode == 1 && a.stopped[b]) return;
  const int c_begin = grp * C / a.split, c_end = (grp + 1) * C / a.split;
  const int lid = threadIdx.x, c = lid % WT, tc = lid / WT;
  const int col = tile * WT + c;
  const bool valid = col < W2;
  const int colc = valid ? col : W2 - 1;
  for (int i = lid; i < N; i += T * WT) tw[i] = a.tw[i];
  // psf of this column at the thread's frequencies, with the 1 / (4 H W) of
  // the two unnormalised 2-D transforms
  const float scale = 1.0f / ((float)N * (float)W2);
  float ps[P];
  {
    const float* pc = a.psf + 4 * d.xoff + colc;
#pragma unroll
    for (int i = 0; i < Sd::GFIN; ++i)
#pragma unroll
      for (int r = 0; r < Sd::NFIN; ++r)
        ps[i * Sd::NFIN + r] = pc[(int64_t)Sd::freq(tc, i, r) * W2] * scale;
  }
  __syncthreads();
  for (int coil = c_begin; coil < c_end; ++coil) {
    float2* base = a.tbuf + 2 * d.soff + (int64_t)coil * H * W2 + colc;
    float2 v[P];
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i) {
      v[2 * i] = base[(int64_t)(tc + T * i) * W2];
      v[2 * i + 1] = make_float2(0.f, 0.f);
    }
    fft_forward<Sd, L, BlockSyncPost>(v, lds, tw, tc, c);
#pragma unroll
    for (int k = 0; k < P; ++k) v[k] = cscale(v[k], ps[k]);
    fft_inverse<Sd, L, BlockSyncPost>(v, lds, tw, tc, c);
    if (valid)
#pragma unroll
      for (int i = 0; i < Sd::G1; ++i) base[(int64_t)(tc + T * i) * W2] = v[2 * i];
  }
}

// ------------------------------------------------------------- last pass
// WT rows a workgroup, T threads a row; grid.x = row blocks x output
// planes, grid.y = slices.  Plane 0 adds lambda p; each plane writes the
// partial sums of Re<p, q> of its rows (CG steps).
template <class Sd, int WT>
__global__ void __launch_bounds__(Sd::T * WT)
k_toep_rows_adj(ToepArgs a) {
  constexpr int N = Sd::N, P = Sd::P, T = Sd::T, W = N / 2;
  static_assert(Sd::N1 == 2 && Sd::M1 == W, "padded transforms need a first radix of 2");
  using L = LdsContig<N, WT>;
  __shared__ float2 lds[L::SIZE];
  __shared__ float2 tw[N];
  __shared__ float red[(T * WT + 63) / 64];
  const int b = a.slices[blockIdx.y];
  const SliceDesc d = a.desc[b];
  if (2 * d.W != N) return;
  const int H = d.H, C = d.C;
  const int rblocks = (H + WT - 1) / WT;
  const int rb = blockIdx.x % rblocks, ks = blockIdx.x / rblocks;
  if (ks >= a.split) return;
  const bool cg = a.mode == 1;
  if (cg && a.stopped[b]) return;
  const int c_begin = ks * C / a.split, c_end = (ks + 1) * C / a.split;
  const int lid = threadIdx.x, tc = lid % T, c = lid / T;
  const int row = rb * WT + c;
  const bool valid = row < H;
  const int rowc = valid ? row : H - 1;
  for (int i = lid; i < N; i += T * WT) tw[i] = a.tw[i];
  __syncthreads();
  float2 acc[Sd::G1];
#pragma unroll
  for (int i = 0; i < Sd::G1; ++i) acc[i] = make_float2(0.f, 0.f);
  for (int coil = c_begin; coil < c_end; ++coil) {
    const float2* t = a.tbuf + 2 * d.soff + ((int64_t)coil * H + rowc) * N;
    float2 v[P];
#pragma unroll
    for (int i = 0; i < Sd::GFIN; ++i)
#pragma unroll
      for (int r = 0; r < Sd::NFIN; ++r) v[i * Sd::NFIN + r] = t[Sd::freq(tc, i, r)];
    fft_inverse<Sd, L>(v, lds, tw, tc, c);
    const float2* Sr = a.S + d.soff + ((int64_t)coil * H + rowc) * W;
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i) acc[i] = cadd(acc[i], cmulc(Sr[tc + T * i], v[2 * i]));
  }
  const int64_t prow = d.xoff + (int64_t)rowc * W;
  const float2* pp = (cg && a.iter > 0) ? a.pout : a.pin;
  const float lam = (a.lam && ks == 0) ? a.lam[b] : 0.f;
  float2* qo = a.qout + (cg ? (int64_t)ks * a.qstride : 0) + prow;
  float dot = 0.f;
#pragma unroll
  for (int i = 0; i < Sd::G1; ++i) {
    const int n = tc + T * i;
    const float2 p = pp[prow + n];
    const float2 q = make_float2(acc[i].x + lam * p.x, acc[i].y + lam * p.y);
    dot += p.x * q.x + p.y * q.y;
    if (valid) qo[n] = q;
  }
  if (!valid) dot = 0.f;
  if (cg) {
    const float s = block_sum_fixed(dot, red);
    if (lid == 0) a.pq_part[(int64_t)b * a.npq + rb * a.split + ks] = s;
  }
}

// ------------------------------------------------------------- launchers
template <class Sd, int WT>
hipError_t launch_toep_rows_fwd(const ToepArgs& a, int maxH, hipStream_t s) {
  dim3 grid((unsigned)(((maxH + WT - 1) / WT) * a.split), (unsigned)a.nslices);
  hipLaunchKernelGGL((k_toep_rows_fwd<Sd, WT>), grid, dim3(Sd::T * WT), 0, s, a);
  return hipGetLastError();
}
template <class Sd, int WT>
hipError_t launch_toep_cols(const ToepArgs& a, int maxW2, hipStream_t s) {
  const int n = ((maxW2 + WT - 1) / WT) * a.split;
  dim3 grid((unsigned)(((n + 15) / 16) * 16), (unsigned)a.nslices);
  hipLaunchKernelGGL((k_toep_cols<Sd, WT>), grid, dim3(Sd::T * WT), 0, s, a);
  return hipGetLastError();
}
template <class Sd, int WT>
hipError_t launch_toep_rows_adj(const ToepArgs& a, int maxH, hipStream_t s) {
  dim3 grid((unsigned)(((maxH + WT - 1) / WT) * a.split), (unsigned)a.nslices);
  hipLaunchKernelGGL((k_toep_rows_adj<Sd, WT>), grid, dim3(Sd::T * WT), 0, s, a);
  return hipGetLastError();
}

template <class Sd, int WTR, int WTC>
struct RegistrarToep {
  RegistrarToep(const char* name) {
    ToepVariant v{Sd::N, &launch_toep_rows_fwd<Sd, WTR>, &launch_toep_cols<Sd, WTC>,
                  &launch_toep_rows_adj<Sd, WTR>, WTR, WTC, name};
    register_toep_variant(v);
  }
};

}  // namespace mrx
