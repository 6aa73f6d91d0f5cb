// Variational-network stage (Variational Network subsection, eq. update_vn):
//   x' = x - sum_i K_i^T Phi'_i(Re(k_i * x)) - lambda (A^H A x - A^H y)
// with N_k = 24 complex 11 x 11 filters (cross-correlation, zero "same"
// padding, imaginary part of the filter response discarded) and trainable
// activations Phi'_i(s) = sum_j w_ij exp(-(s - mu_j)^2 / (2 sigma^2)),
// mu_j = -1 + 2j/30, sigma = 2/30 (31 knots).  All in fp32: the activation's
// width (sigma = 1/15) turns a 2^-9 relative error of the filter response
// into a several-percent error of Phi', so bf16 operands would not hold
// parity.  The filter responses run on the fp32 matrix cores, everything
// else on the vector ALUs with the filter and RBF weights read through
// scalar loads (uniform across a wavefront); image tiles are staged in LDS.
#include "../../include/mrx.h"
#include "api_internal.h"
#include "vn.h"

namespace mrx {

constexpr int VT = 16;                 // output tile edge (16 x 16 pixels, 256 threads)
constexpr int VH = VT + 2 * VN_R;      // tile with halo
constexpr float VN_SIG = 2.0f / (VN_NW - 1);
constexpr float VN_INV2S2 = 1.0f / (2.0f * VN_SIG * VN_SIG);
typedef __attribute__((address_space(4))) float ConstF;  // read-only global memory
// The adjoint stages the activations of 12 filters at a time: a 12-float
// pixel stride puts the float4 reads of 16 consecutive pixels in distinct
// banks, and the 32 KB tile lets four workgroups share a CU.
constexpr int VNH = VN_NK / 2;

// kt[tap][i] = k_i[tap] (complex), from k[i][tap]; and the matrix-core
// operand layout wa[tap][c][32]: c = 0 Re k_i[tap], c = 1 -Im k_i[tap], for
// i < 24, zero for the padding rows 24..31.
constexpr int VN_WA = VN_TAPS * 64;  // floats of wa
__global__ void k_vn_pack(const float2* k, float2* kt, float* wa) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < VN_NK * VN_TAPS) {
    const int i = idx % VN_NK, tap = idx / VN_NK;
    kt[idx] = k[i * VN_TAPS + tap];
  }
  if (idx < VN_WA) {
    const int tap = idx / 64, c = (idx / 32) % 2, i = idx % 32;
    float v = 0.f;
    if (i < VN_NK) {
      const float2 kk = k[i * VN_TAPS + tap];
      v = c ? -kk.y : kk.x;
    }
    wa[idx] = v;
  }
}

__device__ __forceinline__ void load_ctile(float2* tile, const float2* img, int H, int W, int y0, int x0) {
  for (int p = threadIdx.x; p < VH * VH; p += 256) {
    const int gy = y0 + p / VH - VN_R, gx = x0 + p % VH - VN_R;
    float2 v = make_float2(0.f, 0.f);
    if (gy >= 0 && gy < H && gx >= 0 && gx < W) v = img[(int64_t)gy * W + gx];
    tile[p] = v;
  }
}

// A 16 x 16 tile: slice and corner
struct VnTile {
  int b, x0, y0;
};

// The Gaussian RBF in groups of 8 knots.  With knot spacing D (= sigma),
// group g's centre m = -1 + (8 g + 3.5) D and u = s - m, each of its knots
// mu = m + (k - 3.5) D (k = 0..7) gives
//   exp(-(s - mu)^2 / (2 sigma^2)) = F Q^k D_k,
//   F = exp(-c u (u + 7 D)), Q = exp(2 c D u), D_k = exp(-c D^2 (k - 3.5)^2),
// c = 1 / (2 sigma^2), so that sum_k w_k exp(...) = F P(Q) with the
// polynomial P(Q) = sum_k (w_k D_k) Q^k: two exponentials and a Horner
// scheme per 8 knots.  And sum_k w_k t_k exp(...) (t_k = s - mu_k, for
// Phi'') = F (u P(Q) - P2(Q)), P2(Q) = sum_k ((k - 3.5) D w_k D_k) Q^k.
// u is held to [-VN_UC, VN_UC]: Q^7 stays below 2^122, and beyond the bound
// every knot of the group is more than 0.56 from s, where each term is below
// exp(-35) of its weight (the held value is that small, or zero).
constexpr int VN_GK = 8;                      // knots per group
constexpr int VN_NG = (VN_NW + VN_GK - 1) / VN_GK;  // groups (the last padded with zero weights)
constexpr int VN_WD = VN_NK * 2 * VN_NG * VN_GK;    // floats of the coefficient table
constexpr float VN_UC = 0.8f;
constexpr float VN_LOG2E = 1.44269504088896341f;

// wd[i][0][8 g + k] = w_i,8g+k D_k, wd[i][1][8 g + k] = (k - 3.5) D w_i,8g+k D_k
// (zero past the last knot), from w[i][31].
__global__ void k_vn_pack_rbf(const float* w, float* wd) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= VN_WD) return;
  const int i = idx / (2 * VN_NG * VN_GK), c = (idx / (VN_NG * VN_GK)) % 2, j = idx % (VN_NG * VN_GK);
  const int k = j % VN_GK;
  float v = 0.f;
  if (j < VN_NW) {
    const double dk = (double)k - 0.5 * (VN_GK - 1);
    const double Dk = exp(-(double)VN_INV2S2 * (double)VN_SIG * (double)VN_SIG * dk * dk);
    v = (float)((double)w[i * VN_NW + j] * Dk * (c ? dk * (double)VN_SIG : 1.0));
  }
  wd[idx] = v;
}
// The activation of one pixel (pix = ly * 16 + lx of the tile) from its 24
// filter responses s (and, reverse, Kg); stores the [pixel][24] outputs.
template <bool REV>
__device__ __forceinline__ void vn_activation(const VnArgs& a, const VnTile& tl, int pix, const float (&s)[VN_NK],
                                              const float (&kg)[REV ? VN_NK : 1]) {
  const SliceDesc d = a.desc[tl.b];
  const int H = d.H, W = d.W;
  const int ly = pix / VT, lx = pix % VT;
  const int y0 = tl.y0, x0 = tl.x0;
  const int gy = y0 + ly, gx = x0 + lx;
  if (gy >= H || gx >= W) return;
  const int64_t o = (d.xoff + (int64_t)gy * W + gx) * VN_NK;
  // The kernel never writes the coefficients: read through the constant
  // address space they stay scalar loads between the output stores.
  const ConstF* wd = (const ConstF*)a.wd;
  constexpr float KF = -VN_INV2S2 * VN_LOG2E;                // F = 2^(KF u (u + 7 D))
  constexpr float KQ = 2.0f * VN_INV2S2 * VN_SIG * VN_LOG2E;  // Q = 2^(KQ u)
  constexpr float SPAN = (VN_GK - 1) * VN_SIG;
#pragma unroll
  for (int i0 = 0; i0 < VN_NK; i0 += 4) {
    float4 u4, e4, kg4, s4;
    float* pu = &u4.x;
    float* pe = &e4.x;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = i0 + k;
      float p1 = 0.f, p2 = 0.f;
#pragma unroll
      for (int g = 0; g < VN_NG; ++g) {
        const float m = -1.0f + (VN_GK * g + 0.5f * (VN_GK - 1)) * VN_SIG;
        const float u = fminf(fmaxf(s[i] - m, -VN_UC), VN_UC);
        const float F = __builtin_amdgcn_exp2f((u * KF) * (u + SPAN));
        const float Q = __builtin_amdgcn_exp2f(u * KQ);
        const ConstF* c1 = wd + (i * 2) * (VN_NG * VN_GK) + VN_GK * g;
        float P1 = c1[VN_GK - 1];
#pragma unroll
        for (int q = VN_GK - 2; q >= 0; --q) P1 = fmaf(P1, Q, c1[q]);
        p1 = fmaf(F, P1, p1);
        if constexpr (REV) {
          const ConstF* c2 = c1 + VN_NG * VN_GK;
          float P2 = c2[VN_GK - 1];
#pragma unroll
          for (int q = VN_GK - 2; q >= 0; --q) P2 = fmaf(P2, Q, c2[q]);
          p2 = fmaf(F, fmaf(u, P1, -P2), p2);
        }
      }
      pu[k] = p1;
      if constexpr (REV) pe[k] = (-2.0f * VN_INV2S2) * p2 * kg[i];
    }
    *(float4*)(a.u + o + i0) = u4;
    if constexpr (REV) {
      kg4 = make_float4(kg[i0], kg[i0 + 1], kg[i0 + 2], kg[i0 + 3]);
      s4 = make_float4(s[i0], s[i0 + 1], s[i0 + 2], s[i0 + 3]);
      *(float4*)(a.e + o + i0) = e4;
      *(float4*)(a.kg + o + i0) = kg4;
      *(float4*)(a.s + o + i0) = s4;
    }
  }
}

// Filter responses s_i = Re(k_i * x) (and Kg_i = Re(k_i * g) in the reverse
// mode) for a 16 x 16 tile, then the activation:
//   forward: u_i = Phi'_i(s_i)
//   reverse: u_i = Phi'_i(s_i), e_i = Phi''_i(s_i) * Kg_i, and Kg_i, s_i kept
// Outputs are [pixel][24] fp32 at offset xoff * 24.
//
// The responses run on the fp32 matrix cores: per tap one 32 x 32 x 2
// product D[i][j] += sum_c A[i][c] B[c][j] with A[i][c] = (Re k_i, -Im k_i)
// (filters padded to 32 rows) and B[c][j] = (Re x, Im x) at pixel j shifted
// by the tap, so every lane supplies one weight and one pixel value.  Each
// wavefront owns four rows of the tile (two 32-pixel column blocks); the
// responses go through LDS to one pixel per lane for the activation on the
// vector ALUs.
typedef float v16f __attribute__((ext_vector_type(16)));
constexpr int VMS = VN_NK + 4;  // LDS pixel stride of the transposed responses (float4 reads conflict-free)

// D layout of the 32 x 32 x 2 product: lane l holds column l % 32, and its
// register r row 8 (r / 4) + 4 (l / 32) + r % 4; rows 24..31 (r >= 12) are
// padding.  Writes the 24 real rows of a column block to ts[pixel][VMS].
__device__ __forceinline__ void vn_put(const v16f& acc, float* ts, int pix, int half) {
#pragma unroll
  for (int r = 0; r < 12; ++r) ts[pix * VMS + 8 * (r / 4) + 4 * half + (r % 4)] = acc[r];
}

// ts[pix][0..23] -> v (the wavefront's own pixels: LDS ordering within the
// wavefront suffices)
__device__ __forceinline__ void vn_take(const float* ts, int pix, float (&v)[VN_NK]) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const float4* r4 = (const float4*)&ts[pix * VMS];
#pragma unroll
  for (int q = 0; q < VN_NK / 4; ++q) {
    const float4 t = r4[q];
    v[4 * q] = t.x;
    v[4 * q + 1] = t.y;
    v[4 * q + 2] = t.z;
    v[4 * q + 3] = t.w;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool REV>
__global__ void __launch_bounds__(256) k_vn_filter(VnArgs a) {
  __shared__ float tx[2][VH * VH];  // Re, Im planes of the tile with halo
  __shared__ float tg[REV ? 2 : 1][REV ? VH * VH : 1];
  __shared__ __attribute__((aligned(16))) float ts[VT * VT * VMS];
  VnTile tl;
  tl.b = a.slices[blockIdx.z];
  tl.x0 = blockIdx.x * VT;
  tl.y0 = blockIdx.y * VT;
  const SliceDesc d = a.desc[tl.b];
  const int H = d.H, W = d.W;
  if (tl.x0 >= W || tl.y0 >= H) return;
  for (int p = threadIdx.x; p < VH * VH; p += 256) {
    const int gy = tl.y0 + p / VH - VN_R, gx = tl.x0 + p % VH - VN_R;
    const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
    const int64_t o = d.xoff + (int64_t)gy * W + gx;
    const float2 xv = in ? a.x[o] : make_float2(0.f, 0.f);
    tx[0][p] = xv.x;
    tx[1][p] = xv.y;
    if constexpr (REV) {
      const float2 gv = in ? a.g[o] : make_float2(0.f, 0.f);
      tg[0][p] = gv.x;
      tg[1][p] = gv.y;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int half = lane >> 5, j = lane & 31;
  // column block nb holds tile pixels 64 wv + 32 nb + j: row 4 wv + 2 nb + j / 16, column j % 16
  const int t0 = (4 * wv + j / 16) * VH + j % 16;
  const float* px = tx[half];
  const float* pg = tg[REV ? half : 0];
  v16f s0 = {}, s1 = {}, g0 = {}, g1 = {};
  const float* wa = a.wa + half * 32 + j;
#pragma unroll 1
  for (int dy = 0; dy < VN_KS; ++dy) {
    float wr[VN_KS];
#pragma unroll
    for (int dx = 0; dx < VN_KS; ++dx) wr[dx] = wa[(dy * VN_KS + dx) * 64];
#pragma unroll
    for (int dx = 0; dx < VN_KS; ++dx) {
      const int tp = t0 + dy * VH + dx;
      s0 = __builtin_amdgcn_mfma_f32_32x32x2f32(wr[dx], px[tp], s0, 0, 0, 0);
      s1 = __builtin_amdgcn_mfma_f32_32x32x2f32(wr[dx], px[tp + 2 * VH], s1, 0, 0, 0);
      if constexpr (REV) {
        g0 = __builtin_amdgcn_mfma_f32_32x32x2f32(wr[dx], pg[tp], g0, 0, 0, 0);
        g1 = __builtin_amdgcn_mfma_f32_32x32x2f32(wr[dx], pg[tp + 2 * VH], g1, 0, 0, 0);
      }
    }
  }
  // one pixel per lane (pixel = threadIdx.x: the wavefront's own 64 pixels)
  float s[VN_NK], kg[REV ? VN_NK : 1];
  vn_put(s0, ts, 64 * wv + j, half);
  vn_put(s1, ts, 64 * wv + 32 + j, half);
  vn_take(ts, threadIdx.x, s);
  if constexpr (REV) {
    vn_put(g0, ts, 64 * wv + j, half);
    vn_put(g1, ts, 64 * wv + 32 + j, half);
    vn_take(ts, threadIdx.x, kg);
  }
  vn_activation<REV>(a, tl, threadIdx.x, s, kg);
}

// r = K^T v (v: [pixel][24] fp32) for a 16 x 16 tile, fused with the update
//   forward: out = x - r - lambda (q - aHy)        (q = A^H A x)
//   reverse: out = g - r - lambda q                (q = A^H A g)
// and, in the reverse mode, per-workgroup partials of Re<g, qx - aHy>.
template <bool REV>
__global__ void __launch_bounds__(256) k_vn_adjoint(VnArgs a) {
  __shared__ __attribute__((aligned(16))) float tv[VH * VH * VNH];  // [pixel][12]: one half of the filters
  __shared__ float red[4];
  const int b = a.slices[blockIdx.z];
  const SliceDesc d = a.desc[b];
  const int H = d.H, W = d.W;
  const int x0 = blockIdx.x * VT, y0 = blockIdx.y * VT;
  const int wgid = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  float lam_part = 0.f;
  if (x0 < W && y0 < H) {
    const float* v = REV ? a.e : a.u;
    const int ly = threadIdx.x / VT, lx = threadIdx.x % VT;
    // four partial sums per component (filter index mod 4), added at the end
    float ra[4] = {0.f, 0.f, 0.f, 0.f}, ia[4] = {0.f, 0.f, 0.f, 0.f};
    for (int h = 0; h < 2; ++h) {
      if (h) __syncthreads();  // every read of the first half is done
      // three float4 chunks per pixel
      for (int q = threadIdx.x; q < VH * VH * (VNH / 4); q += 256) {
        const int p = q / (VNH / 4), k = q % (VNH / 4);
        const int gy = y0 + p / VH - VN_R, gx = x0 + p % VH - VN_R;
        float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gy >= 0 && gy < H && gx >= 0 && gx < W)
          val = *(const float4*)(v + (d.xoff + (int64_t)gy * W + gx) * VN_NK + h * VNH + 4 * k);
        *(float4*)&tv[p * VNH + 4 * k] = val;
      }
      __syncthreads();
      // s[p] used x[p + d] => adjoint gathers v[p - d]
      for (int dy = 0; dy < VN_KS; ++dy) {
        for (int dx = 0; dx < VN_KS; ++dx) {
          const int tap = dy * VN_KS + dx;
          const int tp = (ly + 2 * VN_R - dy) * VH + lx + 2 * VN_R - dx;
          const float2* kt = a.kt + tap * VN_NK + h * VNH;
          const float4* t4 = (const float4*)&tv[tp * VNH];  // the 12 values of pixel tp: 3 reads
#pragma unroll
          for (int k = 0; k < VNH / 4; ++k) {
            const float4 v4 = t4[k];
            const float vs[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              const float2 kk = kt[4 * k + m];
              ra[m] = fmaf(kk.x, vs[m], ra[m]);
              ia[m] = fmaf(-kk.y, vs[m], ia[m]);
            }
          }
        }
      }
    }
    const float rr = (ra[0] + ra[1]) + (ra[2] + ra[3]), ri = (ia[0] + ia[1]) + (ia[2] + ia[3]);
    const int gy = y0 + ly, gx = x0 + lx;
    if (gy < H && gx < W) {
      const int64_t o = d.xoff + (int64_t)gy * W + gx;
      const float lam = a.lam[0];
      const float2 q = a.q[o];
      if constexpr (!REV) {
        const float2 xv = a.x[o], ay = a.aHy[o];
        a.out[o] = make_float2(xv.x - rr - lam * (q.x - ay.x), xv.y - ri - lam * (q.y - ay.y));
      } else {
        const float2 gv = a.g[o];
        a.out[o] = make_float2(gv.x - rr - lam * q.x, gv.y - ri - lam * q.y);
        const float2 qx = a.qx[o], ay = a.aHy[o];
        lam_part = -(gv.x * (qx.x - ay.x) + gv.y * (qx.y - ay.y));
      }
    }
  }
  if constexpr (REV) {
    float v = lam_part;
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) a.part_lam[wgid] = red[0] + red[1] + red[2] + red[3];
  }
}

// Filter gradients of one stage (reverse mode):
//   dkr_i[d] = -sum_p (u_i[p] Re g[p+d] + e_i[p] Re x[p+d])
//   dki_i[d] = +sum_p (u_i[p] Im g[p+d] + e_i[p] Im x[p+d])
// One workgroup per (band of VN_KBAND rows, slice), 256 threads: thread t
// owns tap t % 128 (< 121) for the 12 filters of half t / 128, with 24
// accumulators; 64-column chunks keep the LDS small (25 KB) so that many
// workgroups share a CU.  Partials per workgroup, summed by k_vn_reduce.
constexpr int VN_KBAND = 2;
constexpr int VKC = 64;  // columns per chunk
__global__ void __launch_bounds__(256) k_vn_kgrad(VnArgs a) {
  constexpr int RW = VKC + 2 * VN_R;
  constexpr int NH = VN_NK / 2;
  __shared__ float2 rowg[VN_KS * RW];
  __shared__ float2 rowx[VN_KS * RW];
  __shared__ __attribute__((aligned(16))) float uv[VKC * VN_NK];
  __shared__ __attribute__((aligned(16))) float ev[VKC * VN_NK];
  const int wg = blockIdx.y * gridDim.x + blockIdx.x;
  float* part = a.part_k + (int64_t)wg * (VN_NK * VN_TAPS * 2);
  const int b = a.slices[blockIdx.y];
  const SliceDesc d = a.desc[b];
  const int H = d.H, W = d.W;
  const int tap = threadIdx.x & 127, fh = __builtin_amdgcn_readfirstlane(threadIdx.x >> 7);
  const int dy = tap / VN_KS, dx = tap % VN_KS;
  float ar[NH], ai[NH];
#pragma unroll
  for (int i = 0; i < NH; ++i) { ar[i] = 0.f; ai[i] = 0.f; }
  for (int rr = 0; rr < VN_KBAND; ++rr) {
    const int row = blockIdx.x * VN_KBAND + rr;
    if (row >= H) break;
    for (int c0 = 0; c0 < W; c0 += VKC) {
      const int cw = min(VKC, W - c0);
      __syncthreads();
      // rows row-5 .. row+5 of g and x, columns c0-5 .. c0+cw+4
      for (int q = threadIdx.x; q < VN_KS * RW; q += 256) {
        const int r = q / RW, c = q % RW;
        const int gy = row + r - VN_R, gx = c0 + c - VN_R;
        float2 gv = make_float2(0.f, 0.f), xv = make_float2(0.f, 0.f);
        if (c < cw + 2 * VN_R && gy >= 0 && gy < H && gx >= 0 && gx < W) {
          gv = a.g[d.xoff + (int64_t)gy * W + gx];
          xv = a.x[d.xoff + (int64_t)gy * W + gx];
        }
        rowg[q] = gv;
        rowx[q] = xv;
      }
      for (int q = threadIdx.x; q < cw * VN_NK; q += 256) {
        const int64_t o = (d.xoff + (int64_t)row * W + c0) * VN_NK + q;
        uv[q] = a.u[o];
        ev[q] = a.e[o];
      }
      __syncthreads();
      if (tap < VN_TAPS) {
        for (int c = 0; c < cw; ++c) {
          const int tp = dy * RW + c + dx;
          const float2 gv = rowg[tp], xv = rowx[tp];
          const float4* u4 = (const float4*)&uv[c * VN_NK + fh * NH];
          const float4* e4 = (const float4*)&ev[c * VN_NK + fh * NH];
#pragma unroll
          for (int k = 0; k < NH / 4; ++k) {
            const float4 u = u4[k], e = e4[k];
            const float us[4] = {u.x, u.y, u.z, u.w}, es[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              ar[4 * k + m] = fmaf(us[m], gv.x, fmaf(es[m], xv.x, ar[4 * k + m]));
              ai[4 * k + m] = fmaf(us[m], gv.y, fmaf(es[m], xv.y, ai[4 * k + m]));
            }
          }
        }
      }
    }
  }
  if (tap < VN_TAPS) {
#pragma unroll
    for (int k = 0; k < NH; ++k) {
      const int i = fh * NH + k;
      part[(i * VN_TAPS + tap) * 2 + 0] = -ar[k];
      part[(i * VN_TAPS + tap) * 2 + 1] = ai[k];
    }
  }
}

// RBF-weight gradients: dw_ij = -sum_p Kg_i[p] exp(-(s_i[p] - mu_j)^2 / (2 sigma^2)).
// One workgroup per (band, slice).  The knots go in the groups of 8 of the
// activation (F Q^k D_k per knot): thread t takes filter i and group g
// (t % 96) on pixel lane t / 96 (every eighth pixel of a chunk), sums
// Kg F Q^k for its 8 knots with two exponentials per pixel, and the 8
// lanes are added in order at the end; D_k multiplies the sums.  A chunk of
// up to 256 columns is staged filter-major ([24][260]).
constexpr int VWC = 256;      // columns per chunk
constexpr int VWS = VWC + 4;  // LDS row stride (floats)
constexpr int VW_PAIRS = VN_NK * VN_NG;  // (filter, group) pairs
constexpr int VW_LANES = 8;              // pixel lanes
static_assert(VW_PAIRS * VW_LANES == 768 && VW_PAIRS * VN_GK * VW_LANES <= VN_NK * VWS, "wgrad layout");
__global__ void __launch_bounds__(768) k_vn_wgrad(VnArgs a) {
  __shared__ float sv[VN_NK * VWS];  // (reused for the lane sums at the end)
  __shared__ float gv[VN_NK * VWS];
  const int wg = blockIdx.y * gridDim.x + blockIdx.x;
  float* part = a.part_w + (int64_t)wg * (VN_NK * VN_NW);
  const int b = a.slices[blockIdx.y];
  const SliceDesc d = a.desc[b];
  const int H = d.H, W = d.W;
  const int t = threadIdx.x, pl = t / VW_PAIRS, ig = t % VW_PAIRS;
  const int i = ig / VN_NG, g = ig % VN_NG;
  const float m = -1.0f + (VN_GK * g + 0.5f * (VN_GK - 1)) * VN_SIG;
  constexpr float KF = -VN_INV2S2 * VN_LOG2E;
  constexpr float KQ = 2.0f * VN_INV2S2 * VN_SIG * VN_LOG2E;
  constexpr float SPAN = (VN_GK - 1) * VN_SIG;
  float acc[VN_GK];
#pragma unroll
  for (int k = 0; k < VN_GK; ++k) acc[k] = 0.f;
  for (int rr = 0; rr < VN_BAND; ++rr) {
    const int row = blockIdx.x * VN_BAND + rr;
    if (row >= H) break;
    for (int c0 = 0; c0 < W; c0 += VWC) {
      const int cw = min(VWC, W - c0);
      __syncthreads();
      for (int q = t; q < cw * VN_NK; q += 768) {
        const int c = q / VN_NK, ii = q % VN_NK;
        const int64_t o = (d.xoff + (int64_t)row * W + c0) * VN_NK + q;
        sv[ii * VWS + c] = a.s[o];
        gv[ii * VWS + c] = a.kg[o];
      }
      __syncthreads();
      for (int c = pl; c < cw; c += VW_LANES) {
        const float u = fminf(fmaxf(sv[i * VWS + c] - m, -VN_UC), VN_UC);
        const float F = __builtin_amdgcn_exp2f((u * KF) * (u + SPAN));
        const float Q = __builtin_amdgcn_exp2f(u * KQ);
        float tt = gv[i * VWS + c] * F;
        acc[0] += tt;
#pragma unroll
        for (int k = 1; k < VN_GK; ++k) {
          tt *= Q;
          acc[k] += tt;
        }
      }
    }
  }
  __syncthreads();
  float* red = sv;  // [lane][pair][8]
#pragma unroll
  for (int k = 0; k < VN_GK; ++k) red[(pl * VW_PAIRS + ig) * VN_GK + k] = acc[k];
  __syncthreads();
  if (t < VN_NK * VN_NW) {
    const int fi = t / VN_NW, j = t % VN_NW, gg = j / VN_GK, k = j % VN_GK;
    float sum = 0.f;
    for (int l = 0; l < VW_LANES; ++l) sum += red[(l * VW_PAIRS + fi * VN_NG + gg) * VN_GK + k];
    const double dk = (double)k - 0.5 * (VN_GK - 1);
    const float Dk = (float)exp(-(double)VN_INV2S2 * (double)VN_SIG * (double)VN_SIG * dk * dk);
    part[t] = -Dk * sum;
  }
}

// out[i] (+)= sum_s part[s][i] in a fixed order: a block takes 64 entries;
// its 16 waves sum the slots s = w, w + 16, ... in increasing order, then
// the 16 wave sums are added in wave order.
constexpr int VR_WAVES = 16;
__global__ void __launch_bounds__(64 * VR_WAVES) k_vn_reduce(const float* part, int nslots, int nout, float* out,
                                                            int accumulate) {
  __shared__ float red[VR_WAVES][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  float s = 0.f;
  if (i < nout)
    for (int k = wv; k < nslots; k += VR_WAVES) s += part[(int64_t)k * nout + i];
  red[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && i < nout) {
    float t = red[0][lane];
#pragma unroll
    for (int w = 1; w < VR_WAVES; ++w) t += red[w][lane];
    out[i] = accumulate ? out[i] + t : t;
  }
}

}  // namespace mrx

using namespace mrx;

namespace {

mrx_status vn_ready(mrx_plan_s* p, const char* who) {
  if (!p->ws) return fail(MRX_ENOWORKSPACE, std::string(who) + ": workspace not set");
  if (!(p->flags & MRX_PLAN_VN)) return fail(MRX_ENOWORKSPACE, std::string(who) + ": plan needs MRX_PLAN_VN");
  return MRX_OK;
}

VnArgs vn_args(mrx_plan_s* p, const mrx_vn_params* prm) {
  VnArgs a{};
  a.desc = p->d_desc;
  a.slices = p->d_all;
  a.nslices = p->B;
  a.kt = (const float2*)(p->ws + p->ws_vn_kt);
  a.wa = (const float*)(p->ws + p->ws_vn_wa);
  a.wd = (const float*)(p->ws + p->ws_vn_wd);
  a.w = prm->w;
  a.lam = prm->lam;
  a.u = (float*)(p->ws + p->ws_vn_u);
  a.e = (float*)(p->ws + p->ws_vn_e);
  a.kg = (float*)(p->ws + p->ws_vn_kg);
  a.s = (float*)(p->ws + p->ws_vn_s);
  a.part_lam = (float*)(p->ws + p->ws_vn_plam);
  a.part_k = (float*)(p->ws + p->ws_vn_pk);
  a.part_w = (float*)(p->ws + p->ws_vn_pw);
  return a;
}

}  // namespace

namespace mrx {

size_t vn_workspace_bytes(mrx_plan_s* p, size_t base) {
  if (!(p->flags & MRX_PLAN_VN)) return 0;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t ni = (size_t)p->n_image;
  size_t w = 0;
  auto take = [&](size_t bytes) { size_t o = base + w; w += al(bytes); return o; };
  p->ws_vn_kt = take(sizeof(float2) * VN_NK * VN_TAPS);
  p->ws_vn_wa = take(sizeof(float) * VN_WA);
  p->ws_vn_wd = take(sizeof(float) * VN_WD);
  p->ws_vn_u = take(ni * VN_NK * 4);
  p->ws_vn_e = take(ni * VN_NK * 4);
  p->ws_vn_kg = take(ni * VN_NK * 4);
  p->ws_vn_s = take(ni * VN_NK * 4);
  p->ws_vn_qx = take(ni * 8);
  p->ws_vn_qg = take(ni * 8);
  const size_t tiles = (size_t)((p->maxW + VT - 1) / VT) * ((p->maxH + VT - 1) / VT) * p->B;
  p->ws_vn_plam = take(tiles * 4);
  const size_t bands = (size_t)((p->maxH + VN_BAND - 1) / VN_BAND) * p->B;
  const size_t kbands = (size_t)((p->maxH + VN_KBAND - 1) / VN_KBAND) * p->B;
  p->ws_vn_pk = take(kbands * VN_NK * VN_TAPS * 2 * 4);
  p->ws_vn_pw = take(bands * VN_NK * VN_NW * 4);
  return w;
}

}  // namespace mrx

extern "C" {

mrx_status mrx_vn_stage(mrx_plan p, const float* x, const float* aHy, const float* S, const float* mask,
                        const mrx_vn_params* prm, float* x_next, void* stream) {
  if (!p || !prm) return fail(MRX_EINVAL, "vn_stage: null argument");
  if (!x || !aHy || !S || !mask || !x_next || !prm->k || !prm->w || !prm->lam)
    return fail(MRX_EINVAL, "vn_stage: null data pointer");
  if (x == x_next) return fail(MRX_EINVAL, "vn_stage: x and x_next must not alias");
  mrx_status st = vn_ready(p, "vn_stage");
  if (st != MRX_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  VnArgs a = vn_args(p, prm);
  float2* q = (float2*)(p->ws + p->ws_vn_qx);
  hipLaunchKernelGGL(k_vn_pack, dim3((VN_WA + 255) / 256), dim3(256), 0, s, (const float2*)prm->k,
                     (float2*)(p->ws + p->ws_vn_kt), (float*)(p->ws + p->ws_vn_wa));
  hipLaunchKernelGGL(k_vn_pack_rbf, dim3((VN_WD + 255) / 256), dim3(256), 0, s, prm->w,
                     (float*)(p->ws + p->ws_vn_wd));
  st = normal_impl(p, (const float2*)x, (const float2*)S, mask, nullptr, q, s);
  if (st != MRX_OK) return st;
  a.x = (const float2*)x;
  a.aHy = (const float2*)aHy;
  a.q = q;
  a.out = (float2*)x_next;
  dim3 grid((p->maxW + VT - 1) / VT, (p->maxH + VT - 1) / VT, p->B);
  {
    KernelTimer kt(p, MRX_KERNEL_VN_FILTER, s);
    hipLaunchKernelGGL(k_vn_filter<false>, grid, dim3(256), 0, s, a);
  }
  {
    KernelTimer kt(p, MRX_KERNEL_VN_ADJOINT, s);
    hipLaunchKernelGGL(k_vn_adjoint<false>, grid, dim3(256), 0, s, a);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MRX_OK : hip_fail(e, "vn_stage");
}

mrx_status mrx_vn_stage_backward(mrx_plan p, const float* g, const float* x, const float* aHy, const float* S,
                                 const float* mask, const mrx_vn_params* prm, float* g_x, float* g_k, float* g_w,
                                 float* g_lam, int32_t accumulate, void* stream) {
  if (!p || !prm) return fail(MRX_EINVAL, "vn_stage_backward: null argument");
  if (!g || !x || !aHy || !S || !mask || !g_x || !g_k || !g_w || !g_lam || !prm->k || !prm->w || !prm->lam)
    return fail(MRX_EINVAL, "vn_stage_backward: null data pointer");
  if (g == g_x) return fail(MRX_EINVAL, "vn_stage_backward: g and g_x must not alias");
  mrx_status st = vn_ready(p, "vn_stage_backward");
  if (st != MRX_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  VnArgs a = vn_args(p, prm);
  float2* qx = (float2*)(p->ws + p->ws_vn_qx);
  float2* qg = (float2*)(p->ws + p->ws_vn_qg);
  hipLaunchKernelGGL(k_vn_pack, dim3((VN_WA + 255) / 256), dim3(256), 0, s, (const float2*)prm->k,
                     (float2*)(p->ws + p->ws_vn_kt), (float*)(p->ws + p->ws_vn_wa));
  hipLaunchKernelGGL(k_vn_pack_rbf, dim3((VN_WD + 255) / 256), dim3(256), 0, s, prm->w,
                     (float*)(p->ws + p->ws_vn_wd));
  st = normal_impl(p, (const float2*)x, (const float2*)S, mask, nullptr, qx, s);
  if (st == MRX_OK) st = normal_impl(p, (const float2*)g, (const float2*)S, mask, nullptr, qg, s);
  if (st != MRX_OK) return st;
  a.x = (const float2*)x;
  a.g = (const float2*)g;
  a.aHy = (const float2*)aHy;
  a.q = qg;
  a.qx = qx;
  a.out = (float2*)g_x;
  dim3 grid((p->maxW + VT - 1) / VT, (p->maxH + VT - 1) / VT, p->B);
  const int tiles = grid.x * grid.y * grid.z;
  {
    KernelTimer kt(p, MRX_KERNEL_VN_FILTER_REV, s);
    hipLaunchKernelGGL(k_vn_filter<true>, grid, dim3(256), 0, s, a);
  }
  {
    KernelTimer kt(p, MRX_KERNEL_VN_ADJOINT, s);
    hipLaunchKernelGGL(k_vn_adjoint<true>, grid, dim3(256), 0, s, a);
  }
  const int bands = (p->maxH + VN_BAND - 1) / VN_BAND;
  const int kbands = (p->maxH + VN_KBAND - 1) / VN_KBAND;
  {
    KernelTimer kt(p, MRX_KERNEL_VN_KGRAD, s);
    hipLaunchKernelGGL(k_vn_kgrad, dim3(kbands, p->B), dim3(256), 0, s, a);
  }
  hipLaunchKernelGGL(k_vn_wgrad, dim3(bands, p->B), dim3(768), 0, s, a);
  const int nk = VN_NK * VN_TAPS * 2, nw = VN_NK * VN_NW;
  const dim3 rb(64 * VR_WAVES);
  hipLaunchKernelGGL(k_vn_reduce, dim3((nk + 63) / 64), rb, 0, s, a.part_k, kbands * p->B, nk, g_k, accumulate);
  hipLaunchKernelGGL(k_vn_reduce, dim3((nw + 63) / 64), rb, 0, s, a.part_w, bands * p->B, nw, g_w, accumulate);
  hipLaunchKernelGGL(k_vn_reduce, dim3(1), rb, 0, s, a.part_lam, tiles, 1, g_lam, accumulate);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MRX_OK : hip_fail(e, "vn_stage_backward");
}

}  // extern "C"
