// Weight and bias gradients of the denoiser's 3x3 convolutions
//   dW[co][ci][tap] = sum_p g[p][co] * a[p + d(tap)][ci],   db[co] = sum_p g[p][co]
// as MFMA products with the pixel index as the reduction (K) dimension.  Tiles
// of WG_ROWS rows x 32 columns are staged in LDS channel-major ([channel][pixel]),
// so a fragment of 8 consecutive pixels of one channel is one 16-byte read.
// Every workgroup writes its partial sums to its own slot; a second kernel
// adds the slots in a fixed order (deterministic, no float atomics).
#include "conv.h"
#include "wgrad.h"

namespace mrx {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

__device__ __forceinline__ uint16_t f2bf_w(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f_w(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ bf16x8 as_bf(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

constexpr int RT = WG_ROWS;             // rows per tile
constexpr int TPX = RT * 32;            // pixels per tile

// gT[ch][p] = g[tile pixel p][ch] for 64-channel bf16 NHWC g (zero outside).
// All of a thread's loads are issued before its LDS writes.
__device__ __forceinline__ void fill_gT(uint16_t* gT, const uint16_t* g, int H, int W, int row0, int col0) {
  constexpr int PER = (TPX * 8 + 255) / 256;
  uint4 v[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int q = threadIdx.x + 256 * j;
    const int p = q % TPX, ch = q / TPX;
    const int gy = row0 + p / 32, gx = col0 + p % 32;
    v[j] = make_uint4(0, 0, 0, 0);
    if (q < TPX * 8 && gy < H && gx < W) v[j] = *(const uint4*)(g + ((int64_t)gy * W + gx) * CNN_F + ch * 8);
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int q = threadIdx.x + 256 * j;
    if (q >= TPX * 8) break;
    const int p = q % TPX, ch = q / TPX;
    const uint16_t* h = (const uint16_t*)&v[j];
#pragma unroll
    for (int e = 0; e < 8; ++e) gT[(ch * 8 + e) * TPX + p] = h[e];
  }
}

// aT[dx][ch][r * 32 + c] = a[row0 - 1 + r][col0 + c + dx - 1][ch], r < RT + 2:
// every pixel of the (RT + 2) x 34 halo tile is loaded once and written to
// the (up to three) column-shifted copies that use it.
__device__ __forceinline__ void fill_aT3(uint16_t* aT, const uint16_t* a, int H, int W, int row0, int col0) {
  constexpr int HP = (RT + 2) * 32;
  constexpr int NQ = (RT + 2) * 34 * 8;
  constexpr int PER = (NQ + 255) / 256;
  uint4 v[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int q = threadIdx.x + 256 * j;
    const int hp = q % ((RT + 2) * 34), ch = q / ((RT + 2) * 34);
    const int r = hp / 34, hx = hp % 34;
    const int gy = row0 - 1 + r, gx = col0 - 1 + hx;
    v[j] = make_uint4(0, 0, 0, 0);
    if (q < NQ && gy >= 0 && gy < H && gx >= 0 && gx < W)
      v[j] = *(const uint4*)(a + ((int64_t)gy * W + gx) * CNN_F + ch * 8);
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int q = threadIdx.x + 256 * j;
    if (q >= NQ) break;
    const int hp = q % ((RT + 2) * 34), ch = q / ((RT + 2) * 34);
    const int r = hp / 34, hx = hp % 34;
    const uint16_t* h = (const uint16_t*)&v[j];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      const int c = hx - dx;
      if (c < 0 || c >= 32) continue;
#pragma unroll
      for (int e = 0; e < 8; ++e) aT[(dx * 64 + ch * 8 + e) * HP + r * 32 + c] = h[e];
    }
  }
}

// Sum of the 8 bf16 values of a fragment, in fp32, in index order.
__device__ __forceinline__ float frag_sum(uint4 v) {
  const uint16_t* h = (const uint16_t*)&v;
  float s = 0.f;
#pragma unroll
  for (int e = 0; e < 8; ++e) s += bf2f_w(h[e]);
  return s;
}

// ------------------------------------------------------------ 64 -> 64
__global__ void __launch_bounds__(256) k_wgrad_mid(WgradArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t gT[64 * TPX];
  __shared__ __attribute__((aligned(16))) uint16_t aT[3 * 64 * (RT + 2) * 32];
  const int slot = blockIdx.y * gridDim.x + blockIdx.x;
  float* part = a.partial + (int64_t)slot * a.nout;
  const int b = a.slices[blockIdx.y];
  const SliceDesc d = a.desc[b];
  const int H = d.H, W = d.W;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int mb = wv >> 1, nb = wv & 1;
  f32x16 acc[9];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[t][v] = 0.f;
  float bsum = 0.f;
  const uint16_t* g = a.g + d.xoff * CNN_F;
  const uint16_t* act = a.act + d.xoff * CNN_F;
  const int band0 = blockIdx.x * WG_BAND;
  for (int rt = 0; rt < WG_BAND / RT; ++rt) {
    const int row0 = band0 + rt * RT;
    if (row0 >= H) break;
    for (int col0 = 0; col0 < W; col0 += 32) {
      __syncthreads();
      fill_gT(gT, g, H, W, row0, col0);
      fill_aT3(aT, act, H, W, row0, col0);
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < TPX / 16; ++ks) {
        const int r = ks >> 1, c = (ks & 1) * 16 + (lane >> 5) * 8;
        const uint4 araw = *(const uint4*)&gT[(mb * 32 + (lane & 31)) * TPX + r * 32 + c];
        const bf16x8 av = as_bf(araw);
        // bias gradient of channel mb * 32 + lane % 32: this lane's 8 pixels
        if (nb == 0) bsum += frag_sum(araw);
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
          const int dy = tap / 3, dx = tap % 3;
          const bf16x8 bv = as_bf(*(const uint4*)&aT[(dx * 64 + nb * 32 + (lane & 31)) * ((RT + 2) * 32) +
                                                     (r + dy) * 32 + c]);
          acc[tap] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[tap], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int tap = 0; tap < 9; ++tap)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int co = mb * 32 + 8 * (v >> 2) + (lane >> 5) * 4 + (v & 3);
      const int ci = nb * 32 + (lane & 31);
      part[(co * 64 + ci) * 9 + tap] = acc[tap][v];
    }
  // lanes l and l + 32 hold the two pixel halves of channel mb * 32 + l % 32
  bsum += __shfl_xor(bsum, 32, 64);
  if (nb == 0 && lane < 32) part[64 * 64 * 9 + mb * 32 + lane] = bsum;
}

// ------------------------------------------------------------- 2 -> 64
// dW1[co][ci][tap] with N = (tap, ci) = 18 padded to 32; waves split
// (co block) x (k-step parity); each parity has its own partial slot.
__global__ void __launch_bounds__(256) k_wgrad_first(WgradArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t gT[64 * TPX];
  __shared__ uint16_t xT[2 * (RT + 2) * 34];
  const int wg = blockIdx.y * gridDim.x + blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int mb = wv & 1, par = wv >> 1;
  float* part = a.partial + (int64_t)(wg * 2 + par) * a.nout;
  const int b = a.slices[blockIdx.y];
  const SliceDesc d = a.desc[b];
  const int H = d.H, W = d.W;
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  float bsum = 0.f;
  const uint16_t* g = a.g + d.xoff * CNN_F;
  const float2* x = a.x + d.xoff;
  const int j = lane & 31;
  const int tap = j >> 1, ci = j & 1;
  const int dy = tap / 3, dx = tap % 3;
  const int band0 = blockIdx.x * WG_BAND;
  for (int rt = 0; rt < WG_BAND / RT; ++rt) {
    const int row0 = band0 + rt * RT;
    if (row0 >= H) break;
    for (int col0 = 0; col0 < W; col0 += 32) {
      __syncthreads();
      fill_gT(gT, g, H, W, row0, col0);
      for (int p = threadIdx.x; p < (RT + 2) * 34; p += 256) {
        const int gy = row0 - 1 + p / 34, gx = col0 - 1 + p % 34;
        float2 v = make_float2(0.f, 0.f);
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) v = x[(int64_t)gy * W + gx];
        xT[p] = f2bf_w(v.x);
        xT[(RT + 2) * 34 + p] = f2bf_w(v.y);
      }
      __syncthreads();
#pragma unroll
      for (int ks = par; ks < TPX / 16; ks += 2) {
        const int r = ks >> 1, c = (ks & 1) * 16 + (lane >> 5) * 8;
        const uint4 araw = *(const uint4*)&gT[(mb * 32 + (lane & 31)) * TPX + r * 32 + c];
        const bf16x8 av = as_bf(araw);
        bsum += frag_sum(araw);  // bias gradient, this parity's pixels
        uint4 raw;
        uint16_t* h = (uint16_t*)&raw;
#pragma unroll
        for (int e = 0; e < 8; ++e)
          h[e] = (j < 18) ? xT[ci * (RT + 2) * 34 + (r + dy) * 34 + c + e + dx] : (uint16_t)0;
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, as_bf(raw), acc, 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int co = mb * 32 + 8 * (v >> 2) + (lane >> 5) * 4 + (v & 3);
    if (j < 18) part[(co * 2 + ci) * 9 + tap] = acc[v];
  }
  bsum += __shfl_xor(bsum, 32, 64);
  if (lane < 32) part[64 * 2 * 9 + mb * 32 + lane] = bsum;
}

// ------------------------------------------------------------- 64 -> 2
// dW5[co][ci][tap] = sum_q g5[q - d][co] a4[q][ci]; M = (tap, co) = 18 padded
// to 32, N = ci (two blocks); waves split (ci block) x (k-step parity).
__global__ void __launch_bounds__(256) k_wgrad_last(WgradArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t aT[64 * TPX];
  __shared__ uint16_t gH[2 * (RT + 2) * 34];
  const int wg = blockIdx.y * gridDim.x + blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nb = wv & 1, par = wv >> 1;
  float* part = a.partial + (int64_t)(wg * 2 + par) * a.nout;
  const int b = a.slices[blockIdx.y];
  const SliceDesc d = a.desc[b];
  const int H = d.H, W = d.W;
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  float bs0 = 0.f, bs1 = 0.f;
  const float2* g5 = a.x + d.xoff;  // complex gradient of the network output
  const uint16_t* act = a.act + d.xoff * CNN_F;
  const int i = lane & 31;
  const int tap = i >> 1, co = i & 1;
  const int dy = tap / 3, dx = tap % 3;
  const int band0 = blockIdx.x * WG_BAND;
  for (int rt = 0; rt < WG_BAND / RT; ++rt) {
    const int row0 = band0 + rt * RT;
    if (row0 >= H) break;
    for (int col0 = 0; col0 < W; col0 += 32) {
      __syncthreads();
      fill_gT(aT, act, H, W, row0, col0);
      for (int p = threadIdx.x; p < (RT + 2) * 34; p += 256) {
        const int gy = row0 - 1 + p / 34, gx = col0 - 1 + p % 34;
        float2 v = make_float2(0.f, 0.f);
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) v = g5[(int64_t)gy * W + gx];
        gH[p] = f2bf_w(v.x);
        gH[(RT + 2) * 34 + p] = f2bf_w(v.y);
      }
      __syncthreads();
      if (threadIdx.x < TPX) {  // bias gradient from the fp32 output gradient
        const int gy = row0 + threadIdx.x / 32, gx = col0 + threadIdx.x % 32;
        if (gy < H && gx < W) {
          const float2 v = g5[(int64_t)gy * W + gx];
          bs0 += v.x;
          bs1 += v.y;
        }
      }
#pragma unroll
      for (int ks = par; ks < TPX / 16; ks += 2) {
        const int r = ks >> 1, c = (ks & 1) * 16 + (lane >> 5) * 8;
        uint4 raw;
        uint16_t* h = (uint16_t*)&raw;
        // q - d in halo coordinates: (r + 2 - dy, c + e + 2 - dx)
#pragma unroll
        for (int e = 0; e < 8; ++e)
          h[e] = (i < 18) ? gH[co * (RT + 2) * 34 + (r + 2 - dy) * 34 + c + e + 2 - dx] : (uint16_t)0;
        const bf16x8 bv = as_bf(*(const uint4*)&aT[(nb * 32 + (lane & 31)) * TPX + r * 32 + c]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(raw), bv, acc, 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int ii = 8 * (v >> 2) + (lane >> 5) * 4 + (v & 3);
    const int ci = nb * 32 + (lane & 31);
    if (ii < 18) part[((ii & 1) * 64 + ci) * 9 + (ii >> 1)] = acc[v];
  }
  // threads 0..63 (wave 0: par 0) hold per-position sums; fixed butterfly
  if (wv == 0) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      bs0 += __shfl_xor(bs0, off, 64);
      bs1 += __shfl_xor(bs1, off, 64);
    }
  }
  // slot (wg, par 0) carries the bias sums, slot (wg, par 1) zeros
  if (wv == 0 && lane == 0) {
    part[2 * 64 * 9 + 0] = bs0;
    part[2 * 64 * 9 + 1] = bs1;
  }
  if (wv == 2 && lane == 0) {
    part[2 * 64 * 9 + 0] = 0.f;
    part[2 * 64 * 9 + 1] = 0.f;
  }
}

// out[i] (+)= sum_s partial[s][i] over nslots slots in a fixed order: a
// block takes 64 outputs; its 4 waves sum the slots s = w, w + 4, ... in
// increasing order, then the 4 wave sums are added in wave order.
__global__ void __launch_bounds__(256) k_wgrad_reduce(const float* partial, int nslots, int nout, float* w_out,
                                                      float* b_out, int nweights, int accumulate) {
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  float s = 0.f;
  if (i < nout) {
    int k = wv;
    for (; k + 12 < nslots; k += 16) {
      const float a0 = partial[(int64_t)k * nout + i], a1 = partial[(int64_t)(k + 4) * nout + i];
      const float a2 = partial[(int64_t)(k + 8) * nout + i], a3 = partial[(int64_t)(k + 12) * nout + i];
      s += a0; s += a1; s += a2; s += a3;
    }
    for (; k < nslots; k += 4) s += partial[(int64_t)k * nout + i];
  }
  red[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && i < nout) {
    const float t = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    float* dst = i < nweights ? w_out + i : b_out + (i - nweights);
    *dst = accumulate ? *dst + t : t;
  }
}

hipError_t wgrad_launch(int kind, const WgradArgs& a, int bands, hipStream_t s) {
  dim3 grid(bands, a.nslices);
  if (kind == 0) hipLaunchKernelGGL(k_wgrad_first, grid, dim3(256), 0, s, a);
  else if (kind == 1) hipLaunchKernelGGL(k_wgrad_mid, grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_wgrad_last, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t wgrad_reduce(const float* partial, int nslots, int nout, float* w_out, float* b_out, int nweights,
                        int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((nout + 63) / 64), dim3(256), 0, s, partial, nslots, nout, w_out,
                     b_out, nweights, accumulate);
  return hipGetLastError();
}

}  // namespace mrx
