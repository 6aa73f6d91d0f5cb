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
__device__ __forceinline__ void fill_gT(uint16_t* gT, const uint16_t* g, int H, int W, int row0, int col0) {
  for (int q = threadIdx.x; q < TPX * 8; q += 256) {
    const int p = q % TPX, ch = q / TPX;
    const int gy = row0 + p / 32, gx = col0 + p % 32;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (gy < H && gx < W) v = *(const uint4*)(g + ((int64_t)gy * W + gx) * CNN_F + ch * 8);
    const uint16_t* h = (const uint16_t*)&v;
#pragma unroll
    for (int e = 0; e < 8; ++e) gT[(ch * 8 + e) * TPX + p] = h[e];
  }
}

// aT[dx][ch][r * 32 + c] = a[row0 - 1 + r][col0 + c + dx - 1][ch], r < RT + 2.
__device__ __forceinline__ void fill_aT3(uint16_t* aT, const uint16_t* a, int H, int W, int row0, int col0) {
  constexpr int HP = (RT + 2) * 32;
  for (int q = threadIdx.x; q < 3 * HP * 8; q += 256) {
    const int p = q % HP, rest = q / HP;
    const int ch = rest % 8, dx = rest / 8;
    const int gy = row0 - 1 + p / 32, gx = col0 + p % 32 + dx - 1;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (gy >= 0 && gy < H && gx >= 0 && gx < W) v = *(const uint4*)(a + ((int64_t)gy * W + gx) * CNN_F + ch * 8);
    const uint16_t* h = (const uint16_t*)&v;
#pragma unroll
    for (int e = 0; e < 8; ++e) aT[(dx * 64 + ch * 8 + e) * HP + p] = h[e];
  }
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
      if (threadIdx.x < 64)
        for (int p = 0; p < TPX; ++p) bsum += bf2f_w(gT[threadIdx.x * TPX + p]);
#pragma unroll
      for (int ks = 0; ks < TPX / 16; ++ks) {
        const int r = ks >> 1, c = (ks & 1) * 16 + (lane >> 5) * 8;
        const bf16x8 av = as_bf(*(const uint4*)&gT[(mb * 32 + (lane & 31)) * TPX + r * 32 + c]);
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
  if (threadIdx.x < 64) part[64 * 64 * 9 + threadIdx.x] = bsum;
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
      if (par == 0 && mb == 0) {
        for (int p = 0; p < TPX; ++p) bsum += bf2f_w(gT[lane * TPX + p]);
      }
#pragma unroll
      for (int ks = par; ks < TPX / 16; ks += 2) {
        const int r = ks >> 1, c = (ks & 1) * 16 + (lane >> 5) * 8;
        const bf16x8 av = as_bf(*(const uint4*)&gT[(mb * 32 + (lane & 31)) * TPX + r * 32 + c]);
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
  if (par == 0 && mb == 0) part[64 * 2 * 9 + lane] = bsum;
  if (par == 1 && mb == 0) part[64 * 2 * 9 + lane] = 0.f;
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
      if (threadIdx.x == 0) {  // bias gradient from the fp32 output gradient
        for (int p = 0; p < TPX; ++p) {
          const int gy = row0 + p / 32, gx = col0 + p % 32;
          if (gy < H && gx < W) {
            const float2 v = g5[(int64_t)gy * W + gx];
            bs0 += v.x;
            bs1 += v.y;
          }
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
  if (threadIdx.x == 0) {
    part[2 * 64 * 9 + 0] = par == 0 && nb == 0 ? bs0 : 0.f;
    part[2 * 64 * 9 + 1] = par == 0 && nb == 0 ? bs1 : 0.f;
  }
  if (wv == 2 && lane == 0) {
    part[2 * 64 * 9 + 0] = 0.f;
    part[2 * 64 * 9 + 1] = 0.f;
  }
}

// out[i] (+)= sum_s partial[s][i] over nslots slots, fixed order.
__global__ void k_wgrad_reduce(const float* partial, int nslots, int nout, float* w_out, float* b_out,
                               int nweights, int accumulate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nout) return;
  float s = 0.f;
  for (int k = 0; k < nslots; ++k) s += partial[(int64_t)k * nout + i];
  float* dst = i < nweights ? w_out + i : b_out + (i - nweights);
  *dst = accumulate ? *dst + s : s;
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
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((nout + 255) / 256), dim3(256), 0, s, partial, nslots, nout, w_out,
                     b_out, nweights, accumulate);
  return hipGetLastError();
}

}  // namespace mrx
