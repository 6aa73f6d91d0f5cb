// Weight and bias gradients of the denoiser's 3x3 convolutions
//   dW[co][ci][tap] = sum_p g[p][co] * a[p + d(tap)][ci],   db[co] = sum_p g[p][co]
// as MFMA products with the pixel index as the reduction (K) dimension.  Tiles
// of WG_ROWS rows x 32 columns are staged in LDS channel-major ([channel][pixel]),
// so a fragment of 8 consecutive pixels of one channel is one 16-byte read.
// Every workgroup writes its partial sums to its own slot; a second kernel
// adds the slots in a fixed order (deterministic, no float atomics).
#include <type_traits>

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
// Row strides of the channel-major LDS tiles, padded by 16 bytes so that the
// 16-byte fragment reads of 16 consecutive channels start in distinct bank
// groups (an unpadded 128- or 256-byte stride puts them all in one).
constexpr int GROW = TPX + 8;
constexpr int AROW = (RT + 2) * 32 + 8;

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
    for (int e = 0; e < 8; ++e) gT[(ch * 8 + e) * GROW + p] = h[e];
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
// A fixed grid of WGM_WGS workgroups walks the batch's tiles (RT rows x 32
// columns, slices in order) in contiguous ranges; each keeps its sums in
// registers over all its tiles and writes one slot at the end.  8 waves:
// (co block, ci block, tap half).  The next tile's global data are loaded
// into registers while the current tile's MFMAs run, then transposed into
// the channel-major LDS tiles.
struct TileCursor {
  int si;         // slice index (into a.slices)
  int64_t base;   // global index of the slice's first tile
  int ntx, ntiles, H, W;
  int64_t xoff;
};

__device__ __forceinline__ void cursor_load(TileCursor& c, const WgradArgs& a, int si, int64_t base) {
  c.si = si;
  c.base = base;
  if (si < a.nslices) {
    const SliceDesc d = a.desc[a.slices[si]];
    c.H = d.H; c.W = d.W; c.xoff = d.xoff;
    c.ntx = (d.W + 31) / 32;
    c.ntiles = ((d.H + RT - 1) / RT) * c.ntx;
  } else {
    c.H = c.W = c.ntx = c.ntiles = 0; c.xoff = 0;
  }
}
// advance the cursor to the slice holding tile t (t never decreases)
__device__ __forceinline__ void cursor_seek(TileCursor& c, const WgradArgs& a, int64_t t) {
  while (c.si < a.nslices && t >= c.base + c.ntiles) cursor_load(c, a, c.si + 1, c.base + c.ntiles);
}

// Loads and channel-major stores of one tile, four consecutive pixels of one
// 8-channel chunk per work item, so that each channel's four values leave as
// one 8-byte LDS write (instead of four 2-byte ones).
//   g items:  (chunk, pixel quad) of the RT x 32 tile: 8 x TPX / 4 = 128
//   a items:  (dx, chunk, row, column quad) of the shifted copies:
//             3 x 8 x (RT + 2) x 8 = 768; copy dx, columns 4k..4k+3 read the
//             halo pixels 4k + dx .. 4k + dx + 3
constexpr int WGM_GITEMS = 8 * TPX / 4;
constexpr int WGM_AITEMS = 3 * 8 * (RT + 2) * 8;
constexpr int WGM_PER_A = (WGM_AITEMS + 511) / 512;

__device__ __forceinline__ void wgm_load(uint4 (&gv)[4], uint4 (&av)[WGM_PER_A][4], const WgradArgs& a,
                                         const TileCursor& c, int64_t t) {
  const int loc = (int)(t - c.base);
  const int row0 = (loc / c.ntx) * RT, col0 = (loc % c.ntx) * 32;
  const uint16_t* g = a.g + c.xoff * CNN_F;
  const uint16_t* act = a.act + c.xoff * CNN_F;
  {
    const int q = threadIdx.x;
    const int quad = q % (TPX / 4), ch = q / (TPX / 4);
    const int p0 = quad * 4, gy = row0 + p0 / 32, gx0 = col0 + p0 % 32;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      gv[u] = make_uint4(0, 0, 0, 0);
      if (q < WGM_GITEMS && gy < c.H && gx0 + u < c.W)
        gv[u] = *(const uint4*)(g + ((int64_t)gy * c.W + gx0 + u) * CNN_F + ch * 8);
    }
  }
#pragma unroll
  for (int j = 0; j < WGM_PER_A; ++j) {
    const int q = threadIdx.x + 512 * j;
    const int k = q % 8, r = (q / 8) % (RT + 2), ch = (q / (8 * (RT + 2))) % 8, dx = q / (8 * (RT + 2) * 8);
    const int gy = row0 - 1 + r, gx0 = col0 + 4 * k + dx - 1;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      av[j][u] = make_uint4(0, 0, 0, 0);
      if (q < WGM_AITEMS && gy >= 0 && gy < c.H && gx0 + u >= 0 && gx0 + u < c.W)
        av[j][u] = *(const uint4*)(act + ((int64_t)gy * c.W + gx0 + u) * CNN_F + ch * 8);
    }
  }
}

// element e (0..7) of the 8 bf16 channels of a 16-byte chunk
__device__ __forceinline__ uint32_t chunk_elem(const uint4& v, int e) {
  const uint32_t w = (e < 2) ? v.x : (e < 4) ? v.y : (e < 6) ? v.z : v.w;
  return (e & 1) ? (w >> 16) : (w & 0xffffu);
}

__device__ __forceinline__ void wgm_store(uint16_t* gT, uint16_t* aT, const uint4 (&gv)[4],
                                          const uint4 (&av)[WGM_PER_A][4]) {
  {
    const int q = threadIdx.x;
    if (q < WGM_GITEMS) {
      const int quad = q % (TPX / 4), ch = q / (TPX / 4);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint2 w = make_uint2(chunk_elem(gv[0], e) | (chunk_elem(gv[1], e) << 16),
                                   chunk_elem(gv[2], e) | (chunk_elem(gv[3], e) << 16));
        *(uint2*)&gT[(ch * 8 + e) * GROW + quad * 4] = w;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < WGM_PER_A; ++j) {
    const int q = threadIdx.x + 512 * j;
    if (q >= WGM_AITEMS) break;
    const int k = q % 8, r = (q / 8) % (RT + 2), ch = (q / (8 * (RT + 2))) % 8, dx = q / (8 * (RT + 2) * 8);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const uint2 w = make_uint2(chunk_elem(av[j][0], e) | (chunk_elem(av[j][1], e) << 16),
                                 chunk_elem(av[j][2], e) | (chunk_elem(av[j][3], e) << 16));
      *(uint2*)&aT[(dx * 64 + ch * 8 + e) * AROW + r * 32 + 4 * k] = w;
    }
  }
}

__global__ void __launch_bounds__(512) k_wgrad_mid(WgradArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t gT[64 * GROW];
  __shared__ __attribute__((aligned(16))) uint16_t aT[3 * 64 * AROW];
  float* part = a.partial + (int64_t)blockIdx.x * a.nout;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int mb = wv & 1, nb = (wv >> 1) & 1, th = wv >> 2;
  const int tap0 = th ? 5 : 0;
  // this workgroup's tiles [t0, t1) of the batch
  int64_t total = 0;
  for (int si = 0; si < a.nslices; ++si) {
    const SliceDesc d = a.desc[a.slices[si]];
    total += (int64_t)((d.H + RT - 1) / RT) * ((d.W + 31) / 32);
  }
  const int64_t t0 = total * blockIdx.x / gridDim.x, t1 = total * (blockIdx.x + 1) / gridDim.x;
  f32x16 acc[5];
#pragma unroll
  for (int t = 0; t < 5; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[t][v] = 0.f;
  float bsum = 0.f;
  TileCursor cur, nxt;
  cursor_load(cur, a, 0, 0);
  cursor_seek(cur, a, t0);
  nxt = cur;
  uint4 gv[4], av[WGM_PER_A][4];
  if (t0 < t1) wgm_load(gv, av, a, cur, t0);
  for (int64_t t = t0; t < t1; ++t) {
    __syncthreads();
    wgm_store(gT, aT, gv, av);
    __syncthreads();
    if (t + 1 < t1) {
      cursor_seek(nxt, a, t + 1);
      wgm_load(gv, av, a, nxt, t + 1);
    }
    // one fragment set: the reads of k-step ks + 1 are issued right behind the
    // MFMAs of k-step ks (which read their operands at issue)
    auto compute = [&](auto th_c) {
      constexpr int TAP0 = decltype(th_c)::value ? 5 : 0, NTAP = decltype(th_c)::value ? 4 : 5;
      uint4 af, bfr[NTAP];
      auto ld = [&](int ks) {
        const int r = ks >> 1, c = (ks & 1) * 16 + (lane >> 5) * 8;
        af = *(const uint4*)&gT[(mb * 32 + (lane & 31)) * GROW + r * 32 + c];
#pragma unroll
        for (int k = 0; k < NTAP; ++k) {
          const int tap = TAP0 + k, dy = tap / 3, dx = tap % 3;
          bfr[k] = *(const uint4*)&aT[(dx * 64 + nb * 32 + (lane & 31)) * AROW + (r + dy) * 32 + c];
        }
      };
      ld(0);
#pragma unroll
      for (int ks = 0; ks < TPX / 16; ++ks) {
        if (nb == 0 && TAP0 == 0) bsum += frag_sum(af);  // bias gradient, channel mb * 32 + lane % 32
#pragma unroll
        for (int k = 0; k < NTAP; ++k)
          acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(af), as_bf(bfr[k]), acc[k], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
        if (ks + 1 < TPX / 16) ld(ks + 1);
      }
    };
    if (th == 0) compute(std::integral_constant<int, 0>{});
    else compute(std::integral_constant<int, 1>{});
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const int tap = tap0 + k;
    if (tap > 8) break;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int co = mb * 32 + 8 * (v >> 2) + (lane >> 5) * 4 + (v & 3);
      const int ci = nb * 32 + (lane & 31);
      part[(co * 64 + ci) * 9 + tap] = acc[k][v];
    }
  }
  // lanes l and l + 32 hold the two pixel halves of channel mb * 32 + l % 32
  bsum += __shfl_xor(bsum, 32, 64);
  if (nb == 0 && th == 0 && lane < 32) part[64 * 64 * 9 + mb * 32 + lane] = bsum;
}

// ------------------------------------------------------------- 2 -> 64
// dW1[co][ci][tap] with N = (tap, ci) = 18 padded to 32; waves split
// (co block) x (k-step parity); each parity has its own partial slot.
__global__ void __launch_bounds__(256) k_wgrad_first(WgradArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t gT[64 * GROW];
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
        const uint4 araw = *(const uint4*)&gT[(mb * 32 + (lane & 31)) * GROW + r * 32 + c];
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
  __shared__ __attribute__((aligned(16))) uint16_t aT[64 * GROW];
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
      if (wv == 0) {  // bias gradient from the fp32 output gradient: wave 0, per lane
        for (int p = lane; p < TPX; p += 64) {
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
        const bf16x8 bv = as_bf(*(const uint4*)&aT[(nb * 32 + (lane & 31)) * GROW + r * 32 + c]);
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
  // wave 0 (par 0) holds per-lane sums; fixed butterfly
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
  else if (kind == 1) hipLaunchKernelGGL(k_wgrad_mid, dim3(WGM_WGS), dim3(512), 0, s, a);
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
