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

// The tiles are kept pixel-major (NHWC, 128 bytes a pixel) in LDS and the
// MFMA fragments are read with the transposing LDS load ds_read_b64_tr_b16:
// in each 16-lane group, lane r names the 8 bytes (4 channels of one pixel)
// of row r of a 16 x 4 matrix and receives the column r % 4 ... of rows
// 4j + r / 4 (j = 0..3), i.e. one channel at 4 consecutive pixels.  Two such
// reads give a 32 x 16 operand fragment (8 consecutive K = pixels a lane).
// Because the layout is pixel-major, the column shift of a tap is only an
// address offset (no shifted copies of the input tile are needed), and the
// global data reach LDS as whole 16-byte chunks.
//   g tile:   RT x 32 pixels
//   act tile: (RT + 2) rows x 34 columns (halo), row stride W2_AROW = 36 so
//             that every row starts at a pixel index divisible by 4
// Bank spread: the 16-byte chunk c of LDS pixel P sits at c ^ (4 * bit 1 of
// P); a 32-lane phase of a transposing read (4 consecutive pixels x 64 bytes)
// then covers the 64 banks once.
constexpr int W2_AROW = 36;
constexpr int W2_GPX = RT * 32;
constexpr int W2_APX = (RT + 2) * W2_AROW;
constexpr int W2_PX = W2_GPX + W2_APX;
constexpr int W2_THREADS = 768;
constexpr int W2_PER = (W2_PX * 8 + W2_THREADS - 1) / W2_THREADS;

typedef short v4s __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int w2_slot(int P, int c) { return P * 8 + (c ^ (((P >> 1) & 1) << 2)); }

__device__ __forceinline__ void w2_load(uint4 (&v)[W2_PER], const WgradArgs& a, const TileCursor& c, int64_t t) {
  const int loc = (int)(t - c.base);
  const int row0 = (loc / c.ntx) * RT, col0 = (loc % c.ntx) * 32;
  const uint16_t* g = a.g + c.xoff * CNN_F;
  const uint16_t* act = a.act + c.xoff * CNN_F;
#pragma unroll
  for (int j = 0; j < W2_PER; ++j) {
    const int q = threadIdx.x + W2_THREADS * j;
    const int P = q >> 3, ch = q & 7;
    v[j] = make_uint4(0, 0, 0, 0);
    if (q >= W2_PX * 8) continue;
    int gy, gx;
    const uint16_t* src;
    if (P < W2_GPX) {
      gy = row0 + P / 32;
      gx = col0 + P % 32;
      src = g;
    } else {
      const int pa = P - W2_GPX, x = pa % W2_AROW;
      gy = x < 34 ? row0 - 1 + pa / W2_AROW : -1;
      gx = col0 - 1 + x;
      src = act;
    }
    if (gy >= 0 && gy < c.H && gx >= 0 && gx < c.W)
      v[j] = *(const uint4*)(src + ((int64_t)gy * c.W + gx) * CNN_F + ch * 8);
  }
}

__device__ __forceinline__ void w2_store(uint4* tile, const uint4 (&v)[W2_PER]) {
#pragma unroll
  for (int j = 0; j < W2_PER; ++j) {
    const int q = threadIdx.x + W2_THREADS * j;
    if (q < W2_PX * 8) tile[w2_slot(q >> 3, q & 7)] = v[j];
  }
}

// two transposing reads at byte offsets o0, o1 of the tile: one 32 x 16 fragment
__device__ __forceinline__ uint4 frag_tr(const char* tile, int o0, int o1) {
  typedef __attribute__((address_space(3))) v4s lds_v4s;
  const v4s lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(tile + o0));
  const v4s hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(tile + o1));
  const uint2 l = __builtin_bit_cast(uint2, lo), h = __builtin_bit_cast(uint2, hi);
  return make_uint4(l.x, l.y, h.x, h.y);
}

// A fixed grid of WGM_WGS workgroups walks the batch's tiles (RT rows x 32
// columns, slices in order) in contiguous ranges; each keeps its sums in
// registers over all its tiles and writes one slot at the end.  12 waves,
// one per (co block of 32, ci block of 32, column tap dx); a wave walks the
// rows of each 16-column half of the tile and keeps the act fragments of
// the last three rows, so that each act fragment serves the three row taps.
// The global data of the next two tiles are loaded into registers while the
// current tile's MFMAs run.
__global__ void __launch_bounds__(W2_THREADS) k_wgrad_mid(WgradArgs a) {
  __shared__ uint4 tile[W2_PX * 8];
  float* part = a.partial + (int64_t)blockIdx.x * a.nout;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int mb = wv & 1, nb = (wv >> 1) & 1, dx = wv >> 2;
  // this workgroup's tiles [t0, t1) of the batch
  int64_t total = 0;
  for (int si = 0; si < a.nslices; ++si) {
    const SliceDesc d = a.desc[a.slices[si]];
    total += (int64_t)((d.H + RT - 1) / RT) * ((d.W + 31) / 32);
  }
  const int64_t t0 = total * blockIdx.x / gridDim.x, t1 = total * (blockIdx.x + 1) / gridDim.x;
  // lane-constant byte offsets of the fragment reads (see the layout above)
  const int grp = lane >> 4, rr = lane & 15;
  int offA[2], offB[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int k = 8 * (grp >> 1) + 4 * t + (rr >> 2);
    const int sA = mb * 8 + 4 * (grp & 1) + (rr & 3), swA = ((k >> 1) & 1) << 3;
    offA[t] = k * 128 + (sA ^ swA) * 8;
    const int sB = nb * 8 + 4 * (grp & 1) + (rr & 3), swB = (((k + dx) >> 1) & 1) << 3;
    offB[t] = W2_GPX * 128 + (k + dx) * 128 + (sB ^ swB) * 8;
  }
  const char* tb = (const char*)tile;
  f32x16 acc[3];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[t][v] = 0.f;
  float bsum = 0.f;
  const bool bias_wave = nb == 0 && dx == 0;
  // two register sets of prefetched tiles (tiles t + 1 and t + 2 are in
  // flight while tile t is computed)
  TileCursor nxt;
  cursor_load(nxt, a, 0, 0);
  uint4 va[W2_PER], vb[W2_PER];
  if (t0 < t1) {
    cursor_seek(nxt, a, t0);
    w2_load(va, a, nxt, t0);
  }
  if (t0 + 1 < t1) {
    cursor_seek(nxt, a, t0 + 1);
    w2_load(vb, a, nxt, t0 + 1);
  }
  auto step = [&](int64_t t, uint4 (&v)[W2_PER]) {
    __syncthreads();
    w2_store(tile, v);
    __syncthreads();
    if (t + 2 < t1) {
      cursor_seek(nxt, a, t + 2);
      w2_load(v, a, nxt, t + 2);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      auto fb = [&](int rho) {
        const int o = (rho * W2_AROW + 16 * h) * 128;
        return frag_tr(tb, o + offB[0], o + offB[1]);
      };
      uint4 b0 = fb(0), b1 = fb(1);
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        const uint4 b2 = fb(r + 2);
        const int o = (r * 32 + 16 * h) * 128;
        const uint4 af = frag_tr(tb, o + offA[0], o + offA[1]);
        if (bias_wave) bsum += frag_sum(af);  // bias gradient, channel mb * 32 + lane % 32
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(af), as_bf(b0), acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(af), as_bf(b1), acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(af), as_bf(b2), acc[2], 0, 0, 0);
        b0 = b1;
        b1 = b2;
      }
    }
  };
  for (int64_t t = t0; t < t1; t += 2) {
    step(t, va);
    if (t + 1 < t1) step(t + 1, vb);
  }
#pragma unroll
  for (int dy = 0; dy < 3; ++dy) {
    const int tap = dy * 3 + dx;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int co = mb * 32 + 8 * (v >> 2) + (lane >> 5) * 4 + (v & 3);
      const int ci = nb * 32 + (lane & 31);
      part[(tap * 64 + co) * 64 + ci] = acc[dy][v];  // tap-major: 128-byte runs of ci
    }
  }
  // lanes l and l + 32 hold the two pixel halves of channel mb * 32 + l % 32
  bsum += __shfl_xor(bsum, 32, 64);
  if (bias_wave && lane < 32) part[64 * 64 * 9 + mb * 32 + lane] = bsum;
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
// increasing order, then the 4 wave sums are added in wave order.  With
// tap_major the weight entries of the slots are ordered [tap][co][ci]
// (64 x 64 channels) and go to the [co][ci][tap] gradient.
__global__ void __launch_bounds__(256) k_wgrad_reduce(const float* partial, int nslots, int nout, float* w_out,
                                                      float* b_out, int nweights, int accumulate, int tap_major) {
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
    int wi = i;
    if (tap_major && i < nweights) wi = (i % 4096) * 9 + i / 4096;
    float* dst = i < nweights ? w_out + wi : b_out + (i - nweights);
    *dst = accumulate ? *dst + t : t;
  }
}

hipError_t wgrad_launch(int kind, const WgradArgs& a, int bands, hipStream_t s) {
  dim3 grid(bands, a.nslices);
  if (kind == 0) hipLaunchKernelGGL(k_wgrad_first, grid, dim3(256), 0, s, a);
  else if (kind == 1) hipLaunchKernelGGL(k_wgrad_mid, dim3(WGM_WGS), dim3(W2_THREADS), 0, s, a);
  else hipLaunchKernelGGL(k_wgrad_last, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t wgrad_reduce(const float* partial, int nslots, int nout, float* w_out, float* b_out, int nweights,
                        int accumulate, int tap_major, hipStream_t s) {
  if (tap_major && nweights != 64 * 64 * 9) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((nout + 63) / 64), dim3(256), 0, s, partial, nslots, nout, w_out,
                     b_out, nweights, accumulate, tap_major);
  return hipGetLastError();
}

}  // namespace mrx
