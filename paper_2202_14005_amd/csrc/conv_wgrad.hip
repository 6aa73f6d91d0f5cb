// Weight gradients of the denoiser's 3x3 convolutions
//   dW[co][ci][tap] = sum_p g[p][co] * a[p + d(tap)][ci]
// as MFMA products with the pixel index as the reduction (K) dimension, and
// the last layer's bias gradient db[co] = sum_p g[p][co] from its fp32
// gradient (the inner layers' bias gradients are summed in fp32 by the
// input-gradient convolutions that produce their gradients, conv.hip).  A
// fixed grid of WGM_WGS workgroups walks the batch's tiles of WG_ROWS rows x
// 32 columns; every workgroup writes its partial sums to its own slot and a
// second kernel adds the slots in a fixed order (deterministic, no float
// atomics) and scatters them to the [co][ci][tap] gradient layout.
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

constexpr int RT = WG_ROWS;  // rows per tile (tiles are RT x 32 pixels)

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
}

// ------------------------------------------------- 2 -> 64 and 64 -> 2
// One 64-channel operand (the first layer's output gradient g1, the last
// layer's input activation a4) comes from an RT x 32 NHWC tile read with the
// transposing loads; the other (the complex input x of the first layer, the
// complex output gradient g5 of the last) from a bf16 halo tile, re and im
// planes with row stride 36, gathered per lane.  The 18 (tap, complex
// component) pairs fill one 32-wide MFMA dimension (padded).  4 waves:
// (64-channel block of 32, 16-column half of the tile); the two halves'
// sums are added through LDS at the end.  Tiles t + 1 and t + 2 are
// prefetched into registers; WGS_WGS workgroups (four a CU) keep enough
// loads in flight.
constexpr int WS_THREADS = 256;
constexpr int WS_CPX = (RT + 2) * 34;          // complex halo pixels
constexpr int WS_CROW = 36;

struct SmallPre {
  uint4 t[4];  // 64-channel tile: 1024 chunks over 256 threads
  float2 c;    // complex halo pixel threadIdx.x (if < WS_CPX)
};

__device__ __forceinline__ void ws_load(SmallPre& v, const uint16_t* t64, const float2* cx, const TileCursor& c,
                                        int64_t t) {
  const int loc = (int)(t - c.base);
  const int row0 = (loc / c.ntx) * RT, col0 = (loc % c.ntx) * 32;
  const uint16_t* src = t64 + c.xoff * CNN_F;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int q = threadIdx.x + WS_THREADS * j;
    const int P = q >> 3, ch = q & 7;
    const int gy = row0 + P / 32, gx = col0 + P % 32;
    v.t[j] = make_uint4(0, 0, 0, 0);
    if (gy < c.H && gx < c.W) v.t[j] = *(const uint4*)(src + ((int64_t)gy * c.W + gx) * CNN_F + ch * 8);
  }
  v.c = make_float2(0.f, 0.f);
  if (threadIdx.x < WS_CPX) {
    const int gy = row0 - 1 + threadIdx.x / 34, gx = col0 - 1 + threadIdx.x % 34;
    if (gy >= 0 && gy < c.H && gx >= 0 && gx < c.W) v.c = cx[c.xoff + (int64_t)gy * c.W + gx];
  }
}

__device__ __forceinline__ void ws_store(uint4* tile, uint16_t* cs, const SmallPre& v) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int q = threadIdx.x + WS_THREADS * j;
    tile[w2_slot(q >> 3, q & 7)] = v.t[j];
  }
  if (threadIdx.x < WS_CPX) {
    const int o = (threadIdx.x / 34) * WS_CROW + threadIdx.x % 34;
    cs[o] = f2bf_w(v.c.x);
    cs[(RT + 2) * WS_CROW + o] = f2bf_w(v.c.y);
  }
}

// LAST = false: dW1 (M = co of g1, N = (tap, ci) of x);
// LAST = true:  dW5 (M = (tap, co) of g5 shifted, N = ci of a4).
template <bool LAST>
__global__ void __launch_bounds__(WS_THREADS) k_wgrad_small(WgradArgs a) {
  __shared__ uint4 tile[RT * 32 * 8];
  __shared__ uint16_t cs[2 * (RT + 2) * WS_CROW];
  __shared__ float comb[2][16][64];
  float* part = a.partial + (int64_t)blockIdx.x * a.nout;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int blk = wv & 1, h = wv >> 1;
  int64_t total = 0;
  for (int si = 0; si < a.nslices; ++si) {
    const SliceDesc d = a.desc[a.slices[si]];
    total += (int64_t)((d.H + RT - 1) / RT) * ((d.W + 31) / 32);
  }
  const int64_t t0 = total * blockIdx.x / gridDim.x, t1 = total * (blockIdx.x + 1) / gridDim.x;
  // transposing-read offsets of the 64-channel operand (channel block blk)
  const int grp = lane >> 4, rr = lane & 15;
  int off[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int k = 8 * (grp >> 1) + 4 * t + (rr >> 2);
    off[t] = k * 128 + ((blk * 8 + 4 * (grp & 1) + (rr & 3)) ^ (((k >> 1) & 1) << 3)) * 8;
  }
  // gathered operand: index j = lane % 32 = 2 tap + component (j < 18)
  const int j = lane & 31, tap = j >> 1, comp = j & 1, dy = tap / 3, dx = tap % 3;
  const int cbase = comp * (RT + 2) * WS_CROW + (LAST ? (2 - dy) * WS_CROW + 2 - dx : dy * WS_CROW + dx) +
                    16 * h + 8 * (lane >> 5);
  const char* tb = (const char*)tile;
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  float bs0 = 0.f, bs1 = 0.f;  // last layer: bias gradient (fp32 input gradient)
  const uint16_t* t64 = LAST ? a.act : a.g;
  TileCursor nxt;
  cursor_load(nxt, a, 0, 0);
  SmallPre va, vb;
  if (t0 < t1) {
    cursor_seek(nxt, a, t0);
    ws_load(va, t64, a.x, nxt, t0);
  }
  if (t0 + 1 < t1) {
    cursor_seek(nxt, a, t0 + 1);
    ws_load(vb, t64, a.x, nxt, t0 + 1);
  }
  auto step = [&](int64_t t, SmallPre& v) {
    __syncthreads();
    ws_store(tile, cs, v);
    if (LAST && threadIdx.x < WS_CPX) {  // bias of the last layer: interior pixels, fp32
      const int y = threadIdx.x / 34, x = threadIdx.x % 34;
      if (y >= 1 && y <= RT && x >= 1 && x <= 32) {
        bs0 += v.c.x;
        bs1 += v.c.y;
      }
    }
    __syncthreads();
    if (t + 2 < t1) {
      cursor_seek(nxt, a, t + 2);
      ws_load(v, t64, a.x, nxt, t + 2);
    }
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      const int o = (r * 32 + 16 * h) * 128;
      const uint4 f = frag_tr(tb, o + off[0], o + off[1]);
      uint4 raw;
      uint16_t* e8 = (uint16_t*)&raw;
#pragma unroll
      for (int e = 0; e < 8; ++e) e8[e] = j < 18 ? cs[cbase + r * WS_CROW + e] : (uint16_t)0;
      if (LAST) {
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(raw), as_bf(f), acc, 0, 0, 0);
      } else {
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(f), as_bf(raw), acc, 0, 0, 0);
      }
    }
  };
  for (int64_t t = t0; t < t1; t += 2) {
    step(t, va);
    if (t + 1 < t1) step(t + 1, vb);
  }
  // add the column halves (h = 1 through LDS, in that fixed order)
  if (h == 1) {
#pragma unroll
    for (int v = 0; v < 16; ++v) comb[blk][v][lane] = acc[v];
  }
  __syncthreads();
  if (h == 0) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float s = acc[v] + comb[blk][v][lane];
      const int m = 8 * (v >> 2) + (lane >> 5) * 4 + (v & 3);  // MFMA row
      if (LAST) {
        if (m < 18) part[m * 64 + blk * 32 + (lane & 31)] = s;  // [tap, co][ci]
      } else {
        part[(blk * 32 + m) * 32 + j] = s;  // [co][tap, ci] (j >= 18: zero padding)
      }
    }
  }
  if (LAST) {
    // bias: per-thread sums -> wave butterfly -> the 4 wave sums in order
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      bs0 += __shfl_xor(bs0, o, 64);
      bs1 += __shfl_xor(bs1, o, 64);
    }
    __syncthreads();
    if (lane == 0) {
      comb[0][0][wv] = bs0;
      comb[0][1][wv] = bs1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      part[18 * 64 + 0] = ((comb[0][0][0] + comb[0][0][1]) + comb[0][0][2]) + comb[0][0][3];
      part[18 * 64 + 1] = ((comb[0][1][0] + comb[0][1][1]) + comb[0][1][2]) + comb[0][1][3];
    }
  }
}

// out (+)= sum_s partial[s] over nslots slots in a fixed order: a block
// takes 64 partial entries; its 16 waves sum the slots s = w, w + 16, ... in
// increasing order, then the 16 wave sums are added in wave order.  Entries
// [0, npw) are weights in the slot layout `layout`, the rest biases:
//   WG_LAYOUT_MID:   [tap][co][ci], 64 x 64
//   WG_LAYOUT_FIRST: [co][2 tap + ci], 64 x 32 (entries 18..31 of a row unused)
//   WG_LAYOUT_LAST:  [2 tap + co][ci], 18 x 64
// and go to the [co][ci][tap] gradient.
__device__ __forceinline__ int wg_dst(int layout, int i) {
  if (layout == WG_LAYOUT_MID) return (i % 4096) * 9 + i / 4096;
  if (layout == WG_LAYOUT_FIRST) {
    const int co = i >> 5, jj = i & 31;
    return jj < 18 ? (co * 2 + (jj & 1)) * 9 + (jj >> 1) : -1;
  }
  const int m = i >> 6, ci = i & 63;
  return ((m & 1) * 64 + ci) * 9 + (m >> 1);
}

constexpr int WR_WAVES = 16;

__global__ void __launch_bounds__(64 * WR_WAVES) k_wgrad_reduce(const float* partial, int nslots, int nout,
                                                               int nred, float* w_out, float* b_out, int npw,
                                                               int accumulate, int layout) {
  __shared__ float red[WR_WAVES][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  float s = 0.f;
  if (i < nred) {
    int k = wv;
    for (; k + 3 * WR_WAVES < nslots; k += 4 * WR_WAVES) {
      const float a0 = partial[(int64_t)k * nout + i];
      const float a1 = partial[(int64_t)(k + WR_WAVES) * nout + i];
      const float a2 = partial[(int64_t)(k + 2 * WR_WAVES) * nout + i];
      const float a3 = partial[(int64_t)(k + 3 * WR_WAVES) * nout + i];
      s += a0; s += a1; s += a2; s += a3;
    }
    for (; k < nslots; k += WR_WAVES) s += partial[(int64_t)k * nout + i];
  }
  red[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && i < nred) {
    float t = red[0][lane];
#pragma unroll
    for (int w = 1; w < WR_WAVES; ++w) t += red[w][lane];
    float* dst = nullptr;
    if (i >= npw) {
      dst = b_out + (i - npw);
    } else {
      const int wi = wg_dst(layout, i);
      if (wi >= 0) dst = w_out + wi;
    }
    if (dst) *dst = accumulate ? *dst + t : t;
  }
}

hipError_t wgrad_launch(int kind, const WgradArgs& a, hipStream_t s) {
  if (a.nout != wgrad_nout(kind)) return hipErrorInvalidValue;
  if (kind == 0) hipLaunchKernelGGL(k_wgrad_small<false>, dim3(WGS_WGS), dim3(WS_THREADS), 0, s, a);
  else if (kind == 1) hipLaunchKernelGGL(k_wgrad_mid, dim3(WGM_WGS), dim3(W2_THREADS), 0, s, a);
  else hipLaunchKernelGGL(k_wgrad_small<true>, dim3(WGS_WGS), dim3(WS_THREADS), 0, s, a);
  return hipGetLastError();
}

hipError_t wgrad_reduce(int kind, const float* partial, float* w_out, float* b_out, int accumulate, hipStream_t s) {
  const int nout = wgrad_nout(kind);
  const int npw = kind == 1 ? 64 * 64 * 9 : kind == 0 ? 64 * 32 : 18 * 64;
  const int layout = kind == 1 ? WG_LAYOUT_MID : kind == 0 ? WG_LAYOUT_FIRST : WG_LAYOUT_LAST;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((nout + 63) / 64), dim3(64 * WR_WAVES), 0, s, partial,
                     wgrad_slots(kind), nout, nout, w_out, b_out, npw, accumulate, layout);
  return hipGetLastError();
}

hipError_t bias_reduce(const float* partial, int nslots, float* b_out, int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(1), dim3(64 * WR_WAVES), 0, s, partial, nslots, 64, 64,
                     (float*)nullptr, b_out, 0, accumulate, WG_LAYOUT_MID);
  return hipGetLastError();
}

}  // namespace mrx
