// MFMA 3x3 convolutions for the MoDL denoiser (bf16 operands, fp32
// accumulation, NHWC activations).  One workgroup (4 waves) computes a
// 16 x 16-pixel output tile of one slice; the input tile with its one-pixel
// halo is staged in LDS, weights stream from L1/L2 as MFMA fragments.
//   first layer:  2 -> 64 channels, v_mfma_f32_32x32x16_bf16, K = 18 -> 32
//   middle layer: 64 -> 64, v_mfma_f32_32x32x16_bf16, K = 9 x 64
//   last layer:   64 -> 2 (+ residual), v_mfma_f32_16x16x32_bf16, co padded to 16
//   first + second layer fused (inference forward only)
// The same kernels (the fused one excepted) run the input-gradient (dgrad)
// pass with transposed, flipped weights and a ReLU-derivative mask in the
// epilogue.
#include "conv.h"
#include "cg_kernels.h"

namespace mrx {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);                      // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ __forceinline__ uint4 ldg16(const uint16_t* p) { return *(const uint4*)p; }

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// Two floats -> two bf16 (round to nearest even, v_cvt_pk_bf16_f32), low
// half first.
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  const f32x2_t f = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2_t));
}


// 64-channel LDS tiles: 8 chunks of 16 bytes per pixel (128 bytes = 32
// banks).  Chunk c of pixel p sits at slot c ^ ((p >> 1) & 7): 16
// consecutive pixels then cover the 64 banks exactly once for a fixed chunk
// (pixel parity picks the bank half, the slot the 4-bank group).
__device__ __forceinline__ int swz(int px) { return (px >> 1) & 7; }

__device__ __forceinline__ bool bf_pos(uint16_t h) { return (h & 0x8000u) == 0 && h != 0; }

// Coalesced epilogue of one 32-pixel x 64-channel block (the two 32 x 32
// accumulators a0 = channels 0-31, a1 = 32-63 of one wave).  The MFMA result
// gives each lane 4 channels of one pixel per register group, so direct
// stores would touch 32 pixels (32 cache lines) per instruction.  Instead the
// block goes through the wave's own 4 KB of LDS (stg, 32 pixel rows of 16
// eight-byte slots; slot s of pixel p sits at s ^ ((p >> 1) & 15), so a
// 32-lane write phase covers the 64 banks once) and is written back as whole
// pixels: 8 lanes x 16 bytes per pixel, 1 KB of consecutive pixels per
// store.  Forward: + bias, ReLU (before staging).  Input gradient: zero where
// relu_ref (read with the same 16-byte pattern) is not positive.
// pix(i) is the element offset (pixel x 64) of block pixel i, or -1 if it
// lies outside the image.
struct WaveFence {
  __device__ static __forceinline__ void sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
};

template <bool NORM, class PixFn>
__device__ __forceinline__ void epi_block64(const f32x16& a0, const f32x16& a1, const float* sbias,
                                            const float* sscl, int mode, uint2* stg, int lane, PixFn pix,
                                            uint16_t* out, const uint16_t* rref) {
  const int n = lane & 31, hsel = lane >> 5, kx = (n >> 1) & 15;
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int co0 = m * 32 + 8 * g + hsel * 4;
      float hv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float v = m ? a1[4 * g + j] : a0[4 * g + j];
        if constexpr (NORM) {
          v = (v + sbias[co0 + j]) * sscl[co0 + j];
        } else if (mode == CONV_FWD) {
          v += sbias[co0 + j];
          v = v > 0.f ? v : 0.f;
        }
        hv[j] = v;
      }
      uint2 pk;
      pk.x = pack_bf16x2(hv[0], hv[1]);
      pk.y = pack_bf16x2(hv[2], hv[3]);
      stg[n * 16 + ((co0 >> 2) ^ kx)] = pk;
    }
  WaveFence::sync();
  const int c = lane & 7;
  uint4 v[4];
  int64_t off[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int pi = r * 8 + (lane >> 3), k = (pi >> 1) & 15;
    uint4 t = *(const uint4*)&stg[pi * 16 + 2 * (c ^ (k >> 1))];
    if (k & 1) t = make_uint4(t.z, t.w, t.x, t.y);
    v[r] = t;
    off[r] = pix(pi);
  }
  WaveFence::sync();  // stg is free for the next block
  if (mode == CONV_DGRAD) {
    uint4 mr[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) mr[r] = off[r] >= 0 ? ldg16(rref + off[r] + c * 8) : make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      uint32_t* vw = (uint32_t*)&v[r];
      const uint32_t* mw = (const uint32_t*)&mr[r];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t lo = bf_pos((uint16_t)(mw[e] & 0xffffu)) ? 0xffffu : 0u;
        const uint32_t hi = bf_pos((uint16_t)(mw[e] >> 16)) ? 0xffff0000u : 0u;
        vw[e] &= lo | hi;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (off[r] >= 0) *(uint4*)(out + off[r] + c * 8) = v[r];
}

// Input-gradient epilogue that also sums the bias gradient in fp32: the
// block is staged as fp32 (each wave's 8 KB: 32 pixel rows of 16 quads of 4
// channels, quad q of pixel n at q ^ (n & 15), conflict-free for both
// phases), read back as whole pixels, masked by relu_ref on the fp32 values,
// rounded to bf16 and stored (the stored values equal those of epi_block64:
// masking commutes with rounding zero).  bs[e] accumulates, per lane, the
// masked values of channel (lane & 7) * 8 + e over the lane's pixels.
template <class PixFn>
__device__ __forceinline__ void epi_block64_bsum(const f32x16& a0, const f32x16& a1, float4* stgf, int lane,
                                                 PixFn pix, uint16_t* out, const uint16_t* rref, float (&bs)[8]) {
  const int n = lane & 31, hsel = lane >> 5;
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int q = m * 8 + 2 * g + hsel;  // channels 4q .. 4q + 3
      const f32x16& a = m ? a1 : a0;
      stgf[n * 16 + (q ^ (n & 15))] = make_float4(a[4 * g], a[4 * g + 1], a[4 * g + 2], a[4 * g + 3]);
    }
  const int c = lane & 7;
  int64_t off[4];
  uint4 mr[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    off[r] = pix(r * 8 + (lane >> 3));
    mr[r] = off[r] >= 0 ? ldg16(rref + off[r] + c * 8) : make_uint4(0, 0, 0, 0);
  }
  WaveFence::sync();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int pi = r * 8 + (lane >> 3), k = pi & 15;
    const float4 f0 = stgf[pi * 16 + ((2 * c) ^ k)], f1 = stgf[pi * 16 + ((2 * c + 1) ^ k)];
    const float fv[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
    const uint32_t* mw = (const uint32_t*)&mr[r];
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const uint16_t h = (uint16_t)((e & 1) ? (mw[e >> 1] >> 16) : (mw[e >> 1] & 0xffffu));
      v[e] = bf_pos(h) ? fv[e] : 0.f;
      bs[e] += v[e];
    }
    uint4 pk;
    pk.x = pack_bf16x2(v[0], v[1]);
    pk.y = pack_bf16x2(v[2], v[3]);
    pk.z = pack_bf16x2(v[4], v[5]);
    pk.w = pack_bf16x2(v[6], v[7]);
    if (off[r] >= 0) *(uint4*)(out + off[r] + c * 8) = pk;
  }
  WaveFence::sync();  // stgf is free for the next block
}

// The workgroup's bias partial from the lanes' sums bs (see epi_block64_bsum):
// a butterfly over the 8 lanes that share a channel group, the 4 waves' sums
// through LDS (wsum, 4 x 64 floats) in wave order, one slot of 64 floats.
__device__ __forceinline__ void bias_partial_store(float (&bs)[8], float* wsum, float* slot) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int o = 8; o <= 32; o <<= 1)
#pragma unroll
    for (int e = 0; e < 8; ++e) bs[e] += __shfl_xor(bs[e], o, 64);
  if (lane < 8) {
#pragma unroll
    for (int e = 0; e < 8; ++e) wsum[wv * 64 + lane * 8 + e] = bs[e];
  }
  __syncthreads();
  if (threadIdx.x < 64)
    slot[threadIdx.x] = ((wsum[threadIdx.x] + wsum[64 + threadIdx.x]) + wsum[128 + threadIdx.x]) + wsum[192 + threadIdx.x];
}

__device__ __forceinline__ float* bias_slot(const ConvArgs& a) {
  return a.bias_part + ((int64_t)blockIdx.x + (int64_t)a.tiles_x * (blockIdx.y + (int64_t)a.tiles_y * blockIdx.z)) * CNN_F;
}

// Statistics epilogue of a convolution feeding a batch normalisation: the
// block is staged as fp32 as in epi_block64_bsum and read back as whole
// pixels; bs[e] and bs2[e] accumulate, per lane, y and y^2 of channel
// (lane & 7) * 8 + e over the lane's pixels inside the image.  Nothing is
// stored.
template <class PixFn>
__device__ __forceinline__ void epi_block64_stats(const f32x16& a0, const f32x16& a1, float4* stgf, int lane,
                                                  PixFn pix, float (&bs)[8], float (&bs2)[8]) {
  const int n = lane & 31, hsel = lane >> 5;
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int q = m * 8 + 2 * g + hsel;
      const f32x16& a = m ? a1 : a0;
      stgf[n * 16 + (q ^ (n & 15))] = make_float4(a[4 * g], a[4 * g + 1], a[4 * g + 2], a[4 * g + 3]);
    }
  const int c = lane & 7;
  WaveFence::sync();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int pi = r * 8 + (lane >> 3), k = pi & 15;
    if (pix(pi) < 0) continue;
    const float4 f0 = stgf[pi * 16 + ((2 * c) ^ k)], f1 = stgf[pi * 16 + ((2 * c + 1) ^ k)];
    const float fv[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      bs[e] += fv[e];
      bs2[e] += fv[e] * fv[e];
    }
  }
  WaveFence::sync();  // stgf is free for the next block
}

// The workgroup's statistics slot (128 floats: sums of y, then of y^2) from
// the lanes' sums, in the fixed order of bias_partial_store; wsum: 512 floats.
__device__ __forceinline__ void stats_partial_store(float (&bs)[8], float (&bs2)[8], float* wsum, float* slot) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int o = 8; o <= 32; o <<= 1)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      bs[e] += __shfl_xor(bs[e], o, 64);
      bs2[e] += __shfl_xor(bs2[e], o, 64);
    }
  if (lane < 8) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      wsum[wv * 128 + lane * 8 + e] = bs[e];
      wsum[wv * 128 + 64 + lane * 8 + e] = bs2[e];
    }
  }
  __syncthreads();
  if (threadIdx.x < 128)
    slot[threadIdx.x] = ((wsum[threadIdx.x] + wsum[128 + threadIdx.x]) + wsum[256 + threadIdx.x]) + wsum[384 + threadIdx.x];
}

__device__ __forceinline__ float* stat_slot(const ConvArgs& a) {
  return a.stat_part + ((int64_t)blockIdx.x + (int64_t)a.tiles_x * (blockIdx.y + (int64_t)a.tiles_y * blockIdx.z)) * 2 * CNN_F;
}

// epilogue kinds of the first and middle layers: plain (forward bias +
// ReLU, or input gradient), input gradient with bias sums, statistics, and
// normalisation (each a compile-time variant, so that the plain forward
// compiles to the same code as without batch normalisation)
constexpr int EPI_PLAIN = 0, EPI_BSUM = 1, EPI_STATS = 2, EPI_NORM = 3;

// ------------------------------------------------------------- 64 -> 64
// 16 x 16-pixel tiles (41.5 KB of LDS) so that three workgroups fit on a CU;
// each wave computes 4 rows x 16 columns x 64 output channels as 2 pixel
// blocks of 2 rows x 16 columns (4 accumulators of 32 x 32), few enough
// registers for three waves per SIMD: while one workgroup fills its tile the
// other two run MFMAs.  K runs over 9 taps x 4 chunks of 16 input channels;
// the weight fragments of the next tap are fetched from L2 while the
// current tap runs, in two register sets used in turn (a rolled loop with
// one set made the compiler wait for the loads at the back edge).
// The epilogue's per-channel terms in LDS: the bias (forward), or, for the
// normalising variant, minus the mean and the inverse standard deviation.
template <bool NORM>
__device__ __forceinline__ void stage_bias(const ConvArgs& a, float* sbias, float* sscl) {
  if (threadIdx.x < CNN_F) {
    const int c = threadIdx.x;
    if constexpr (NORM) {
      sbias[c] = -a.bn_stats[c];
      sscl[c] = a.bn_stats[CNN_F + c];
    } else {
      sbias[c] = (a.mode == CONV_FWD && a.bias) ? a.bias[c] : 0.f;
    }
  }
}

constexpr int TW16 = CONV_TW;
constexpr int TILE16_PX = (CONV_TH + 2) * (TW16 + 2);
constexpr int TILE1_PX = TILE16_PX;  // first layer: complex pixels (bf16 re, im in one word)
constexpr int TILE16_CHUNKS = TILE16_PX * 8;
constexpr int TILE16_PER_THREAD = (TILE16_CHUNKS + 255) / 256;

__device__ __forceinline__ void load_tile64_16(uint4* tile, const uint16_t* in, int H, int W, int ty0, int tx0) {
  uint4 v[TILE16_PER_THREAD];
  int slot[TILE16_PER_THREAD];
#pragma unroll
  for (int j = 0; j < TILE16_PER_THREAD; ++j) {
    const int q = threadIdx.x + 256 * j;
    v[j] = make_uint4(0, 0, 0, 0);
    slot[j] = -1;
    if (q < TILE16_CHUNKS) {
      const int px = q >> 3, ch = q & 7;
      const int ly = px / (TW16 + 2), lx = px - ly * (TW16 + 2);
      const int gy = ty0 + ly - 1, gx = tx0 + lx - 1;
      slot[j] = px * 8 + (ch ^ swz(px));
      if (gy >= 0 && gy < H && gx >= 0 && gx < W) v[j] = ldg16(in + ((int64_t)gy * W + gx) * CNN_F + ch * 8);
    }
  }
#pragma unroll
  for (int j = 0; j < TILE16_PER_THREAD; ++j)
    if (slot[j] >= 0) tile[slot[j]] = v[j];
}

// The 64 -> 64 layer on a staged input tile (all of its 18 x 18 pixels and
// 64 channels in LDS, swizzled): MFMA loop and epilogue.  wa holds the
// first tap's weight fragments on entry.
template <int EPI>
__device__ __forceinline__ void mid16_compute(uint4* tile, const float* sbias, const float* sscl, const ConvArgs& a,
                                              const SliceDesc& d, int ty0, int tx0, uint4 (&wa)[4][2]) {
  const int H = d.H, W = d.W;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int hsel = lane >> 5, n = lane & 31;
  const uint16_t* wp = a.wpk + lane * 8;
  uint4 wb[4][2];
  f32x16 acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[m][nb][v] = 0.f;
  // pixel n of block nb: row wv * 4 + nb * 2 + n / 16, column n % 16
  const int pbase = (wv * 4 + (n >> 4)) * (TW16 + 2) + (n & 15);
  auto tap_step = [&](int tap, uint4 (&cur)[4][2], uint4 (&nxt)[4][2]) {
    const int dy = tap / 3, dx = tap - 3 * dy;
    if (tap + 1 < 9) {
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        nxt[kc][0] = ldg16(wp + (((tap + 1) * 4 + kc) * 2 + 0) * 512);
        nxt[kc][1] = ldg16(wp + (((tap + 1) * 4 + kc) * 2 + 1) * 512);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const bf16x8 w0 = as_bf16x8(cur[kc][0]), w1 = as_bf16x8(cur[kc][1]);
      const int ch = kc * 2 + hsel;
      bf16x8 bv[2];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const int px = pbase + (dy + nb * 2) * (TW16 + 2) + dx;
        bv[nb] = as_bf16x8(tile[px * 8 + (ch ^ swz(px))]);
      }
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        acc[0][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w0, bv[nb], acc[0][nb], 0, 0, 0);
        acc[1][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1, bv[nb], acc[1][nb], 0, 0, 0);
      }
    }
  };
#pragma unroll
  for (int tap = 0; tap < 8; tap += 2) {
    tap_step(tap, wa, wb);
    tap_step(tap + 1, wb, wa);
  }
  tap_step(8, wa, wb);
  // epilogue: the input tile's LDS is reused as the waves' staging areas
  __syncthreads();
  uint16_t* out = a.out_bf16 + d.xoff * CNN_F;
  const uint16_t* rref = a.relu_ref ? a.relu_ref + d.xoff * CNN_F : nullptr;
  float bs[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float bs2[EPI == EPI_STATS ? 8 : 1];
#pragma unroll
  for (int e = 0; e < (EPI == EPI_STATS ? 8 : 1); ++e) bs2[e] = 0.f;
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int gy0 = ty0 + wv * 4 + nb * 2;
    auto pix = [&](int i) -> int64_t {
      const int gy = gy0 + (i >> 4), gx = tx0 + (i & 15);
      return (gy < H && gx < W) ? ((int64_t)gy * W + gx) * CNN_F : -1;
    };
    if constexpr (EPI == EPI_BSUM)
      epi_block64_bsum(acc[0][nb], acc[1][nb], (float4*)tile + wv * 512, lane, pix, out, rref, bs);
    else if constexpr (EPI == EPI_STATS)
      epi_block64_stats(acc[0][nb], acc[1][nb], (float4*)tile + wv * 512, lane, pix, bs, bs2);
    else
      epi_block64<EPI == EPI_NORM>(acc[0][nb], acc[1][nb], sbias, sscl, a.mode, (uint2*)tile + wv * 512, lane, pix,
                                   out, rref);
  }
  // 4 waves x 8 KB of fp32 staging end at 32 KB of the 41.5 KB tile
  if constexpr (EPI == EPI_BSUM) bias_partial_store(bs, (float*)((float4*)tile + 4 * 512), bias_slot(a));
  if constexpr (EPI == EPI_STATS) stats_partial_store(bs, bs2, (float*)((float4*)tile + 4 * 512), stat_slot(a));
}

template <int EPI>
__global__ void __launch_bounds__(256, 3) k_conv_mid16(ConvArgs a) {
  static_assert(4 * 512 * sizeof(float4) + 4 * 2 * CNN_F * sizeof(float) <= TILE16_PX * 8 * sizeof(uint4),
                "fp32 staging and wave sums must fit in the tile");
  __shared__ uint4 tile[TILE16_PX * 8];
  __shared__ float sbias[CNN_F];
  __shared__ float sscl[EPI == EPI_NORM ? CNN_F : 1];
  const int b = a.slices[blockIdx.z];
  const SliceDesc d = a.desc[b];
  const int H = d.H, W = d.W;
  const int tx0 = blockIdx.x * TW16, ty0 = blockIdx.y * CONV_TH;
  if (tx0 >= W || ty0 >= H) {
    if (EPI == EPI_BSUM && threadIdx.x < CNN_F) bias_slot(a)[threadIdx.x] = 0.f;
    if (EPI == EPI_STATS && threadIdx.x < 2 * CNN_F) stat_slot(a)[threadIdx.x] = 0.f;
    return;
  }
  const int lane = threadIdx.x & 63;
  const uint16_t* wp = a.wpk + lane * 8;
  uint4 wa[4][2];
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    wa[kc][0] = ldg16(wp + (kc * 2 + 0) * 512);
    wa[kc][1] = ldg16(wp + (kc * 2 + 1) * 512);
  }
  stage_bias<EPI == EPI_NORM>(a, sbias, sscl);
  load_tile64_16(tile, a.in_bf16 + d.xoff * CNN_F, H, W, ty0, tx0);
  __syncthreads();
  mid16_compute<EPI>(tile, sbias, sscl, a, d, ty0, tx0, wa);
}

// ------------------------------------------- 2 -> 64 -> 64, fused (forward)
// The first two layers of the forward pass in one kernel: the first layer's
// output is computed for the second layer's 18 x 18 input tile (its 16 x 16
// output tile plus halo) straight into the LDS tile, zero outside the image
// (the second layer's zero padding), rounded to bf16 as the separate first
// layer rounds it; the second layer then runs as k_conv_mid16.  The first
// layer's activation never goes to HBM (inference only: the reverse pass
// recomputes the activations with the separate kernels).  The first layer
// reads a 20 x 20 complex tile (two-pixel halo); its 324 output pixels form
// 11 MFMA blocks of 32 (the last one partly padding), blocks wv, wv + 4, ...
// to wave wv.  Uses a.in_c (complex input), a.wpk0 / a.bias0 (first layer)
// and a.wpk / a.bias (second layer).
constexpr int TWC = TW16 + 4;                // complex tile width (20)
constexpr int TILEC_PX = (CONV_TH + 4) * TWC;  // 400
constexpr int FUSE_BLOCKS = (TILE16_PX + 31) / 32;  // 11

__global__ void __launch_bounds__(256, 3) k_conv_first_mid(ConvArgs a) {
  __shared__ uint4 tile[TILE16_PX * 8];
  __shared__ uint32_t ctile[TILEC_PX];
  __shared__ float sbias[CNN_F];
  __shared__ float sbias0[CNN_F];
  const int b = a.slices[blockIdx.z];
  const SliceDesc d = a.desc[b];
  const int H = d.H, W = d.W;
  const int tx0 = blockIdx.x * TW16, ty0 = blockIdx.y * CONV_TH;
  if (tx0 >= W || ty0 >= H) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int hsel = lane >> 5, n = lane & 31;
  uint4 wf[2][2];  // first-layer weight fragments
  {
    const uint16_t* wp0 = a.wpk0 + lane * 8;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      wf[k][0] = ldg16(wp0 + (k * 2 + 0) * 512);
      wf[k][1] = ldg16(wp0 + (k * 2 + 1) * 512);
    }
  }
  if (threadIdx.x < CNN_F) {
    sbias[threadIdx.x] = a.bias ? a.bias[threadIdx.x] : 0.f;
    sbias0[threadIdx.x] = a.bias0 ? a.bias0[threadIdx.x] : 0.f;
  }
  {
    const float2* in = a.in_c + d.xoff;
    constexpr int PT = (TILEC_PX + 255) / 256;
    float2 v[PT];
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      const int px = threadIdx.x + 256 * j;
      v[j] = make_float2(0.f, 0.f);
      if (px < TILEC_PX) {
        const int ly = px / TWC, lx = px - ly * TWC;
        const int gy = ty0 + ly - 2, gx = tx0 + lx - 2;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) v[j] = in[(int64_t)gy * W + gx];
      }
    }
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      const int px = threadIdx.x + 256 * j;
      if (px < TILEC_PX) ctile[px] = (uint32_t)f2bf(v[j].x) | ((uint32_t)f2bf(v[j].y) << 16);
    }
  }
  __syncthreads();
  // first layer into the LDS tile
  uint2* t2 = (uint2*)tile;
  for (int blk = wv; blk < FUSE_BLOCKS; blk += 4) {
    const int q = blk * 32 + n;  // tile pixel (18 x 18) of this lane
    const bool qv = q < TILE16_PX;
    const int ly = qv ? q / (TW16 + 2) : 0, lx = qv ? q - ly * (TW16 + 2) : 0;
    f32x16 acc[2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[m][v] = 0.f;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      uint4 raw;
      uint32_t* rw = (uint32_t*)&raw;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int t = s * 8 + hsel * 4 + e;  // tap
        uint32_t v = 0;
        if (t < 9) {
          const int dy = t / 3, dx = t % 3;
          v = ctile[(ly + dy) * TWC + lx + dx];
        }
        rw[e] = v;
      }
      const bf16x8 bv = as_bf16x8(raw);
      acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(wf[s][0]), bv, acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(wf[s][1]), bv, acc[1], 0, 0, 0);
    }
    if (qv) {
      const int gy = ty0 + ly - 1, gx = tx0 + lx - 1;
      const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int co0 = m * 32 + 8 * g + hsel * 4;
          float hv[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float v = acc[m][4 * g + j] + sbias0[co0 + j];
            hv[j] = (inside && v > 0.f) ? v : 0.f;
          }
          uint2 pk;
          pk.x = pack_bf16x2(hv[0], hv[1]);
          pk.y = pack_bf16x2(hv[2], hv[3]);
          const int ch = co0 >> 3;
          t2[(q * 8 + (ch ^ swz(q))) * 2 + hsel] = pk;
        }
    }
  }
  const uint16_t* wp = a.wpk + lane * 8;
  uint4 wa[4][2];
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    wa[kc][0] = ldg16(wp + (kc * 2 + 0) * 512);
    wa[kc][1] = ldg16(wp + (kc * 2 + 1) * 512);
  }
  __syncthreads();
  mid16_compute<EPI_PLAIN>(tile, sbias, nullptr, a, d, ty0, tx0, wa);
}

// ---------------------------------------------------------------- 2 -> 64
// Input: complex image (fp32 pairs), rounded to bf16.  K = 9 taps x 2 channels
// = 18, padded to 32 (two 16-deep MFMA steps).  16 x 16-pixel tiles; each
// wave computes 4 rows x 16 columns x 64 channels (2 pixel blocks).
template <int EPI>
__global__ void __launch_bounds__(256, 4) k_conv_first(ConvArgs a) {
  __shared__ uint32_t tile[TILE1_PX];
  __shared__ float sbias[CNN_F];
  __shared__ float sscl[EPI == EPI_NORM ? CNN_F : 1];
  // epilogue staging: 4 KB per wave (bf16), or 8 KB per wave (fp32) and the
  // waves' channel sums (64 floats each for bias sums, 128 for statistics)
  __shared__ uint4 stage[EPI == EPI_STATS ? 4 * 512 + 2 * CNN_F : EPI == EPI_BSUM ? 4 * 512 + CNN_F : 4 * 256];
  const int b = a.slices[blockIdx.z];
  const SliceDesc d = a.desc[b];
  const int H = d.H, W = d.W;
  const int tx0 = blockIdx.x * TW16, ty0 = blockIdx.y * CONV_TH;
  if (tx0 >= W || ty0 >= H) {
    if (EPI == EPI_BSUM && threadIdx.x < CNN_F) bias_slot(a)[threadIdx.x] = 0.f;
    if (EPI == EPI_STATS && threadIdx.x < 2 * CNN_F) stat_slot(a)[threadIdx.x] = 0.f;
    return;
  }
  const float2* in = a.in_c + d.xoff;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint16_t* wp = a.wpk + lane * 8;
  uint4 wf[2][2];  // all four weight fragments, fetched before the tile
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    wf[k][0] = ldg16(wp + (k * 2 + 0) * 512);
    wf[k][1] = ldg16(wp + (k * 2 + 1) * 512);
  }
  stage_bias<EPI == EPI_NORM>(a, sbias, sscl);
  {
    constexpr int PT = (TILE1_PX + 255) / 256;
    float2 v[PT];
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      const int px = threadIdx.x + 256 * j;
      v[j] = make_float2(0.f, 0.f);
      if (px < TILE1_PX) {
        const int ly = px / (TW16 + 2), lx = px - ly * (TW16 + 2);
        const int gy = ty0 + ly - 1, gx = tx0 + lx - 1;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) v[j] = in[(int64_t)gy * W + gx];
      }
    }
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      const int px = threadIdx.x + 256 * j;
      if (px < TILE1_PX) tile[px] = (uint32_t)f2bf(v[j].x) | ((uint32_t)f2bf(v[j].y) << 16);
    }
  }
  __syncthreads();
  f32x16 acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[m][n][v] = 0.f;
  // pixel n of block nb: row wv * 4 + nb * 2 + n / 16, column n % 16
  const int pbase = (wv * 4 + ((lane & 31) >> 4)) * (TW16 + 2) + (lane & 15);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const bf16x8 w0 = as_bf16x8(wf[s][0]);
    const bf16x8 w1 = as_bf16x8(wf[s][1]);
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      uint4 raw;
      uint32_t* rw = (uint32_t*)&raw;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int t = s * 8 + (lane >> 5) * 4 + e;  // tap
        uint32_t v = 0;
        if (t < 9) {
          const int dy = t / 3, dx = t % 3;
          v = tile[pbase + (nb * 2 + dy) * (TW16 + 2) + dx];
        }
        rw[e] = v;
      }
      const bf16x8 bv = as_bf16x8(raw);
      acc[0][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w0, bv, acc[0][nb], 0, 0, 0);
      acc[1][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1, bv, acc[1][nb], 0, 0, 0);
    }
  }
  uint16_t* out = a.out_bf16 + d.xoff * CNN_F;
  const uint16_t* rref = a.relu_ref ? a.relu_ref + d.xoff * CNN_F : nullptr;
  float bs[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float bs2[EPI == EPI_STATS ? 8 : 1];
#pragma unroll
  for (int e = 0; e < (EPI == EPI_STATS ? 8 : 1); ++e) bs2[e] = 0.f;
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int gy0 = ty0 + wv * 4 + nb * 2;
    auto pix = [&](int i) -> int64_t {
      const int gy = gy0 + (i >> 4), gx = tx0 + (i & 15);
      return (gy < H && gx < W) ? ((int64_t)gy * W + gx) * CNN_F : -1;
    };
    if constexpr (EPI == EPI_BSUM)
      epi_block64_bsum(acc[0][nb], acc[1][nb], (float4*)stage + wv * 512, lane, pix, out, rref, bs);
    else if constexpr (EPI == EPI_STATS)
      epi_block64_stats(acc[0][nb], acc[1][nb], (float4*)stage + wv * 512, lane, pix, bs, bs2);
    else
      epi_block64<EPI == EPI_NORM>(acc[0][nb], acc[1][nb], sbias, sscl, a.mode, (uint2*)stage + wv * 512, lane,
                                   pix, out, rref);
  }
  if constexpr (EPI == EPI_BSUM) bias_partial_store(bs, (float*)((float4*)stage + 4 * 512), bias_slot(a));
  if constexpr (EPI == EPI_STATS) stats_partial_store(bs, bs2, (float*)((float4*)stage + 4 * 512), stat_slot(a));
}

// ---------------------------------------------------------------- 64 -> 2
// v_mfma_f32_16x16x32_bf16 with the two output channels padded to 16 rows;
// 16 x 16-pixel tiles (41.5 KB of LDS, three workgroups a CU); each wave
// covers 4 rows x 16 columns = 4 blocks of 16 pixels.
// Output: out_c = resid + (acc + bias)  (fwd: z = x + N(x); dgrad: g_x).
__global__ void __launch_bounds__(256, 3) k_conv_last(ConvArgs a) {
  __shared__ uint4 tile[TILE16_PX * 8];
  const int b = a.slices[blockIdx.z];
  const SliceDesc d = a.desc[b];
  const int H = d.H, W = d.W;
  const int tx0 = blockIdx.x * TW16, ty0 = blockIdx.y * CONV_TH;
  if (tx0 >= W || ty0 >= H) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint16_t* wp = a.wpk + lane * 8;
  uint4 wf[9][2];  // all 18 weight fragments, fetched before the tile
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    wf[k][0] = ldg16(wp + (k * 2 + 0) * 512);
    wf[k][1] = ldg16(wp + (k * 2 + 1) * 512);
  }
  load_tile64_16(tile, a.in_bf16 + d.xoff * CNN_F, H, W, ty0, tx0);
  __syncthreads();
  f32x4 acc[4];
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[n][v] = 0.f;
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int dy = tap / 3, dx = tap % 3;
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
      const bf16x8 w = as_bf16x8(wf[tap][cc]);
      const int ch = cc * 4 + (lane >> 4);
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        const int px = (wv * 4 + n + dy) * (TW16 + 2) + (lane & 15) + dx;
        const bf16x8 bv = as_bf16x8(tile[px * 8 + (ch ^ swz(px))]);
        acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, bv, acc[n], 0, 0, 0);
      }
    }
  }
  if (lane >= 16) return;
  const float b0 = a.bias ? a.bias[0] : 0.f, b1 = a.bias ? a.bias[1] : 0.f;
  float2* out = a.out_c + d.xoff;
  const float2* res = a.resid ? a.resid + d.xoff : nullptr;
  bool bad = false;
  float2 rv[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    const int gy = ty0 + wv * 4 + n, gx = tx0 + lane;
    rv[n] = (res && gy < H && gx < W) ? res[(int64_t)gy * W + gx] : make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    const int gy = ty0 + wv * 4 + n, gx = tx0 + lane;
    if (gy >= H || gx >= W) continue;
    const int64_t o = (int64_t)gy * W + gx;
    float2 v = make_float2(rv[n].x + acc[n][0] + b0, rv[n].y + acc[n][1] + b1);
    bad |= !isfinite(v.x) || !isfinite(v.y);
    out[o] = v;
  }
  if (bad && a.status) a.status[b] |= FLAG_CNN_NONFINITE;
}

// ------------------------------------------------------------- weight packing
// fp32 master weights W[co][ci][3][3] -> MFMA fragment layouts (see conv.h).
// transpose = 1 packs the dgrad operator (swap co/ci, flip taps).
// W[orig_co][orig_ci][tap] with orig_ci_count input channels.  Plain:
// (co, ci) = (orig_co, orig_ci).  Transposed (dgrad operator): the new
// out-channel is the original in-channel and the taps are mirrored.
__device__ __forceinline__ float wget(const float* Wm, int co, int ci, int tap, int orig_ci_count, int transpose) {
  if (!transpose) return Wm[(co * orig_ci_count + ci) * 9 + tap];
  return Wm[(ci * orig_ci_count + co) * 9 + (8 - tap)];
}

// mid: [9][4][2][64][8]; CO = CI = 64 (after the transpose, too)
__global__ void k_pack_mid(const float* Wm, uint16_t* out, int transpose) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 9 * 4 * 2 * 64 * 8) return;
  const int e = idx & 7, lane = (idx >> 3) & 63, mb = (idx >> 9) & 1, kc = (idx >> 10) & 3, tap = idx >> 12;
  const int co = mb * 32 + (lane & 31), ci = kc * 16 + (lane >> 5) * 8 + e;
  out[idx] = f2bf(wget(Wm, co, ci, tap, 64, transpose));
}

// first: [2 s][2 mb][64][8]; out-channels 64, in-channels 2.
// Forward: original W1 [64][2][3][3].  Transposed: original W5 [2][64][3][3]
// used as the dgrad of the last layer (out = 64 = original ci, in = 2).
__global__ void k_pack_first(const float* Wm, uint16_t* out, int transpose) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * 2 * 64 * 8) return;
  const int e = idx & 7, lane = (idx >> 3) & 63, mb = (idx >> 9) & 1, s = idx >> 10;
  const int co = mb * 32 + (lane & 31);
  const int k = s * 16 + (lane >> 5) * 8 + e;
  const int tap = k >> 1, ci = k & 1;
  float v = 0.f;
  if (tap < 9) v = transpose ? wget(Wm, co, ci, tap, 64, 1) : wget(Wm, co, ci, tap, 2, 0);
  out[idx] = f2bf(v);
}

// last: [9][2 cc][64][8]; out-channels 2 padded to 16, in-channels 64.
// Forward: original W5 [2][64][3][3].  Transposed: original W1 [64][2][3][3]
// used as the dgrad of the first layer (out = 2 = original ci, in = 64).
__global__ void k_pack_last(const float* Wm, uint16_t* out, int transpose) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 9 * 2 * 64 * 8) return;
  const int e = idx & 7, lane = (idx >> 3) & 63, cc = (idx >> 9) & 1, tap = idx >> 10;
  const int co = lane & 15, ci = cc * 32 + (lane >> 4) * 8 + e;
  float v = 0.f;
  if (co < 2) v = transpose ? wget(Wm, co, ci, tap, 2, 1) : wget(Wm, co, ci, tap, 64, 0);
  out[idx] = f2bf(v);
}

hipError_t conv_launch(int kind, const ConvArgs& a, hipStream_t s) {
  dim3 g16(a.tiles_x, a.tiles_y, a.nslices);
  const int epi = (a.mode == CONV_DGRAD && a.bias_part) ? EPI_BSUM
                  : a.mode == CONV_STATS                 ? EPI_STATS
                  : a.mode == CONV_NORM                  ? EPI_NORM
                                                         : EPI_PLAIN;
  if (a.mode == CONV_STATS && !a.stat_part) return hipErrorInvalidValue;
  if (a.mode == CONV_NORM && !a.bn_stats) return hipErrorInvalidValue;
  if (kind == 0) {
    if (epi == EPI_BSUM) hipLaunchKernelGGL(k_conv_first<EPI_BSUM>, g16, dim3(256), 0, s, a);
    else if (epi == EPI_STATS) hipLaunchKernelGGL(k_conv_first<EPI_STATS>, g16, dim3(256), 0, s, a);
    else if (epi == EPI_NORM) hipLaunchKernelGGL(k_conv_first<EPI_NORM>, g16, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_conv_first<EPI_PLAIN>, g16, dim3(256), 0, s, a);
  } else if (kind == 1) {
    if (epi == EPI_BSUM) hipLaunchKernelGGL(k_conv_mid16<EPI_BSUM>, g16, dim3(256), 0, s, a);
    else if (epi == EPI_STATS) hipLaunchKernelGGL(k_conv_mid16<EPI_STATS>, g16, dim3(256), 0, s, a);
    else if (epi == EPI_NORM) hipLaunchKernelGGL(k_conv_mid16<EPI_NORM>, g16, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_conv_mid16<EPI_PLAIN>, g16, dim3(256), 0, s, a);
  }
  else if (kind == 2) hipLaunchKernelGGL(k_conv_last, g16, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_conv_first_mid, g16, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t pack_weights(int kind, const float* Wm, uint16_t* out, int transpose, hipStream_t s) {
  if (kind == 0) hipLaunchKernelGGL(k_pack_first, dim3(8), dim3(256), 0, s, Wm, out, transpose);
  else if (kind == 1) hipLaunchKernelGGL(k_pack_mid, dim3(144), dim3(256), 0, s, Wm, out, transpose);
  else hipLaunchKernelGGL(k_pack_last, dim3(36), dim3(256), 0, s, Wm, out, transpose);
  return hipGetLastError();
}

}  // namespace mrx
