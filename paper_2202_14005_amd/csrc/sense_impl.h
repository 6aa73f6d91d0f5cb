// Kernel templates for the SENSE column and row passes.  Included by the
// per-length instantiation units only.
#pragma once
#include <type_traits>

#include "fft.h"
#include "sense_kernels.h"

namespace mrx {

// Non-temporal 8-byte load (second read of a coil map within a workgroup;
// also keeps the compiler from holding the first read live in registers).
__device__ __forceinline__ float2 ld_stream(const float2* p) {
  const unsigned long long v = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long*>(p));
  return __builtin_bit_cast(float2, v);
}

// Raw buffer access to one plane: a scalar descriptor (base and extent in
// bytes), a per-lane byte offset and a wave-uniform byte offset, so that a
// load or store costs no vector address arithmetic.  Offsets at or past the
// extent read zero and drop stores (the hardware's range check).
struct BufPlane {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ BufPlane(const void* base, uint32_t bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000)) {}
  __device__ __forceinline__ float2 ld(uint32_t voff, uint32_t soff) const {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
  }
  // non-temporal (second read of a coil map within a workgroup)
  __device__ __forceinline__ float2 ld_nt(uint32_t voff, uint32_t soff) const {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 2));
  }
  __device__ __forceinline__ void st(float2 v, uint32_t voff, uint32_t soff) const {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, (int)voff, (int)soff, 0);
  }
};

// Column-pass workgroup -> (slice, column tile) unit of a 1-D grid padded
// to 16 workgroups.  Tiles narrower than a 128-byte row segment pair up: the
// two tiles of a segment are 8 workgroups apart, so they run on one XCD (the
// chip deals consecutive workgroups to the 8 XCDs in turn) and read each
// segment through one L2.
template <int WT>
__device__ __forceinline__ int col_pass_unit(int Lb) {
  if constexpr (WT * 8 >= 128) return Lb;
  else return (((Lb >> 4) * 8 + (Lb & 7)) << 1) + ((Lb >> 3) & 1);
}
inline dim3 col_pass_grid(int tiles, int nslices) { return dim3((unsigned)(((tiles * nslices + 15) / 16) * 16)); }

// Deterministic fixed-order sum of n floats by one wavefront: lane l adds
// elements l, l+64, ... in order, then a fixed butterfly over lanes.
__device__ __forceinline__ float wave_sum_fixed(const float* a, int n, int lane) {
  float s = 0.f;
  for (int i = lane; i < n; i += 64) s += a[i];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

// Block-wide fixed-order reduction of one float per thread (blockDim <= 1024).
// Returns the sum to every thread.  red must hold blockDim/64 floats.
__device__ __forceinline__ float block_sum_fixed(float v, float* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  float s = 0.f;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

// --------------------------------------------------------- normal operator
// One workgroup = WT adjacent columns of one slice.  G groups of T x WT
// threads each take every G-th coil of that column tile:
//   acc_g = sum_{c = g, g+G, ...} conj(S_c) F_H^H diag(m') F_H (S_c p),
// then the G partial sums are added through LDS in a fixed order and
// q = sum_g acc_g + lambda p.  Every coil map is read from HBM once per
// application (the conjugate multiply re-reads it from L2).  All groups run
// the same number of coil iterations (idle ones on zeros) so that every
// barrier inside the transforms is reached by the whole workgroup.
//
// Launch: a 1-D grid over (slice, tile) pairs arranged so that tiles 2k and
// 2k+1 of a slice (which share 128-byte lines when WT = 8) get block ids
// that differ by 8 and so land on the same XCD (workgroups are dispatched
// to the 8 XCDs round-robin) and share its L2.
// KS: keep the coil values in registers for the conjugate multiply instead
// of re-reading them from L2.
template <class Sd, int WT, int G, bool KS, int KSPL>
__global__ void __launch_bounds__(Sd::T * WT * G, 2)
k_normal(NormalArgs a) {
  constexpr int N = Sd::N, P = Sd::P, T = Sd::T, NT = T * WT;
  using L = LdsInterleaved<N, WT>;
  __shared__ float2 lds[G * L::SIZE];
  __shared__ float2 tw[N];
  __shared__ float mk[N];
  __shared__ float red[(NT * G + 63) / 64];
  __shared__ float sc[2];

  const int Lb = blockIdx.x;
  int ks, tg;
  if constexpr (KSPL > 1) {
    // consecutive workgroups go to the 8 XCDs in turn: the KSPL splits of a
    // tile, 8 workgroups apart, run on one XCD and share p and r in its L2
    // -- with tiles narrower than a 128-byte row segment, the splits of the
    // RUN adjacent tiles that share each segment
    constexpr int RUN = WT * 8 >= 128 ? 1 : 128 / (WT * 8), PER = 8 * RUN * KSPL;
    const int w = (Lb >> 3) % (RUN * KSPL);
    tg = RUN * ((Lb / PER) * 8 + (Lb & 7)) + w / KSPL;
    ks = w % KSPL;
  } else {
    tg = (((Lb >> 4) * 8 + (Lb & 7)) << 1) + ((Lb >> 3) & 1);
    ks = 0;
  }
  const int si = tg / a.tiles, tile = tg % a.tiles;
  if (si >= a.nslices) return;
  const int b = a.slices[si];
  const SliceDesc d = a.desc[b];
  if (d.H != N) return;
  const int W = d.W;
  if (tile * WT >= W) return;
  // this workgroup's coils: [c_begin, c_end) of the slice's C
  const int c_begin = (ks * d.C) / KSPL, c_end = ((ks + 1) * d.C) / KSPL;
  const int lid = threadIdx.x;
  static_assert(G == 1 || NT % 64 == 0, "a coil group must be whole wavefronts");
  const int grp = G > 1 ? __builtin_amdgcn_readfirstlane(lid / NT) : 0;  // wave-uniform
  const int l2 = lid % NT;
  const int c = l2 % WT, tc = l2 / WT;
  const int col = tile * WT + c;
  const bool valid = col < W;
  // element (a1(tc, i, r), col) of a plane with row stride W: one per-lane
  // byte offset and a wave-uniform one per (i, r).  Lanes past the last
  // column (a ragged tile) read column W - 1 instead: columns transform
  // independently, so their results are only left unstored and out of the
  // dot product, and every load stays unpredicated.
  const uint32_t voff = (uint32_t)(tc * W + (valid ? col : W - 1)) * 8u;
  auto so = [&](int i, int r) { return (uint32_t)((T * i + r * Sd::M1) * W) * 8u; };
  const uint32_t pbytes = (uint32_t)N * (uint32_t)W * 8u;
  const bool cg = a.mode == 1;
  if (cg && a.stopped[b]) return;
  float2* xl = lds + grp * L::SIZE;

  for (int i = lid; i < N; i += NT * G) {
    tw[i] = a.tw[i];
    mk[i] = a.mask[d.moff + (i + N / 2) % N] * (1.0f / N);
  }
  if (cg && lid < 64) {
    float beta = 0.f;
    if (a.iter > 0) {
      const float rc = wave_sum_fixed(a.rr_cur + (int64_t)b * a.nrr, a.nrr, lid);
      const float rp = wave_sum_fixed(a.rr_prev + (int64_t)b * a.nrr, a.nrr, lid);
      beta = rp > 0.f ? rc / rp : 0.f;
    }
    if (lid == 0) sc[0] = beta;
  }
  __syncthreads();

  // The first coil's values are loaded ahead of the operand (and, in CG
  // steps, of r), so that the two memory latencies overlap; v holds them
  // until the first coil iteration.
  const int64_t plane = (int64_t)N * W;
  const float2* Sb = a.S + d.soff;
  const int gc0 = c_begin + grp;  // this group's first coil (or, idle, a real one)
  float2 v[P];
  {
    const BufPlane S0(Sb + (int64_t)(gc0 < c_end ? gc0 : c_begin) * plane, pbytes);
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
      for (int r = 0; r < Sd::N1; ++r) v[i * Sd::N1 + r] = S0.ld(voff, so(i, r));
  }

  const BufPlane pin(a.pin + d.xoff, pbytes);
  float2 p[P];
  if (cg && a.iter > 0) {
    const float beta = sc[0];
    const BufPlane rin(a.r + d.xoff, pbytes), pout(a.pout + d.xoff, pbytes);
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
      for (int r = 0; r < Sd::N1; ++r) {
        float2 pv = pin.ld(voff, so(i, r));
        const float2 rv = rin.ld(voff, so(i, r));
        pv = make_float2(rv.x + beta * pv.x, rv.y + beta * pv.y);
        p[i * Sd::N1 + r] = pv;
      }
    // p updated in place (pout == pin): every group must have read the old
    // values before group 0 writes the new ones.  With a coil split the
    // workgroups of a tile all read pin, so pout must be another buffer; the
    // first split writes it.
    if (G > 1 && a.pout == a.pin) __syncthreads();
    if (valid && grp == 0 && ks == 0) {
#pragma unroll
      for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
        for (int r = 0; r < Sd::N1; ++r) pout.st(p[i * Sd::N1 + r], voff, so(i, r));
    }
  } else {
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
      for (int r = 0; r < Sd::N1; ++r) p[i * Sd::N1 + r] = pin.ld(voff, so(i, r));
  }


  float2 acc[P];
#pragma unroll
  for (int k = 0; k < P; ++k) acc[k] = make_float2(0.f, 0.f);

  const int iters = (c_end - c_begin + G - 1) / G;
  for (int it = 0; it < iters; ++it) {
    const int coil = c_begin + it * G + grp;
    const bool on = coil < c_end;  // wave-uniform: idle groups run on a real coil's values
    const BufPlane Sc(Sb + (int64_t)(on ? coil : c_begin) * plane, pbytes);
    if (it > 0) {
#pragma unroll
      for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
        for (int r = 0; r < Sd::N1; ++r) v[i * Sd::N1 + r] = Sc.ld(voff, so(i, r));
    }
    float2 sk[KS ? P : 1];
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const float2 s = v[k];
      if constexpr (KS) sk[k] = s;
      v[k] = cmul(s, p[k]);
    }
    // (the tile region xl sees only this chain of transforms until the coil
    // loop ends, so the exchanges need no barrier before their writes)
    fft_forward<Sd, L, BlockSyncPost>(v, xl, tw, tc, c);
    // the mask (with the 1/N of the two unnormalised transforms) scales the
    // spectrum inside the inverse transform's first codelet
    fft_inverse<Sd, L, BlockSyncPost, FreqScale>(v, xl, tw, tc, c, FreqScale{mk});
    if (on) {
#pragma unroll
      for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
        for (int r = 0; r < Sd::N1; ++r) {
          const int k = i * Sd::N1 + r;
          float2 s;
          if constexpr (KS) s = sk[k];
          else s = Sc.ld_nt(voff, so(i, r));
          acc[k] = cadd(acc[k], cmulc(s, v[k]));
        }
    }
  }

  if constexpr (G > 1) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
      for (int r = 0; r < Sd::N1; ++r) xl[L::idx(Sd::a1(tc, i, r), c)] = acc[i * Sd::N1 + r];
    __syncthreads();
    if (grp == 0) {
#pragma unroll
      for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
        for (int r = 0; r < Sd::N1; ++r) {
          const int id = L::idx(Sd::a1(tc, i, r), c);
          float2 s = lds[id];
#pragma unroll
          for (int g = 1; g < G; ++g) s = cadd(s, lds[g * L::SIZE + id]);
          acc[i * Sd::N1 + r] = s;
        }
    }
  }

  // the first split adds lambda p; each split writes its own partial plane
  const float lam = (a.lam && ks == 0) ? a.lam[b] : 0.f;
  float dot = 0.f;
  if (grp == 0) {
    const BufPlane qout(a.qout + (int64_t)ks * a.qstride + d.xoff, pbytes);
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
      for (int r = 0; r < Sd::N1; ++r) {
        const int k = i * Sd::N1 + r;
        const float2 q = make_float2(acc[k].x + lam * p[k].x, acc[k].y + lam * p[k].y);
        dot += p[k].x * q.x + p[k].y * q.y;
        if (valid) qout.st(q, voff, so(i, r));
      }
    if (!valid) dot = 0.f;
  }
  if (cg) {
    const float s = block_sum_fixed(dot, red);
    if (lid == 0) a.pq_part[(int64_t)b * a.npq + tile * KSPL + ks] = s;
  }
}

// ------------------------------------- normal operator, wave-local variant
// Each wavefront owns CW = 64 / T adjacent columns and transforms them with
// its own LDS region, so the exchanges inside the transforms need no
// workgroup barrier and the wavefronts of a workgroup drift freely.  The G
// wavefronts of a workgroup work on the same CW columns and take every G-th
// coil; the coil map of a wavefront's next coil is loaded while the current
// one is transformed, and the current one is re-read (from L2) for the
// conjugate multiply.  The G partial sums are added through LDS in a fixed
// order at the end.
//
// Launch: 1-D grid over (slice, column tile) pairs, rounded up to a multiple
// of 32, arranged so that four consecutive tiles (CW = 4: one 128-byte row
// segment) get block ids 8 apart and land on the same XCD and its L2.
template <class Sd, int G, bool PAD>
__global__ void __launch_bounds__(64 * G, 2)
k_normal_wl(NormalArgs a) {
  constexpr int N = Sd::N, P = Sd::P, T = Sd::T, CW = 64 / T;
  static_assert(64 % T == 0, "a transform must fit in one wavefront");
  using L = std::conditional_t<PAD && Sd::LEVELS == 3 && Sd::N3 % 4 == 0, LdsPadded<N, CW, Sd::N3>,
                               LdsInterleaved<N, CW>>;
  __shared__ float2 lds[G * L::SIZE];
  __shared__ float2 pl[N * CW];
  __shared__ float2 tw[N];
  __shared__ float mk[N];
  __shared__ float sc[1];

  const int Lb = blockIdx.x;
  const int k8 = Lb >> 3;
  const int tg = (((k8 >> 2) * 8 + (Lb & 7)) << 2) + (k8 & 3);
  const int si = tg / a.tiles, tile = tg % a.tiles;
  if (si >= a.nslices) return;
  const int b = a.slices[si];
  const SliceDesc d = a.desc[b];
  if (d.H != N) return;
  const int W = d.W;
  if (tile * CW >= W) return;
  const bool cg = a.mode == 1;
  if (cg && a.stopped[b]) return;
  const int lid = threadIdx.x, lane = lid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(lid >> 6);
  const int c = lane % CW, tc = lane / CW;
  const int col = tile * CW + c;
  const bool valid = col < W;
  // Columns past W (ragged last tile) read column 0 instead: their transforms
  // are independent of the others and their results are never stored.
  const unsigned colv = valid ? (unsigned)col : 0u;
  // Coil-map and image elements of register slot (i, r) sit at row
  // tc + T i + M1 r: a per-thread offset plus a wave-uniform row offset.
  const unsigned toff = ((unsigned)tc * (unsigned)W + colv) * (unsigned)sizeof(float2);  // bytes
  float2* xl = lds + wv * L::SIZE;

  for (int i = lid; i < N; i += 64 * G) {
    tw[i] = a.tw[i];
    mk[i] = a.mask[d.moff + (i + N / 2) % N] * (1.0f / N);
  }
  if (cg && lid < 64) {
    float beta = 0.f;
    if (a.iter > 0) {
      const float rc = wave_sum_fixed(a.rr_cur + (int64_t)b * a.nrr, a.nrr, lid);
      const float rp = wave_sum_fixed(a.rr_prev + (int64_t)b * a.nrr, a.nrr, lid);
      beta = rp > 0.f ? rc / rp : 0.f;
    }
    if (lid == 0) sc[0] = beta;
  }
  __syncthreads();

  // The operand tile (N rows x CW columns, element (row, j) at LDS row * CW + j)
  // is loaded once per workgroup; in CG mode it is first replaced by
  // r + beta p and written back (each element by the thread that read it).
  {
    const bool upd = cg && a.iter > 0;
    const float beta = upd ? sc[0] : 0.f;
    const float2* pbase = a.pin + d.xoff;
    const float2* rbase = a.r + d.xoff;
    float2* pobase = a.pout + d.xoff;
    for (int e = lid; e < N * CW; e += 64 * G) {
      const int row = e / CW, j = e % CW;
      const int cc = tile * CW + j;
      float2 pv = make_float2(0.f, 0.f);
      if (cc < W) {
        const unsigned o = (unsigned)row * (unsigned)W + (unsigned)cc;
        pv = pbase[o];
        if (upd) {
          const float2 rv = rbase[o];
          pv = make_float2(rv.x + beta * pv.x, rv.y + beta * pv.y);
          pobase[o] = pv;
        }
      }
      pl[e] = pv;
    }
  }
  __syncthreads();

  float2 acc[P];
#pragma unroll
  for (int k = 0; k < P; ++k) acc[k] = make_float2(0.f, 0.f);

  const unsigned plane = (unsigned)N * (unsigned)W;
  const float2* Sb = a.S + d.soff;
  const float2* plt = pl + tc * CW + c;  // operand slot (i, r) at plt[(T i + M1 r) CW]
  // Coil-map rows through a buffer resource on the coil plane: the row offset
  // of slot (i, r) is wave-uniform, the column offset per thread, so the
  // loads need no vector address arithmetic.
  auto plane_rsrc = [&](int coil) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)(Sb + (size_t)coil * plane), (short)0,
                                             (int)(plane * sizeof(float2)), 0x00020000);
  };
  auto load_coil = [&](float2* dst, int coil) {
    const auto rs = plane_rsrc(coil);
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
      for (int r = 0; r < Sd::N1; ++r) {
        const unsigned so = (unsigned)((T * i + Sd::M1 * r) * W) * (unsigned)sizeof(float2);
        dst[i * Sd::N1 + r] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, toff, so, 0));
      }
  };
  auto body = [&](const float2* sv, int coil) {
    float2 v[P];
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
      for (int r = 0; r < Sd::N1; ++r) {
        const int k = i * Sd::N1 + r;
        v[k] = cmul(sv[k], plt[(T * i + Sd::M1 * r) * CW]);
      }
    fft_forward<Sd, L, WaveSync>(v, xl, tw, tc, c);
    // the mask (with the 1/N of the two unnormalised transforms) scales the
    // spectrum inside the inverse transform's first codelet
    fft_inverse<Sd, L, WaveSync, FreqScale>(v, xl, tw, tc, c, FreqScale{mk});
    // the conjugate multiply re-reads this coil's values (non-temporal; an
    // L2 hit)
    const auto rs = plane_rsrc(coil);
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
      for (int r = 0; r < Sd::N1; ++r) {
        const int k = i * Sd::N1 + r;
        const unsigned so = (unsigned)((T * i + Sd::M1 * r) * W) * (unsigned)sizeof(float2);
        const float2 s2 = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, toff, so, 2));
        acc[k] = cadd(acc[k], cmulc(s2, v[k]));
      }
  };
  // two register buffers for the coil maps: the next coil's values load
  // while the current coil is transformed
  float2 sa[P], sb[P];
  if (wv < d.C) load_coil(sa, wv);
  for (int coil = wv; coil < d.C; coil += 2 * G) {
    if (coil + G < d.C) load_coil(sb, coil + G);
    body(sa, coil);
    if (coil + G >= d.C) break;
    if (coil + 2 * G < d.C) load_coil(sa, coil + 2 * G);
    body(sb, coil + G);
  }

  if constexpr (G > 1) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
      for (int r = 0; r < Sd::N1; ++r) xl[L::idx(Sd::a1(tc, i, r), c)] = acc[i * Sd::N1 + r];
    __syncthreads();
    if (wv == 0) {
#pragma unroll
      for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
        for (int r = 0; r < Sd::N1; ++r) {
          const int id = L::idx(Sd::a1(tc, i, r), c);
          float2 t = lds[id];
#pragma unroll
          for (int g = 1; g < G; ++g) t = cadd(t, lds[g * L::SIZE + id]);
          acc[i * Sd::N1 + r] = t;
        }
    }
  }

  if (wv == 0) {
    const float lam = a.lam ? a.lam[b] : 0.f;
    float dot = 0.f;
    float2* qbase = a.qout + d.xoff;
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
      for (int r = 0; r < Sd::N1; ++r) {
        const int k = i * Sd::N1 + r;
        const float2 pv = plt[(T * i + Sd::M1 * r) * CW];
        const float2 q = make_float2(acc[k].x + lam * pv.x, acc[k].y + lam * pv.y);
        dot += pv.x * q.x + pv.y * q.y;
        if (valid) qbase[(unsigned)Sd::a1(tc, i, r) * (unsigned)W + colv] = q;
      }
    if (cg) {
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) dot += __shfl_xor(dot, off, 64);
      if (lane == 0) a.pq_part[(int64_t)b * a.npq + tile] = dot;
    }
  }
}

// ----------------------------------------------- forward column pass (A, H)
// v = S_c x, transform along H, keep sampled rows: out[c, k, :] for m[k] = 1
// gets (-1)^j (F v)[j] / sqrt(H) with k = (j + H/2) mod H.
template <class Sd, int WT>
__global__ void __launch_bounds__(Sd::T * WT)
k_fwd_col(SenseColArgs a) {
  constexpr int N = Sd::N, P = Sd::P, T = Sd::T;
  using L = LdsInterleaved<N, WT>;
  __shared__ float2 lds[L::SIZE];
  __shared__ float2 tw[N];
  const int unit = col_pass_unit<WT>(blockIdx.x), si = unit / a.tiles, tile = unit % a.tiles;
  if (si >= a.nslices) return;
  const int b = a.slices[si];
  const SliceDesc d = a.desc[b];
  if (d.H != N) return;
  const int W = d.W;
  if (tile * WT >= W) return;
  const int lid = threadIdx.x, c = lid % WT, tc = lid / WT, col = tile * WT + c;
  const bool valid = col < W;
  for (int i = lid; i < N; i += T * WT) tw[i] = a.tw[i];
  __syncthreads();
  const float scale = rsqrtf((float)N);
  float2 x[P];
#pragma unroll
  for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
    for (int r = 0; r < Sd::N1; ++r)
      x[i * Sd::N1 + r] = valid ? a.in[d.xoff + (int64_t)Sd::a1(tc, i, r) * W + col] : make_float2(0.f, 0.f);
  const int64_t plane = (int64_t)N * W;
  const float* mrow = a.mask + d.moff;
  for (int coil = 0; coil < d.C; ++coil) {
    const float2* Sc = a.S + d.soff + coil * plane;
    float2 v[P];
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
      for (int r = 0; r < Sd::N1; ++r) {
        const float2 s = valid ? Sc[(int64_t)Sd::a1(tc, i, r) * W + col] : make_float2(0.f, 0.f);
        v[i * Sd::N1 + r] = cmul(s, x[i * Sd::N1 + r]);
      }
    fft_forward<Sd, L>(v, lds, tw, tc, c);
    float2* oc = a.out + d.soff + coil * plane;
#pragma unroll
    for (int i = 0; i < Sd::GFIN; ++i)
#pragma unroll
      for (int r = 0; r < Sd::NFIN; ++r) {
        const int j = Sd::freq(tc, i, r);
        const int k = (j + N / 2) % N;
        const float sg = (j & 1) ? -scale : scale;
        if (valid && mrow[k] != 0.f) oc[(int64_t)k * W + col] = cscale(v[i * Sd::NFIN + r], sg);
      }
  }
}

// ------------------------------------------- adjoint column pass (A^H, H)
// For each coil: gather sampled rows of the row-pass output into frequency
// order with the centering sign, inverse transform along H, multiply by
// conj(S_c) and accumulate over coils.  G groups of T x WT threads take
// every G-th coil (all groups run the same number of transforms, idle ones
// on zeros, so every barrier is reached by the whole workgroup); their sums
// are added through LDS in a fixed order.
template <class Sd, int WT, int G>
__global__ void __launch_bounds__(Sd::T * WT * G, 2)
k_adj_col(SenseColArgs a) {
  constexpr int N = Sd::N, P = Sd::P, T = Sd::T, NT = T * WT;
  using L = LdsInterleaved<N, WT>;
  __shared__ float2 lds[G * L::SIZE];
  __shared__ float2 tw[N];
  __shared__ float mk[N];
  const int unit = col_pass_unit<WT>(blockIdx.x), si = unit / a.tiles, tile = unit % a.tiles;
  if (si >= a.nslices) return;
  const int b = a.slices[si];
  const SliceDesc d = a.desc[b];
  if (d.H != N) return;
  const int W = d.W;
  if (tile * WT >= W) return;
  const int lid = threadIdx.x, grp = lid / NT, l2 = lid % NT;
  const int c = l2 % WT, tc = l2 / WT, col = tile * WT + c;
  const bool valid = col < W;
  float2* xl = lds + grp * L::SIZE;
  for (int i = lid; i < N; i += NT * G) {
    tw[i] = a.tw[i];
    mk[i] = a.mask[d.moff + i];
  }
  __syncthreads();
  const float scale = rsqrtf((float)N);
  const int64_t plane = (int64_t)N * W;
  // coil-map element (a1(tc, i, r), col): per-lane offset + uniform row part
  const uint32_t voff = (uint32_t)(tc * W + col) * 8u;
  auto at = [&](const float2* base, int i, int r) {
    return (const float2*)((const char*)(base + (T * i + r * Sd::M1) * W) + voff);
  };
  float2 acc[P];
#pragma unroll
  for (int k = 0; k < P; ++k) acc[k] = make_float2(0.f, 0.f);
  const int iters = (d.C + G - 1) / G;
  for (int it = 0; it < iters; ++it) {
    const int coil = it * G + grp;
    const bool on = valid && coil < d.C;
    const int cc = coil < d.C ? coil : 0;
    const float2* ic = a.in + d.soff + cc * plane;
    float2 v[P];
#pragma unroll
    for (int i = 0; i < Sd::GFIN; ++i)
#pragma unroll
      for (int r = 0; r < Sd::NFIN; ++r) {
        const int j = Sd::freq(tc, i, r);
        const int k = (j + N / 2) % N;
        const float sg = (j & 1) ? -scale : scale;
        float2 u = make_float2(0.f, 0.f);
        if (on && mk[k] != 0.f) u = cscale(ic[(int64_t)k * W + col], sg);
        v[i * Sd::NFIN + r] = u;
      }
    fft_inverse<Sd, L>(v, xl, tw, tc, c);
    if (on) {
      const float2* Sc = a.S + d.soff + cc * plane;
#pragma unroll
      for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
        for (int r = 0; r < Sd::N1; ++r)
          acc[i * Sd::N1 + r] = cadd(acc[i * Sd::N1 + r], cmulc(*at(Sc, i, r), v[i * Sd::N1 + r]));
    }
  }
  if constexpr (G > 1) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
      for (int r = 0; r < Sd::N1; ++r) xl[L::idx(Sd::a1(tc, i, r), c)] = acc[i * Sd::N1 + r];
    __syncthreads();
    if (grp == 0) {
#pragma unroll
      for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
        for (int r = 0; r < Sd::N1; ++r) {
          const int id = L::idx(Sd::a1(tc, i, r), c);
          float2 sm = lds[id];
#pragma unroll
          for (int g = 1; g < G; ++g) sm = cadd(sm, lds[g * L::SIZE + id]);
          acc[i * Sd::N1 + r] = sm;
        }
    }
  }
  if (grp == 0 && valid) {
#pragma unroll
    for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
      for (int r = 0; r < Sd::N1; ++r) a.out[d.xoff + (int64_t)Sd::a1(tc, i, r) * W + col] = acc[i * Sd::N1 + r];
  }
}

// ----------------------------------------------------- row passes (along W)
// One workgroup = WT rows (of any slices' coil planes), T threads per row;
// grid.x enumerates (slice, coil, row-block) via blockIdx.x over
// ceil(H/WT) * C row blocks of slice blockIdx.y.
template <class Sd, int WT>
__global__ void __launch_bounds__(Sd::T * WT)
k_fwd_row(SenseRowArgs a) {
  constexpr int N = Sd::N, P = Sd::P, T = Sd::T;
  using L = LdsContig<N, WT>;
  __shared__ float2 lds[L::SIZE];
  __shared__ float2 tw[N];
  const int b = a.slices[blockIdx.y];
  const SliceDesc d = a.desc[b];
  if (d.W != N) return;
  const int H = d.H;
  const int rblocks = (H + WT - 1) / WT;
  if ((int)blockIdx.x >= rblocks * d.C) return;
  const int coil = blockIdx.x / rblocks, rb = blockIdx.x % rblocks;
  const int lid = threadIdx.x, tc = lid % T, c = lid / T;
  const int row = rb * WT + c;
  for (int i = lid; i < N; i += T * WT) tw[i] = a.tw[i];
  __syncthreads();
  const bool valid = row < H;
  const bool sampled = valid && a.mask[d.moff + row] != 0.f;
  const int64_t base = d.soff + ((int64_t)coil * H + row) * N;
  float2 v[P];
#pragma unroll
  for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
    for (int r = 0; r < Sd::N1; ++r)
      v[i * Sd::N1 + r] = sampled ? a.in[base + Sd::a1(tc, i, r)] : make_float2(0.f, 0.f);
  fft_forward<Sd, L>(v, lds, tw, tc, c);
  if (!valid) return;
  const float scale = rsqrtf((float)N);
#pragma unroll
  for (int i = 0; i < Sd::GFIN; ++i)
#pragma unroll
    for (int r = 0; r < Sd::NFIN; ++r) {
      const int j = Sd::freq(tc, i, r);
      const int l = (j + N / 2) % N;
      const float sg = (j & 1) ? -scale : scale;
      float2 y = make_float2(0.f, 0.f);
      if (sampled) {
        y = cscale(v[i * Sd::NFIN + r], sg);
        if (a.noise) y = cadd(y, a.noise[base + l]);
      }
      a.out[base + l] = y;
    }
}

template <class Sd, int WT>
__global__ void __launch_bounds__(Sd::T * WT)
k_adj_row(SenseRowArgs a) {
  constexpr int N = Sd::N, P = Sd::P, T = Sd::T;
  using L = LdsContig<N, WT>;
  __shared__ float2 lds[L::SIZE];
  __shared__ float2 tw[N];
  const int b = a.slices[blockIdx.y];
  const SliceDesc d = a.desc[b];
  if (d.W != N) return;
  const int H = d.H;
  const int rblocks = (H + WT - 1) / WT;
  if ((int)blockIdx.x >= rblocks * d.C) return;
  const int coil = blockIdx.x / rblocks, rb = blockIdx.x % rblocks;
  const int lid = threadIdx.x, tc = lid % T, c = lid / T;
  const int row = rb * WT + c;
  for (int i = lid; i < N; i += T * WT) tw[i] = a.tw[i];
  __syncthreads();
  const bool valid = row < H;
  const bool sampled = valid && a.mask[d.moff + row] != 0.f;
  const int64_t base = d.soff + ((int64_t)coil * H + row) * N;
  const float scale = rsqrtf((float)N);
  float2 v[P];
#pragma unroll
  for (int i = 0; i < Sd::GFIN; ++i)
#pragma unroll
    for (int r = 0; r < Sd::NFIN; ++r) {
      const int j = Sd::freq(tc, i, r);
      const int l = (j + N / 2) % N;
      const float sg = (j & 1) ? -scale : scale;
      v[i * Sd::NFIN + r] = sampled ? cscale(a.in[base + l], sg) : make_float2(0.f, 0.f);
    }
  fft_inverse<Sd, L>(v, lds, tw, tc, c);
  if (!sampled) return;
#pragma unroll
  for (int i = 0; i < Sd::G1; ++i)
#pragma unroll
    for (int r = 0; r < Sd::N1; ++r) a.out[base + Sd::a1(tc, i, r)] = v[i * Sd::N1 + r];
}

// ------------------------------------------------------------- launchers
// CG steps (mode 1) split each column tile's coils over KSPL workgroups
// writing partial planes that the CG update adds (a.qstride apart; pin and
// pout must then differ); operator applications (mode 0) do the same when the
// caller asks for it (split_plain, partial planes then added by the caller)
// and otherwise run unsplit.
template <class Sd, int WT, int G, bool KS, int KSPL>
hipError_t launch_normal(const NormalArgs& a0, int maxW, hipStream_t s) {
  NormalArgs a = a0;
  a.tiles = (maxW + WT - 1) / WT;
  if ((a.mode == 1 || a.split_plain) && KSPL > 1) {
    if (a.mode == 1 && (a.tiles * KSPL > a.npq || (a.iter > 0 && a.pin == a.pout))) return hipErrorInvalidValue;
    if (a.qstride <= 0) return hipErrorInvalidValue;
    const int total = a.tiles * a.nslices * KSPL, per = 8 * (WT * 8 >= 128 ? 1 : 128 / (WT * 8)) * KSPL;
    dim3 grid((unsigned)(((total + per - 1) / per) * per));
    hipLaunchKernelGGL((k_normal<Sd, WT, G, KS, KSPL>), grid, dim3(Sd::T * WT * G), 0, s, a);
  } else {
    const int total = a.tiles * a.nslices;
    dim3 grid((unsigned)(((total + 15) / 16) * 16));
    hipLaunchKernelGGL((k_normal<Sd, WT, G, KS, 1>), grid, dim3(Sd::T * WT * G), 0, s, a);
  }
  return hipGetLastError();
}
template <class Sd, int G, bool PAD>
hipError_t launch_normal_wl(const NormalArgs& a0, int maxW, hipStream_t s) {
  constexpr int CW = 64 / Sd::T;
  NormalArgs a = a0;
  a.tiles = (maxW + CW - 1) / CW;
  const int total = a.tiles * a.nslices;
  dim3 grid((unsigned)(((total + 31) / 32) * 32));
  hipLaunchKernelGGL((k_normal_wl<Sd, G, PAD>), grid, dim3(64 * G), 0, s, a);
  return hipGetLastError();
}
template <class Sd, int WT>
hipError_t launch_fwd_col(const SenseColArgs& a, int maxW, hipStream_t s) {
  SenseColArgs c = a;
  c.tiles = (maxW + WT - 1) / WT;
  hipLaunchKernelGGL((k_fwd_col<Sd, WT>), col_pass_grid(c.tiles, c.nslices), dim3(Sd::T * WT), 0, s, c);
  return hipGetLastError();
}
// The adjoint column pass uses its own tile: 8 columns, two coil groups.
constexpr int ADJ_WT = 8, ADJ_G = 2;
template <class Sd, int WT>
hipError_t launch_adj_col(const SenseColArgs& a, int maxW, hipStream_t s) {
  (void)WT;
  SenseColArgs c = a;
  c.tiles = (maxW + ADJ_WT - 1) / ADJ_WT;
  hipLaunchKernelGGL((k_adj_col<Sd, ADJ_WT, ADJ_G>), col_pass_grid(c.tiles, c.nslices), dim3(Sd::T * ADJ_WT * ADJ_G), 0,
                     s, c);
  return hipGetLastError();
}
template <class Sd, int WT>
hipError_t launch_fwd_row(const SenseRowArgs& a, int maxH, int maxC, hipStream_t s) {
  dim3 grid(((maxH + WT - 1) / WT) * maxC, a.nslices);
  hipLaunchKernelGGL((k_fwd_row<Sd, WT>), grid, dim3(Sd::T * WT), 0, s, a);
  return hipGetLastError();
}
template <class Sd, int WT>
hipError_t launch_adj_row(const SenseRowArgs& a, int maxH, int maxC, hipStream_t s) {
  dim3 grid(((maxH + WT - 1) / WT) * maxC, a.nslices);
  hipLaunchKernelGGL((k_adj_row<Sd, WT>), grid, dim3(Sd::T * WT), 0, s, a);
  return hipGetLastError();
}

// Registers one column schedule and one row schedule for a length.
template <class Sd, int WTC, int WTR, int G, bool KS, int KSPL>
struct Registrar {
  Registrar(const char* name) {
    static_assert(KSPL >= 1 && KSPL <= KSPL_MAX, "coil split out of range");
    ColVariant cv{Sd::N, Sd::N1, Sd::N2, Sd::N3, Sd::T, WTC,
                  &launch_normal<Sd, WTC, G, KS, KSPL>, &launch_fwd_col<Sd, WTC>, &launch_adj_col<Sd, WTC>, name,
                  KSPL};
    register_col_variant(cv);
    RowVariant rv{Sd::N, Sd::N1, Sd::N2, Sd::N3, Sd::T, WTR,
                  &launch_fwd_row<Sd, WTR>, &launch_adj_row<Sd, WTR>, name};
    register_row_variant(rv);
  }
};

// Registers a wave-local normal-operator schedule (column passes of the
// forward and adjoint operators use tiles of WTC columns).
template <class Sd, int WTC, int WTR, int G, bool PAD>
struct RegistrarWL {
  RegistrarWL(const char* name) {
    ColVariant cv{Sd::N, Sd::N1, Sd::N2, Sd::N3, Sd::T, 64 / Sd::T,
                  &launch_normal_wl<Sd, G, PAD>, &launch_fwd_col<Sd, WTC>, &launch_adj_col<Sd, WTC>, name};
    register_col_variant(cv);
    RowVariant rv{Sd::N, Sd::N1, Sd::N2, Sd::N3, Sd::T, WTR,
                  &launch_fwd_row<Sd, WTR>, &launch_adj_row<Sd, WTR>, name};
    register_row_variant(rv);
  }
};

}  // namespace mrx
