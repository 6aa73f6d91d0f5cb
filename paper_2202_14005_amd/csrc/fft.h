// Mixed-radix (2/3/4/5) FFT engine for gfx950: in-register DFT codelets and a
// multi-level decomposition whose levels are exchanged through LDS.
//
// A length-N transform (N = N1 * N2 * N3) is computed "in digit space": the
// element whose input index is n = n1*M1 + n2*M2 + n3 (M1 = N2*N3, M2 = N3)
// keeps its LDS address while each level replaces one input digit n_j by an
// output digit k_j.  Level 1 is a DFT over n1 followed by the twiddle
// W_N^{k1 (n2 N3 + n3)}, level 2 a DFT over n2 followed by W_N^{N1 k2 n3},
// level 3 a DFT over n3.  The output X[k1 + N1 k2 + N1 N2 k3] ends at the
// address k1*M1 + k2*M2 + k3 (digit reversed), which is never reordered:
// the normal operator multiplies by the mask there and runs the exact adjoint
// sequence back, so every thread ends holding the same points it started
// with.  T threads cooperate on one transform; at level j each thread owns
// (N / N_j) / T complete sub-transforms of length N_j held in registers.
#pragma once
#include "common.h"

namespace mrx {

// x * exp(-/+ 2 pi i e / R); e is a compile-time constant after unrolling.
template <int R, bool INV>
__device__ __forceinline__ float2 twc(float2 x, int e) {
  e %= R;
  if (e == 0) return x;
  if (2 * e == R) return cneg(x);
  if (4 * e == R) return INV ? cmul_pi(x) : cmul_mi(x);
  if (4 * e == 3 * R) return INV ? cmul_mi(x) : cmul_pi(x);
  static constexpr TwTab<R> tab{};
  const float c = tab.c[e], s = tab.s[e];
  return cmul(x, make_float2(c, INV ? s : -s));
}

template <int R>
constexpr int first_factor() {
  return (R % 4 == 0) ? 4 : (R % 2 == 0) ? 2 : (R % 3 == 0) ? 3 : (R % 5 == 0) ? 5 : R;
}

// In-register DFT of length R on v[0..R-1], natural order in and out.
// Forward: X[k] = sum_n x[n] exp(-2 pi i n k / R); INV: exp(+...), unscaled.
template <int R, bool INV>
__device__ __forceinline__ void dft(float2* v) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 3) {
    constexpr float s3 = 0.86602540378443864676f;
    float2 t1 = cadd(v[1], v[2]);
    float2 t2 = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
    float2 t3 = cscale(csub(v[1], v[2]), s3);
    v[0] = cadd(v[0], t1);
    float2 it3 = INV ? cmul_pi(t3) : cmul_mi(t3);
    v[1] = cadd(t2, it3);
    v[2] = csub(t2, it3);
  } else if constexpr (R == 4) {
    float2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    float2 c = cadd(v[1], v[3]), d = csub(v[1], v[3]);
    float2 id = INV ? cmul_pi(d) : cmul_mi(d);
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, id);
    v[3] = csub(b, id);
  } else if constexpr (R == 5) {
    constexpr float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
    constexpr float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
    constexpr float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
    constexpr float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
    float2 x0 = v[0];
    float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    float2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    float2 a1 = make_float2(x0.x + c1 * t1.x + c2 * t2.x, x0.y + c1 * t1.y + c2 * t2.y);
    float2 a2 = make_float2(x0.x + c2 * t1.x + c1 * t2.x, x0.y + c2 * t1.y + c1 * t2.y);
    float2 b1 = make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y);
    float2 b2 = make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y);
    float2 ib1 = INV ? cmul_pi(b1) : cmul_mi(b1);
    float2 ib2 = INV ? cmul_pi(b2) : cmul_mi(b2);
    v[0] = cadd(x0, cadd(t1, t2));
    v[1] = cadd(a1, ib1);
    v[4] = csub(a1, ib1);
    v[2] = cadd(a2, ib2);
    v[3] = csub(a2, ib2);
  } else {
    // R = R1 * R2 with n = R2 n1 + n2, k = k1 + R1 k2.
    constexpr int R1 = first_factor<R>();
    constexpr int R2 = R / R1;
    static_assert(R1 > 1 && R1 < R, "length must factor into 2, 3, 4, 5");
    float2 a[R];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
      float2 t[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) t[n1] = v[R2 * n1 + n2];
      dft<R1, INV>(t);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) a[k1 * R2 + n2] = twc<R, INV>(t[k1], n2 * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      float2 t[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) t[n2] = a[k1 * R2 + n2];
      dft<R2, INV>(t);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = t[k2];
    }
  }
}

// Static description of one decomposition N = N1 * N2 * N3 over T threads.
template <int N1_, int N2_, int N3_, int T_>
struct Sched {
  static constexpr int N1 = N1_, N2 = N2_, N3 = N3_, T = T_;
  static constexpr int N = N1 * N2 * N3;
  static constexpr int P = N / T;  // points per thread
  static constexpr int M1 = N2 * N3, M2 = N3;
  static constexpr int G1 = N / N1 / T, G2 = N / N2 / T, G3 = N / N3 / T;
  static constexpr int LEVELS = (N3 > 1) ? 3 : 2;
  static_assert((N / N1) % T == 0 && (N / N2) % T == 0 && (N / N3) % T == 0,
                "threads per transform must divide every level's transform count");
  // Address of register slot (group i, digit r) at each level.
  __device__ static __forceinline__ int a1(int tc, int i, int r) { return (tc + T * i) + r * M1; }
  __device__ static __forceinline__ int a2(int tc, int i, int r) {
    int q = tc + T * i;
    return (q / N3) * M1 + r * M2 + (q % N3);
  }
  __device__ static __forceinline__ int a3(int tc, int i, int r) {
    int q = tc + T * i;
    return (q / N2) * M1 + (q % N2) * M2 + r;
  }
  // Frequency held in the final-level slot (group i, digit r).
  __device__ static __forceinline__ int freq(int tc, int i, int r) {
    if constexpr (LEVELS == 3) {
      int q = tc + T * i;
      return (q / N2) + N1 * (q % N2) + N1 * N2 * r;
    } else {
      return (tc + T * i) + N1 * r;
    }
  }
  // Final-level address (for storing the transform in digit order).
  __device__ static __forceinline__ int afin(int tc, int i, int r) {
    if constexpr (LEVELS == 3) return a3(tc, i, r);
    else return a2(tc, i, r);
  }
  static constexpr int GFIN = (LEVELS == 3) ? G3 : G2;
  static constexpr int NFIN = (LEVELS == 3) ? N3 : N2;
};

// Synchronisation between the LDS exchanges of a transform.  BlockSync: the T
// threads of a transform span several wavefronts.  WaveSync: they all belong
// to one wavefront, whose LDS operations execute in issue order, so only the
// compiler has to be kept from moving LDS accesses across the exchange.
struct BlockSync {
  __device__ static __forceinline__ void sync() { __syncthreads(); }
};
struct WaveSync {
  __device__ static __forceinline__ void sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
};

// LDS layouts: element (address a, transform c) of a tile of WT transforms.
// Column tiles keep the WT transforms interleaved (a * WT + c) so that a row
// of the image maps to contiguous LDS; row tiles keep each transform
// contiguous with one pad slot per transform.
template <int N, int WT>
struct LdsInterleaved {
  static constexpr int SIZE = N * WT;
  __device__ static __forceinline__ int idx(int a, int c) { return a * WT + c; }
};
// Interleaved with CW = WT transforms and one pad row of WT slots after
// every SEG addresses: for WT = 4 and SEG = N3 the reads of the last level
// (addresses N3 apart across threads) fall in distinct bank groups.
template <int N, int WT, int SEG>
struct LdsPadded {
  static constexpr int SIZE = (N + N / SEG) * WT;
  __device__ static __forceinline__ int idx(int a, int c) { return (a + a / SEG) * WT + c; }
};
template <int N, int WT>
struct LdsContig {
  static constexpr int SIZE = (N + 1) * WT;
  __device__ static __forceinline__ int idx(int a, int c) { return c * (N + 1) + a; }
};

// Forward transform of the thread's P points (level-1 layout in, final-level
// layout out).  tw = table of exp(-2 pi i j / N), j < N, in LDS.
template <class S, class L, class Sync = BlockSync>
__device__ __forceinline__ void fft_forward(float2* v, float2* lds, const float2* tw, int tc, int c) {
  // level 1
#pragma unroll
  for (int i = 0; i < S::G1; ++i) {
    dft<S::N1, false>(v + i * S::N1);
    const int g = tc + S::T * i;
#pragma unroll
    for (int r = 1; r < S::N1; ++r) v[i * S::N1 + r] = cmul(v[i * S::N1 + r], tw[g * r]);
  }
  Sync::sync();
#pragma unroll
  for (int i = 0; i < S::G1; ++i)
#pragma unroll
    for (int r = 0; r < S::N1; ++r) lds[L::idx(S::a1(tc, i, r), c)] = v[i * S::N1 + r];
  Sync::sync();
#pragma unroll
  for (int i = 0; i < S::G2; ++i)
#pragma unroll
    for (int r = 0; r < S::N2; ++r) v[i * S::N2 + r] = lds[L::idx(S::a2(tc, i, r), c)];
  // level 2
#pragma unroll
  for (int i = 0; i < S::G2; ++i) {
    dft<S::N2, false>(v + i * S::N2);
    if constexpr (S::LEVELS == 3) {
      const int n3 = (tc + S::T * i) % S::N3;
#pragma unroll
      for (int r = 1; r < S::N2; ++r) v[i * S::N2 + r] = cmul(v[i * S::N2 + r], tw[S::N1 * r * n3]);
    }
  }
  if constexpr (S::LEVELS == 3) {
    Sync::sync();
#pragma unroll
    for (int i = 0; i < S::G2; ++i)
#pragma unroll
      for (int r = 0; r < S::N2; ++r) lds[L::idx(S::a2(tc, i, r), c)] = v[i * S::N2 + r];
    Sync::sync();
#pragma unroll
    for (int i = 0; i < S::G3; ++i)
#pragma unroll
      for (int r = 0; r < S::N3; ++r) v[i * S::N3 + r] = lds[L::idx(S::a3(tc, i, r), c)];
#pragma unroll
    for (int i = 0; i < S::G3; ++i) dft<S::N3, false>(v + i * S::N3);
  }
}

// Exact adjoint of fft_forward (unscaled inverse): final-level layout in,
// level-1 layout out.
template <class S, class L, class Sync = BlockSync>
__device__ __forceinline__ void fft_inverse(float2* v, float2* lds, const float2* tw, int tc, int c) {
  if constexpr (S::LEVELS == 3) {
#pragma unroll
    for (int i = 0; i < S::G3; ++i) dft<S::N3, true>(v + i * S::N3);
    Sync::sync();
#pragma unroll
    for (int i = 0; i < S::G3; ++i)
#pragma unroll
      for (int r = 0; r < S::N3; ++r) lds[L::idx(S::a3(tc, i, r), c)] = v[i * S::N3 + r];
    Sync::sync();
#pragma unroll
    for (int i = 0; i < S::G2; ++i)
#pragma unroll
      for (int r = 0; r < S::N2; ++r) v[i * S::N2 + r] = lds[L::idx(S::a2(tc, i, r), c)];
#pragma unroll
    for (int i = 0; i < S::G2; ++i) {
      const int n3 = (tc + S::T * i) % S::N3;
#pragma unroll
      for (int r = 1; r < S::N2; ++r) v[i * S::N2 + r] = cmulc(tw[S::N1 * r * n3], v[i * S::N2 + r]);
    }
  }
#pragma unroll
  for (int i = 0; i < S::G2; ++i) dft<S::N2, true>(v + i * S::N2);
  Sync::sync();
#pragma unroll
  for (int i = 0; i < S::G2; ++i)
#pragma unroll
    for (int r = 0; r < S::N2; ++r) lds[L::idx(S::a2(tc, i, r), c)] = v[i * S::N2 + r];
  Sync::sync();
#pragma unroll
  for (int i = 0; i < S::G1; ++i)
#pragma unroll
    for (int r = 0; r < S::N1; ++r) v[i * S::N1 + r] = lds[L::idx(S::a1(tc, i, r), c)];
#pragma unroll
  for (int i = 0; i < S::G1; ++i) {
    const int g = tc + S::T * i;
#pragma unroll
    for (int r = 1; r < S::N1; ++r) v[i * S::N1 + r] = cmulc(tw[g * r], v[i * S::N1 + r]);
    dft<S::N1, true>(v + i * S::N1);
  }
}

}  // namespace mrx
