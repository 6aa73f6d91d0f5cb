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
#include <type_traits>

#include "common.h"

namespace mrx {

template <int I>
using ic = std::integral_constant<int, I>;

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(ic<B>{});
    static_for<B + 1, E>(f);
  }
}

// Input multipliers of the DFT codelets.  A codelet forms m_n * x_n for each
// input; where such a product meets the first addition of a butterfly it is
// folded into fused multiply-adds (see bfly).  Cheap kinds (1, -1, +-i) cost
// no multiplication.
struct MOne {  // 1
  static constexpr bool cheap = true;
  __device__ __forceinline__ float2 mul(float2 x) const { return x; }
};
struct MNeg {  // -1
  static constexpr bool cheap = true;
  __device__ __forceinline__ float2 mul(float2 x) const { return cneg(x); }
};
template <bool POS>
struct MI {  // +i (POS) or -i
  static constexpr bool cheap = true;
  __device__ __forceinline__ float2 mul(float2 x) const { return POS ? cmul_pi(x) : cmul_mi(x); }
};
struct MRe {  // real scale
  static constexpr bool cheap = false;
  float s;
  __device__ __forceinline__ float2 mul(float2 x) const { return cscale(x, s); }
  __device__ __forceinline__ float2 madd(float2 u, float2 z) const {
    return make_float2(__builtin_fmaf(z.x, s, u.x), __builtin_fmaf(z.y, s, u.y));
  }
};
struct MCw {  // complex w
  static constexpr bool cheap = false;
  float2 w;
  __device__ __forceinline__ float2 mul(float2 x) const { return cmul(x, w); }
  __device__ __forceinline__ float2 madd(float2 u, float2 z) const {
    return make_float2(__builtin_fmaf(z.x, w.x, __builtin_fmaf(-z.y, w.y, u.x)),
                       __builtin_fmaf(z.x, w.y, __builtin_fmaf(z.y, w.x, u.y)));
  }
};
struct MCwc {  // conj(w)
  static constexpr bool cheap = false;
  float2 w;
  __device__ __forceinline__ float2 mul(float2 x) const { return cmulc(w, x); }
  __device__ __forceinline__ float2 madd(float2 u, float2 z) const {
    return make_float2(__builtin_fmaf(z.x, w.x, __builtin_fmaf(z.y, w.y, u.x)),
                       __builtin_fmaf(z.y, w.x, __builtin_fmaf(-z.x, w.y, u.y)));
  }
};
struct OneMul {  // every input multiplier 1
  template <class I>
  __device__ __forceinline__ MOne operator()(I) const { return {}; }
};

// s = a x + b z, d = a x - b z.  With one product a fused chain gives s
// (u + b z in four multiply-adds on u = a x) and d = 2u - s takes two more,
// instead of a complex multiply (four) and two complex additions (four).
template <class A, class B>
__device__ __forceinline__ void bfly(float2 x, A a, float2 z, B b, float2& s, float2& d) {
  if constexpr (A::cheap && B::cheap) {
    const float2 u = a.mul(x), y = b.mul(z);
    s = cadd(u, y);
    d = csub(u, y);
  } else if constexpr (!B::cheap) {
    const float2 u = a.mul(x);
    s = b.madd(u, z);
    d = make_float2(__builtin_fmaf(2.f, u.x, -s.x), __builtin_fmaf(2.f, u.y, -s.y));
  } else {
    const float2 y = b.mul(z);
    s = a.madd(y, x);
    d = make_float2(__builtin_fmaf(-2.f, y.x, s.x), __builtin_fmaf(-2.f, y.y, s.y));
  }
}

// Multiplier exp(-/+ 2 pi i E / R) for a compile-time exponent.
template <int R, bool INV, int E>
__device__ __forceinline__ auto twm() {
  constexpr int e = E % R;
  if constexpr (e == 0) {
    return MOne{};
  } else if constexpr (2 * e == R) {
    return MNeg{};
  } else if constexpr (4 * e == R) {
    return MI<INV>{};
  } else if constexpr (4 * e == 3 * R) {
    return MI<!INV>{};
  } else {
    constexpr TwTab<R> tab{};
    return MCw{make_float2(tab.c[e], INV ? tab.s[e] : -tab.s[e])};
  }
}

template <int R>
constexpr int first_factor() {
  return (R % 4 == 0) ? 4 : (R % 2 == 0) ? 2 : (R % 3 == 0) ? 3 : (R % 5 == 0) ? 5 : R;
}

// In-register DFT of length R of the inputs m(n) * v[n], natural order in
// and out: X[k] = sum_n m(n) v[n] exp(-/+ 2 pi i n k / R) (INV: +, unscaled).
// m(ic<n>) gives input n's multiplier.  Composite R = R1 * R2 with
// n = R2 n1 + n2, k = k1 + R1 k2: R2 DFTs of length R1 over n1, then R1 of
// length R2 over n2 whose inputs carry the twiddles exp(-/+ 2 pi i n2 k1 / R).
template <int R, bool INV, class M>
__device__ __forceinline__ void dft_in(float2* v, const M& m) {
  if constexpr (R == 1) {
    v[0] = m(ic<0>{}).mul(v[0]);
  } else if constexpr (R == 2) {
    float2 a, b;
    bfly(v[0], m(ic<0>{}), v[1], m(ic<1>{}), a, b);
    v[0] = a;
    v[1] = b;
  } else if constexpr (R == 3) {
    constexpr float s3 = 0.86602540378443864676f;
    const float2 x0 = m(ic<0>{}).mul(v[0]);
    float2 t1, d;
    bfly(v[1], m(ic<1>{}), v[2], m(ic<2>{}), t1, d);
    const float2 t2 = make_float2(x0.x - 0.5f * t1.x, x0.y - 0.5f * t1.y);
    const float2 t3 = cscale(d, s3);
    v[0] = cadd(x0, t1);
    const float2 it3 = INV ? cmul_pi(t3) : cmul_mi(t3);
    v[1] = cadd(t2, it3);
    v[2] = csub(t2, it3);
  } else if constexpr (R == 4) {
    float2 a, b, c, d;
    bfly(v[0], m(ic<0>{}), v[2], m(ic<2>{}), a, b);
    bfly(v[1], m(ic<1>{}), v[3], m(ic<3>{}), c, d);
    const float2 id = INV ? cmul_pi(d) : cmul_mi(d);
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, id);
    v[3] = csub(b, id);
  } else if constexpr (R == 5) {
    constexpr float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
    constexpr float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
    constexpr float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
    constexpr float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
    const float2 x0 = m(ic<0>{}).mul(v[0]);
    float2 t1, t2, t3, t4;
    bfly(v[1], m(ic<1>{}), v[4], m(ic<4>{}), t1, t3);
    bfly(v[2], m(ic<2>{}), v[3], m(ic<3>{}), t2, t4);
    const float2 a1 = make_float2(x0.x + c1 * t1.x + c2 * t2.x, x0.y + c1 * t1.y + c2 * t2.y);
    const float2 a2 = make_float2(x0.x + c2 * t1.x + c1 * t2.x, x0.y + c2 * t1.y + c1 * t2.y);
    const float2 b1 = make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y);
    const float2 b2 = make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y);
    const float2 ib1 = INV ? cmul_pi(b1) : cmul_mi(b1);
    const float2 ib2 = INV ? cmul_pi(b2) : cmul_mi(b2);
    v[0] = cadd(x0, cadd(t1, t2));
    v[1] = cadd(a1, ib1);
    v[4] = csub(a1, ib1);
    v[2] = cadd(a2, ib2);
    v[3] = csub(a2, ib2);
  } else {
    constexpr int R1 = first_factor<R>();
    constexpr int R2 = R / R1;
    static_assert(R1 > 1 && R1 < R, "length must factor into 2, 3, 4, 5");
    float2 a[R];
    static_for<0, R2>([&](auto n2c) {
      constexpr int n2 = decltype(n2c)::value;
      float2 t[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) t[n1] = v[R2 * n1 + n2];
      dft_in<R1, INV>(t, [&](auto n1c) { return m(ic<R2 * decltype(n1c)::value + n2>{}); });
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) a[k1 * R2 + n2] = t[k1];
    });
    static_for<0, R1>([&](auto k1c) {
      constexpr int k1 = decltype(k1c)::value;
      float2 t[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) t[n2] = a[k1 * R2 + n2];
      dft_in<R2, INV>(t, [](auto n2c) { return twm<R, INV, decltype(n2c)::value * k1>(); });
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = t[k2];
    });
  }
}

// In-register DFT of length R on v[0..R-1], natural order in and out.
template <int R, bool INV>
__device__ __forceinline__ void dft(float2* v) {
  dft_in<R, INV>(v, OneMul{});
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

// Synchronisation between the LDS exchanges of a transform: pre() before a
// thread writes its values of an exchange, sync() between those writes and
// the reads of the next level.  BlockSync: the T threads of a transform span
// several wavefronts.  WaveSync: they all belong to one wavefront, whose LDS
// operations execute in issue order, so only the compiler has to be kept
// from moving LDS accesses across the exchange.  BlockSyncPost: as
// BlockSync without the barrier before the writes, for a tile region that
// sees nothing but alternating transforms (forward, inverse, forward, ...).
// There every exchange writes exactly the LDS slots that the same thread
// read in the exchange before it: the second exchange of a transform those
// of its first, the first exchange of an inverse those of the last exchange
// of the forward before it, and the first exchange of a forward those of the
// last exchange of the inverse before it.  Each slot is read by one thread
// only, so no other thread can still need a slot when it is overwritten.
// (Two inverses in a row do not qualify: the first exchange of the second
// writes other slots than the last exchange of the first read.)
struct BlockSync {
  __device__ static __forceinline__ void pre() { __syncthreads(); }
  __device__ static __forceinline__ void sync() { __syncthreads(); }
};
struct BlockSyncPost {
  __device__ static __forceinline__ void pre() {}
  __device__ static __forceinline__ void sync() { __syncthreads(); }
};
struct WaveSync {
  __device__ static __forceinline__ void sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __device__ static __forceinline__ void pre() { sync(); }
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
  Sync::pre();
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
    Sync::pre();
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

// Scale of the final-level slots for fft_inverse: none, or a real factor
// per frequency read from a table (the sampling mask of the normal
// operator), applied inside the first codelet.
struct NoScale {
  static constexpr bool on = false;
  const float* tab;
};
struct FreqScale {
  static constexpr bool on = true;
  const float* tab;
};

// Exact adjoint of fft_forward (unscaled inverse): final-level layout in,
// level-1 layout out.  With FreqScale the input at frequency k is first
// multiplied by sc.tab[k].
template <class S, class L, class Sync = BlockSync, class Sc = NoScale>
__device__ __forceinline__ void fft_inverse(float2* v, float2* lds, const float2* tw, int tc, int c,
                                            Sc sc = Sc{nullptr}) {
  // first codelet of the final level, with the per-frequency scale folded in
  auto fin = [&](int i) {
    if constexpr (Sc::on) {
      dft_in<S::NFIN, true>(v + i * S::NFIN,
                            [&](auto rc) { return MRe{sc.tab[S::freq(tc, i, decltype(rc)::value)]}; });
    } else {
      dft<S::NFIN, true>(v + i * S::NFIN);
    }
  };
  if constexpr (S::LEVELS == 3) {
#pragma unroll
    for (int i = 0; i < S::G3; ++i) fin(i);
    Sync::pre();
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
      float2 w[S::N2];
#pragma unroll
      for (int r = 1; r < S::N2; ++r) w[r] = tw[S::N1 * r * n3];
      dft_in<S::N2, true>(v + i * S::N2, [&](auto rc) {
        constexpr int r = decltype(rc)::value;
        if constexpr (r == 0) return MOne{};
        else return MCwc{w[r]};
      });
    }
  } else {
#pragma unroll
    for (int i = 0; i < S::G2; ++i) fin(i);
  }
  Sync::pre();
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
    float2 w[S::N1];
#pragma unroll
    for (int r = 1; r < S::N1; ++r) w[r] = tw[g * r];
    dft_in<S::N1, true>(v + i * S::N1, [&](auto rc) {
      constexpr int r = decltype(rc)::value;
      if constexpr (r == 0) return MOne{};
      else return MCwc{w[r]};
    });
  }
}

}  // namespace mrx
