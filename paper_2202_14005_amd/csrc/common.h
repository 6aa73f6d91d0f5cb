// Shared device/host definitions for the mrx HIP library (gfx950 / CDNA4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrx {

// Per-slice geometry of a (possibly uneven) batch.  Offsets are in elements
// of the respective packed buffer: image-sized buffers (x, p, q, ...) use
// xoff, coil-sized buffers (S, y) use soff, masks use moff.
struct SliceDesc {
  int32_t H, W, C;
  int32_t nq;  // partial planes of the normal operator's output in CG mode (coil split)
  int64_t xoff, soff, moff;
};

// ---------------------------------------------------------------- complex
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// multiply by -i and +i
__device__ __forceinline__ float2 cmul_mi(float2 a) { return make_float2(a.y, -a.x); }
__device__ __forceinline__ float2 cmul_pi(float2 a) { return make_float2(-a.y, a.x); }
__device__ __forceinline__ float2 cneg(float2 a) { return make_float2(-a.x, -a.y); }

// ------------------------------------------------- compile-time trigonometry
// Taylor series evaluated by the compiler in double precision (|x| <= pi),
// rounded once to float; used for the constant twiddles inside the
// in-register DFT codelets.
constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double cx_sin(double x) {
  double t = x, s = x, x2 = x * x;
  for (int n = 1; n < 16; ++n) { t *= -x2 / ((2.0 * n) * (2.0 * n + 1)); s += t; }
  return s;
}
constexpr double cx_cos(double x) {
  double t = 1, s = 1, x2 = x * x;
  for (int n = 1; n < 16; ++n) { t *= -x2 / ((2.0 * n - 1) * (2.0 * n)); s += t; }
  return s;
}
template <int R>
struct TwTab {
  float c[R];
  float s[R];
  constexpr TwTab() : c(), s() {
    for (int i = 0; i < R; ++i) {
      double a = 2 * kPi * i / R;
      if (a > kPi) a -= 2 * kPi;
      c[i] = (float)cx_cos(a);
      s[i] = (float)cx_sin(a);
    }
  }
};

}  // namespace mrx
