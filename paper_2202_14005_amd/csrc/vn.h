// Variational-network stage kernels (declarations and sizes).
#pragma once
#include "common.h"

namespace mrx {

constexpr int VN_NK = 24;               // filters per stage
constexpr int VN_KS = 11;               // filter edge
constexpr int VN_R = VN_KS / 2;
constexpr int VN_TAPS = VN_KS * VN_KS;
constexpr int VN_NW = 31;               // radial basis functions
constexpr int VN_BAND = 3;              // rows per RBF-weight-gradient workgroup (384 rows: 2 per CU)

struct VnArgs {
  const SliceDesc* desc;
  const int* slices;
  int nslices;
  const float2* kt;       // filters, tap-major [121][24] complex
  const float* wa;        // filters as matrix-core operands [121][2][32]: Re k_i, then -Im k_i (i >= 24: 0)
  const float* w;         // RBF weights [24][31]
  const float* wd;        // RBF coefficients per group of 8 knots [24][2][32] (k_vn_pack_rbf)
  const float* lam;       // stage step size (device, 1 float)
  const float2* x;        // stage input
  const float2* g;        // reverse mode: gradient w.r.t. the stage output
  const float2* aHy;
  const float2* q;        // A^H A x (forward) or A^H A g (reverse)
  const float2* qx;       // reverse mode: A^H A x
  float2* out;            // x_next (forward) or g_x (reverse)
  float* u;               // [pixel][24] Phi'(s)
  float* e;               // [pixel][24] Phi''(s) * Kg
  float* kg;              // [pixel][24] Re(k * g)
  float* s;               // [pixel][24] Re(k * x)
  float* part_lam;        // per-tile partials of the lambda gradient
  float* part_k;          // per-band partials of the filter gradient
  float* part_w;          // per-band partials of the RBF-weight gradient
};

}  // namespace mrx
