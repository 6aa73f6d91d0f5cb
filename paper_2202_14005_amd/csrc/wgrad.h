// Weight-gradient kernels of the denoiser convolutions (declarations).
#pragma once
#include "common.h"

namespace mrx {

constexpr int WG_ROWS = 4;   // rows per tile (tiles are WG_ROWS x 32 pixels)
constexpr int WGM_WGS = 256;   // workgroups (and partial slots) of the 64 -> 64 weight gradient
constexpr int WGS_WGS = 1024;  // the same for the 2 -> 64 and 64 -> 2 layers (small slots)
constexpr int wgrad_slots(int kind) { return kind == 1 ? WGM_WGS : WGS_WGS; }

// partial-slot layouts of the three kinds (weights; the last layer also its
// two biases)
constexpr int WG_LAYOUT_FIRST = 0, WG_LAYOUT_MID = 1, WG_LAYOUT_LAST = 2;
// floats per partial slot: kind 0 = first (2 -> 64), 1 = middle, 2 = last (64 -> 2)
constexpr int wgrad_nout(int kind) { return kind == 1 ? 64 * 64 * 9 : kind == 0 ? 64 * 32 : 18 * 64 + 2; }

struct WgradArgs {
  const SliceDesc* desc;
  const int* slices;
  int nslices;
  const uint16_t* g;     // gradient w.r.t. the layer's pre-activation (NHWC bf16, 64 ch)
  const uint16_t* act;   // layer input activation (NHWC bf16, 64 ch)
  const float2* x;       // first layer: complex input; last layer: complex output gradient
  float* partial;        // [slots][nout]
  int nout;
};

// kind: 0 = first (2 -> 64), 1 = middle (64 -> 64), 2 = last (64 -> 2); a.partial
// holds wgrad_slots(kind) slots of wgrad_nout(kind) floats
hipError_t wgrad_launch(int kind, const WgradArgs& a, hipStream_t s);
// sums the slots of wgrad_launch into the [co][ci][tap] weight gradient (and,
// for the last layer, its bias gradient b_out)
hipError_t wgrad_reduce(int kind, const float* partial, float* w_out, float* b_out, int accumulate, hipStream_t s);
// b_out[64] (+)= sum over nslots slots of 64 floats (the per-workgroup bias
// sums of an input-gradient convolution, ConvArgs::bias_part), fixed order
hipError_t bias_reduce(const float* partial, int nslots, float* b_out, int accumulate, hipStream_t s);
// kind: 0 = first, 1 = middle, 2 = last
hipError_t conv_launch(int kind, const struct ConvArgs& a, hipStream_t s);
hipError_t pack_weights(int kind, const float* Wm, uint16_t* out, int transpose, hipStream_t s);

}  // namespace mrx
