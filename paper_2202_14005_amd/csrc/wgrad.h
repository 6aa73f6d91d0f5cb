// Weight-gradient kernels of the denoiser convolutions (declarations).
#pragma once
#include "common.h"

namespace mrx {

constexpr int WG_ROWS = 4;   // rows per LDS tile
constexpr int WG_BAND = 4;   // rows per workgroup (a band of tiles), first and last layers
constexpr int WGM_WGS = 256; // workgroups (and partial slots) of the middle-layer kernel

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

// kind: 0 = first (2 -> 64), 1 = middle (64 -> 64), 2 = last (64 -> 2)
hipError_t wgrad_launch(int kind, const WgradArgs& a, int bands, hipStream_t s);
// tap_major: the slots hold the 64 x 64 x 9 weight entries as [tap][co][ci]
hipError_t wgrad_reduce(const float* partial, int nslots, int nout, float* w_out, float* b_out, int nweights,
                        int accumulate, int tap_major, hipStream_t s);
// kind: 0 = first, 1 = middle, 2 = last
hipError_t conv_launch(int kind, const struct ConvArgs& a, hipStream_t s);
hipError_t pack_weights(int kind, const float* Wm, uint16_t* out, int transpose, hipStream_t s);

}  // namespace mrx
