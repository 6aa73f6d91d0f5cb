// MFMA (bf16 in, fp32 accumulate) 3x3 convolution kernels for the MoDL
// residual denoiser D_W(x) = x + N(x) (MoDL subsection): N = conv(2->64) ReLU
// conv(64->64) ReLU x3, conv(64->2), zero "same" padding, bias.
#pragma once
#include "common.h"

namespace mrx {

constexpr int CNN_F = 64;      // feature channels
constexpr int CNN_L = 5;       // layers
constexpr int CONV_TW = 16;    // output tile width (pixels)
constexpr int CONV_TH = 16;    // output tile height (rows); 4 waves x 4 rows

// Packed bf16 weights of one network (layout chosen for the MFMA operand
// fragments, filled by k_pack_*):
//   first:  [2 ksteps][2 mblk][64 lanes][8]  (K = 9 taps x 2 ch padded to 32)
//   mid:    [9 taps][4 kc][2 mblk][64 lanes][8]
//   last:   [9 taps][2 cc][64 lanes][8]       (16x16x32, co padded to 16)
struct PackedNet {
  const uint16_t* first;
  const uint16_t* mid[3];
  const uint16_t* last;
  const float* bias[5];
};

// Epilogue / input variants
enum ConvMode : int {
  CONV_FWD = 0,     // bias + ReLU (first, mid); bias + residual (last)
  CONV_DGRAD = 1,   // no bias; output multiplied by ReLU'(act) ; last: add residual grad
  // first, mid with batch normalisation (no bias, no ReLU):
  CONV_STATS = 2,   // no output; per-workgroup fp32 sums of y and y^2 per channel into stat_part
  CONV_NORM = 3,    // output (y - mean) * istd per channel (bn_stats), the normalised value
};

struct ConvArgs {
  const SliceDesc* desc;
  const int* slices;
  int nslices;
  int tiles_x;               // max over slices of ceil(W / 16)
  int tiles_y;               // max over slices of ceil(H / 16)
  const uint16_t* in_bf16;   // NHWC bf16, pixel offset xoff * 64
  const float2* in_c;        // complex image (first layer input / last layer residual)
  uint16_t* out_bf16;        // NHWC bf16
  float2* out_c;             // complex output (last layer)
  const uint16_t* wpk;       // packed weights
  const float* bias;         // fp32 bias or null
  const uint16_t* wpk0;      // fused first + second layer: the first layer's packed weights
  const float* bias0;        //   and bias
  const uint16_t* relu_ref;  // dgrad: activation whose ReLU derivative masks the output
  const float2* resid;       // last layer: residual term added to the output
  int mode;
  uint32_t* status;          // per-slice status (non-finite output flag), may be null
  // dgrad of the first (2 -> 64 operator) and middle layers: per-workgroup
  // fp32 sums over pixels of the masked output, [slot][64] with slot =
  // blockIdx.x + tiles_x (blockIdx.y + tiles_y blockIdx.z) (zero for tiles
  // outside their slice) -- the bias gradient of the layer whose ReLU masks
  // the output, before rounding to bf16.  Null: not computed.
  float* bias_part;
  // CONV_STATS: [slot][128] (64 sums of y, then 64 sums of y^2 over the
  // workgroup's pixels inside the image), slot as for bias_part
  float* stat_part;
  // CONV_NORM: per-channel mean [64] then 1 / sqrt(var + eps) [64]
  const float* bn_stats;
};

}  // namespace mrx
