// Batch normalisation of the denoiser's hidden layers (declarations; see
// bn.hip).  Activations are NHWC bf16 with 64 channels, npix pixels.
#pragma once
#include "common.h"
#include "conv.h"

namespace mrx {

constexpr int BN_BLOCKS = 512;   // workgroups (and partial slots) of a statistics pass
constexpr float BN_EPS = 1e-5f;
// per-layer statistics block (floats): mean, 1 / sqrt(var + eps) (the
// layout CONV_NORM reads), and the reverse pass's sums of g_z and g_z yhat
constexpr int BN_MEAN = 0, BN_ISTD = 64, BN_SGZ = 128, BN_SGY = 192;
constexpr int BN_STATS = 256;

// stats[BN_MEAN], stats[BN_ISTD] from nslots convolution slots of 128 floats
// (sums of y, then of y^2, ConvArgs::stat_part).
hipError_t bn_finish_stats(const float* slots, int nslots, int64_t npix, float* stats, hipStream_t s);
// a = ReLU(gamma yhat + beta), rounded to bf16.
hipError_t bn_apply_forward(const uint16_t* yhat, uint16_t* a, int64_t npix, const float* gamma, const float* beta,
                            const float* stats, hipStream_t s);
// In place g_z -> g_y with the forward's stats and yhat; sgz[64] = sum g_z
// (the input-gradient convolution's fp32 channel sums); part: BN_BLOCKS x
// 64 floats; g_gamma, g_beta (+)= (may be null).
hipError_t bn_backward(const uint16_t* yhat, uint16_t* g, int64_t npix, const float* gamma, float* stats,
                       const float* sgz, float* part, float* g_gamma, float* g_beta, int accumulate,
                       hipStream_t s);

}  // namespace mrx
