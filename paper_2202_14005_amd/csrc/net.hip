// Network entry points: the MoDL residual denoiser (forward, reverse mode),
// the MoDL unrolled network (eq. update_modl) with its reverse pass by adjoint
// CG and recomputed unroll activations, the MSE loss gradient and Adam.
#include <algorithm>
#include "../../include/mrx.h"
#include "api_internal.h"
#include "bn.h"
#include "conv.h"
#include "wgrad.h"

namespace mrx {

static size_t al(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int PK_FIRST = 2 * 2 * 64 * 8;
constexpr int PK_MID = 9 * 4 * 2 * 64 * 8;
constexpr int PK_LAST = 9 * 2 * 64 * 8;

size_t net_workspace_bytes(mrx_plan_s* p);

// Network workspace layout, appended after the SENSE/CG part (flags bit 0).
size_t extra_workspace_bytes(mrx_plan_s* p) {
  size_t w = 0;
  if (p->flags & MRX_PLAN_NETWORK) w = net_workspace_bytes(p);
  return w + vn_workspace_bytes(p, p->ws_bytes_base + w);
}

size_t net_workspace_bytes(mrx_plan_s* p) {
  const size_t ni = (size_t)p->n_image;
  size_t w = 0;
  auto take = [&](size_t bytes) { size_t o = p->ws_bytes_base + w; w += al(bytes); return o; };
  for (int i = 0; i < 4; ++i) p->ws_act[i] = take(ni * CNN_F * 2);
  for (int i = 0; i < 2; ++i) p->ws_gact[i] = take(ni * CNN_F * 2);
  const size_t ns = ni * (size_t)p->sets;  // network images of soft-SENSE plans hold every set
  p->ws_z = take(ns * 8);
  for (int i = 0; i < 2; ++i) p->ws_ximg[i] = take(ns * 8);
  for (int i = 0; i < 2; ++i) p->ws_gimg[i] = take(ns * 8);
  p->ws_vimg = take(ns * 8);
  if (p->sets > 1)
    for (int i = 0; i < 3; ++i) p->ws_s1[i] = take(ni * 8);
  p->ws_pk = take((size_t)2 * (PK_FIRST + 3 * PK_MID + PK_LAST) * 2);
  size_t wpart = 0;
  for (int k = 0; k < 3; ++k) wpart = std::max(wpart, (size_t)wgrad_slots(k) * wgrad_nout(k));
  p->ws_wpart = take(wpart * 4);
  // per-workgroup bias sums of the input-gradient convolutions (one slot of
  // 64 floats per 16 x 16 tile of the launch grid)
  p->ws_bpart = take((size_t)((p->maxW + CONV_TW - 1) / CONV_TW) * ((p->maxH + CONV_TH - 1) / CONV_TH) * p->B *
                     CNN_F * 4);
  p->ws_loss = take((size_t)p->B * p->nrr * 4);
  if (p->flags & MRX_PLAN_BATCHNORM) {
    // the hidden layers' normalised outputs, their statistics, the reverse
    // pass's partial and channel sums, the convolutions' statistics slots
    for (int i = 0; i < 4; ++i) p->ws_bnpre[i] = take(ni * CNN_F * 2);
    p->ws_bnstats = take((size_t)4 * BN_STATS * 4);
    p->ws_bnpart = take((size_t)BN_BLOCKS * CNN_F * 4);
    p->ws_bnslots = take((size_t)((p->maxW + CONV_TW - 1) / CONV_TW) * ((p->maxH + CONV_TH - 1) / CONV_TH) * p->B *
                         2 * CNN_F * 4);
    p->ws_bnsgz = take((size_t)CNN_F * 4);
  }
  return w;
}

// Packed weights: the forward set [first | mid x3 | last] followed by the
// dgrad set, whose first-layer operator is last-shaped and whose last-layer
// operator is first-shaped: [last-shaped | mid x3 | first-shaped].
static uint16_t* pk_ptr(mrx_plan_s* p, int transpose, int layer) {
  uint16_t* base = (uint16_t*)(p->ws + p->ws_pk);
  if (!transpose) {
    if (layer == 0) return base;
    if (layer <= 3) return base + PK_FIRST + (layer - 1) * PK_MID;
    return base + PK_FIRST + 3 * PK_MID;
  }
  base += PK_FIRST + 3 * PK_MID + PK_LAST;
  if (layer == 0) return base;
  if (layer <= 3) return base + PK_LAST + (layer - 1) * PK_MID;
  return base + PK_LAST + 3 * PK_MID;
}

static ConvArgs conv_args(mrx_plan_s* p) {
  ConvArgs a{};
  a.desc = p->d_desc;
  a.slices = p->d_all;
  a.nslices = p->B;
  a.tiles_x = (p->maxW + CONV_TW - 1) / CONV_TW;
  a.tiles_y = (p->maxH + CONV_TH - 1) / CONV_TH;
  a.status = (uint32_t*)(p->ws + p->ws_status);
  return a;
}

static mrx_status net_ready(mrx_plan_s* p, const char* who) {
  if (!p->ws) return fail(MRX_ENOWORKSPACE, std::string(who) + ": workspace not set");
  if (!(p->flags & MRX_PLAN_NETWORK))
    return fail(MRX_ENOWORKSPACE, std::string(who) + ": plan was created without MRX_PLAN_NETWORK");
  if (!p->net_ready) return fail(MRX_EINVAL, std::string(who) + ": call mrx_cnn_set_weights first");
  if ((p->flags & MRX_PLAN_BATCHNORM) && !p->bn_gamma)
    return fail(MRX_EINVAL, std::string(who) + ": call mrx_cnn_set_bn first (batch-normalisation plan)");
  return MRX_OK;
}

static float* bn_stats(mrx_plan_s* p, int layer) { return (float*)(p->ws + p->ws_bnstats) + layer * BN_STATS; }

// Forward with batch normalisation after each hidden layer (statistics of
// the batch; the first two layers are not fused, as the second needs the
// first's statistics).  Each hidden convolution runs twice: summing y and
// y^2 per channel, then writing the normalised yhat (kept for the reverse
// pass), from which a = ReLU(gamma yhat + beta).  No hidden bias.
static mrx_status cnn_fwd_bn(mrx_plan_s* p, const float2* x, float2* z, hipStream_t s) {
  uint16_t* act[4];
  uint16_t* pre[4];
  for (int i = 0; i < 4; ++i) {
    act[i] = (uint16_t*)(p->ws + p->ws_act[i]);
    pre[i] = (uint16_t*)(p->ws + p->ws_bnpre[i]);
  }
  float* slots = (float*)(p->ws + p->ws_bnslots);
  const int nslots = ((p->maxW + CONV_TW - 1) / CONV_TW) * ((p->maxH + CONV_TH - 1) / CONV_TH) * p->B;
  hipError_t e = hipSuccess;
  for (int l = 0; l <= 3 && e == hipSuccess; ++l) {
    const int kind = l == 0 ? 0 : 1;
    ConvArgs m = conv_args(p);
    if (l == 0) m.in_c = x;
    else m.in_bf16 = act[l - 1];
    m.wpk = pk_ptr(p, 0, l);
    m.mode = CONV_STATS;
    m.stat_part = slots;
    e = conv_launch(kind, m, s);
    if (e == hipSuccess) e = bn_finish_stats(slots, nslots, p->n_image, bn_stats(p, l), s);
    if (e == hipSuccess) {
      m.mode = CONV_NORM;
      m.bn_stats = bn_stats(p, l);
      m.out_bf16 = pre[l];
      KernelTimer kt(p, kind == 1 ? MRX_KERNEL_CONV_MID : -1, s);
      e = conv_launch(kind, m, s);
    }
    if (e == hipSuccess)
      e = bn_apply_forward(pre[l], act[l], p->n_image, p->bn_gamma + l * CNN_F, p->bn_beta + l * CNN_F,
                           bn_stats(p, l), s);
  }
  if (e == hipSuccess) {
    ConvArgs f = conv_args(p);
    f.mode = CONV_FWD;
    f.in_bf16 = act[3];
    f.out_c = z;
    f.resid = x;
    f.wpk = pk_ptr(p, 0, 4);
    f.bias = p->net_b[4];
    e = conv_launch(2, f, s);
  }
  return e == hipSuccess ? MRX_OK : hip_fail(e, "cnn_forward (batch normalisation)");
}

static mrx_status cnn_fwd(mrx_plan_s* p, const float2* x, float2* z, hipStream_t s, bool fuse12 = false) {
  if (p->flags & MRX_PLAN_BATCHNORM) return cnn_fwd_bn(p, x, z, s);
  uint16_t* act[4];
  for (int i = 0; i < 4; ++i) act[i] = (uint16_t*)(p->ws + p->ws_act[i]);
  ConvArgs a = conv_args(p);
  a.mode = CONV_FWD;
  a.in_c = x;
  hipError_t e;
  if (fuse12) {
    a.out_bf16 = act[1];
    a.wpk0 = pk_ptr(p, 0, 0);
    a.bias0 = p->net_b[0];
    a.wpk = pk_ptr(p, 0, 1);
    a.bias = p->net_b[1];
    e = conv_launch(3, a, s);
  } else {
    a.out_bf16 = act[0];
    a.wpk = pk_ptr(p, 0, 0);
    a.bias = p->net_b[0];
    e = conv_launch(0, a, s);
  }
  for (int l = fuse12 ? 2 : 1; l <= 3 && e == hipSuccess; ++l) {
    ConvArgs m = conv_args(p);
    m.mode = CONV_FWD;
    m.in_bf16 = act[l - 1];
    m.out_bf16 = act[l];
    m.wpk = pk_ptr(p, 0, l);
    m.bias = p->net_b[l];
    KernelTimer kt(p, MRX_KERNEL_CONV_MID, s);
    e = conv_launch(1, m, s);
  }
  if (e == hipSuccess) {
    ConvArgs f = conv_args(p);
    f.mode = CONV_FWD;
    f.in_bf16 = act[3];
    f.out_c = z;
    f.resid = x;
    f.wpk = pk_ptr(p, 0, 4);
    f.bias = p->net_b[4];
    e = conv_launch(2, f, s);
  }
  return e == hipSuccess ? MRX_OK : hip_fail(e, "cnn_forward");
}

// Reverse mode of D at x (activations of cnn_fwd(x) must be in the workspace):
// gx = gz + J_N(x)^T gz; weight/bias gradients into g (accumulate or set).
static mrx_status cnn_bwd(mrx_plan_s* p, const float2* x, const float2* gz, float2* gx, const mrx_cnn_grads* g,
                          int accumulate, hipStream_t s) {
  uint16_t* act[4];
  for (int i = 0; i < 4; ++i) act[i] = (uint16_t*)(p->ws + p->ws_act[i]);
  uint16_t* gb[2] = {(uint16_t*)(p->ws + p->ws_gact[0]), (uint16_t*)(p->ws + p->ws_gact[1])};
  float* part = (float*)(p->ws + p->ws_wpart);
  hipError_t e;
  auto wg = [&](int kind, const uint16_t* gin, const uint16_t* ain, const float2* xin, int layer) {
    WgradArgs w{};
    w.desc = p->d_desc;
    w.slices = p->d_all;
    w.nslices = p->B;
    w.g = gin;
    w.act = ain;
    w.x = xin;
    w.partial = part;
    w.nout = wgrad_nout(kind);
    hipError_t r;
    {
      KernelTimer kt(p, kind == 1 ? MRX_KERNEL_WGRAD_MID : -1, s);
      r = wgrad_launch(kind, w, s);
    }
    if (r != hipSuccess) return r;
    return wgrad_reduce(kind, part, g->w[layer], g->b[layer], accumulate, s);
  };
  float* bpart = (float*)(p->ws + p->ws_bpart);
  const int nbslots = ((p->maxW + CONV_TW - 1) / CONV_TW) * ((p->maxH + CONV_TH - 1) / CONV_TH) * p->B;
  // The fp32 channel sums of the gradient after hidden layer l's ReLU
  // derivative (gbuf holds that gradient, bf16): the bias gradient of layer
  // l, or, with batch normalisation, g_beta, after which gbuf is turned into
  // the gradient before the normalisation (the hidden layers then have no
  // bias: their bias gradient is zero).
  const bool bn = (p->flags & MRX_PLAN_BATCHNORM) != 0;
  auto hidden = [&](int l, uint16_t* gbuf) -> hipError_t {
    if (!bn) return bias_reduce(bpart, nbslots, g->b[l], accumulate, s);
    float* sgz = (float*)(p->ws + p->ws_bnsgz);
    hipError_t r = bias_reduce(bpart, nbslots, sgz, 0, s);
    if (r != hipSuccess) return r;
    return bn_backward((const uint16_t*)(p->ws + p->ws_bnpre[l]), gbuf, p->n_image, p->bn_gamma + l * CNN_F,
                       bn_stats(p, l), sgz, (float*)(p->ws + p->ws_bnpart),
                       p->bn_ggamma ? p->bn_ggamma + l * CNN_F : nullptr,
                       p->bn_gbeta ? p->bn_gbeta + l * CNN_F : nullptr, accumulate, s);
  };
  if (bn && !accumulate)
    for (int l = 0; l < 4; ++l) {
      e = fill_u32((uint32_t*)g->b[l], 0u, CNN_F, s);
      if (e != hipSuccess) return hip_fail(e, "cnn_backward: clear");
    }
  // layer 5 (64 -> 2); its input gradient masked by layer 4's ReLU is layer
  // 4's pre-activation gradient, whose fp32 sums give layer 4's bias gradient
  e = wg(2, nullptr, act[3], gz, 4);
  if (e == hipSuccess) {
    ConvArgs a = conv_args(p);
    a.mode = CONV_DGRAD;
    a.in_c = gz;
    a.out_bf16 = gb[0];
    a.wpk = pk_ptr(p, 1, 4);
    a.relu_ref = act[3];
    a.bias_part = bpart;
    e = conv_launch(0, a, s);
  }
  if (e == hipSuccess) e = hidden(3, gb[0]);
  // layers 4, 3, 2 (64 -> 64)
  int cur = 0;
  for (int l = 3; l >= 1 && e == hipSuccess; --l) {
    e = wg(1, gb[cur], act[l - 1], nullptr, l);
    if (e != hipSuccess) break;
    ConvArgs m = conv_args(p);
    m.mode = CONV_DGRAD;
    m.in_bf16 = gb[cur];
    m.out_bf16 = gb[1 - cur];
    m.wpk = pk_ptr(p, 1, l);
    m.relu_ref = act[l - 1];
    m.bias_part = bpart;
    {
      KernelTimer kt(p, MRX_KERNEL_CONV_MID, s);
      e = conv_launch(1, m, s);
    }
    if (e == hipSuccess) e = hidden(l - 1, gb[1 - cur]);
    cur = 1 - cur;
  }
  // layer 1 (2 -> 64) and the residual
  if (e == hipSuccess) e = wg(0, gb[cur], nullptr, x, 0);
  if (e == hipSuccess) {
    ConvArgs f = conv_args(p);
    f.mode = CONV_DGRAD;
    f.in_bf16 = gb[cur];
    f.out_c = gx;
    f.resid = gz;
    f.wpk = pk_ptr(p, 1, 0);
    e = conv_launch(2, f, s);
  }
  return e == hipSuccess ? MRX_OK : hip_fail(e, "cnn_backward");
}

// ------------------------------------------------------ elementwise helpers
__global__ void k_copy_c(const float2* src, float2* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}
__global__ void k_axpy_c(const float2* src, float2* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) { float2 a = dst[i], b = src[i]; dst[i] = make_float2(a.x + b.x, a.y + b.y); }
}
static hipError_t copy_c(const float2* src, float2* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_c, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}
static hipError_t axpy_c(const float2* src, float2* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_c, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

// g = 2 (x - ref) / n_total; per-slice-block partial sums of |x - ref|^2.
__global__ void __launch_bounds__(256) k_mse(const SliceDesc* desc, const int* slices, const float2* x,
                                             const float2* ref, float2* g, float* part, int nrr, float scale) {
  __shared__ float red[4];
  const int b = slices[blockIdx.y];
  const SliceDesc d = desc[b];
  const int64_t n = (int64_t)d.H * d.W;
  float acc = 0.f;
  const int64_t base = (int64_t)blockIdx.x * CG_EPB;
  for (int k = threadIdx.x; k < CG_EPB; k += 256) {
    const int64_t i = base + k;
    if (i >= n) break;
    const float2 a = x[d.xoff + i], r = ref[d.xoff + i];
    const float dx = a.x - r.x, dy = a.y - r.y;
    acc += dx * dx + dy * dy;
    if (g) g[d.xoff + i] = make_float2(2.f * scale * dx, 2.f * scale * dy);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) red[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)b * nrr + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}
// loss = scale * sum of the partials, in a fixed order: thread t adds
// part[t], part[t + 256], ...; fixed butterflies; the 4 wave sums in order.
__global__ void __launch_bounds__(256) k_mse_total(const float* part, int total, float scale, float* loss) {
  __shared__ float red[4];
  float s = 0.f;
  for (int i = threadIdx.x; i < total; i += 256) s += part[i];
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *loss = (((red[0] + red[1]) + red[2]) + red[3]) * scale;
}

__global__ void k_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace mrx

using namespace mrx;

extern "C" {

mrx_status mrx_cnn_set_weights(mrx_plan p, const mrx_cnn_params* w, void* stream) {
  if (!p || !w) return fail(MRX_EINVAL, "cnn_set_weights: null argument");
  if (!p->ws) return fail(MRX_ENOWORKSPACE, "cnn_set_weights: workspace not set");
  if (!(p->flags & MRX_PLAN_NETWORK))
    return fail(MRX_ENOWORKSPACE, "cnn_set_weights: plan was created without MRX_PLAN_NETWORK");
  for (int l = 0; l < 5; ++l)
    if (!w->w[l] || !w->b[l]) return fail(MRX_EINVAL, "cnn_set_weights: null weight or bias");
  hipStream_t s = (hipStream_t)stream;
  for (int l = 0; l < 5; ++l) p->net_b[l] = w->b[l];
  const int kinds[5] = {0, 1, 1, 1, 2};
  const int tkinds[5] = {2, 1, 1, 1, 0};  // dgrad of first is last-shaped and vice versa
  for (int l = 0; l < 5; ++l) {
    hipError_t e = pack_weights(kinds[l], w->w[l], pk_ptr(p, 0, l), 0, s);
    if (e == hipSuccess) e = pack_weights(tkinds[l], w->w[l], pk_ptr(p, 1, l), 1, s);
    if (e != hipSuccess) return hip_fail(e, "cnn_set_weights: pack");
  }
  p->net_ready = true;
  return MRX_OK;
}

mrx_status mrx_cnn_set_bn(mrx_plan p, const float* gamma, const float* beta, float* g_gamma, float* g_beta) {
  if (!p) return fail(MRX_EINVAL, "cnn_set_bn: null plan");
  if (!(p->flags & MRX_PLAN_BATCHNORM))
    return fail(MRX_EINVAL, "cnn_set_bn: plan was created without MRX_PLAN_BATCHNORM");
  if (!gamma || !beta) return fail(MRX_EINVAL, "cnn_set_bn: null gamma or beta");
  p->bn_gamma = gamma;
  p->bn_beta = beta;
  p->bn_ggamma = g_gamma;
  p->bn_gbeta = g_beta;
  return MRX_OK;
}

mrx_status mrx_cnn_forward(mrx_plan p, const float* x, float* z, void* stream) {
  if (!p) return fail(MRX_EINVAL, "cnn_forward: null plan");
  if (!x || !z) return fail(MRX_EINVAL, "cnn_forward: null data pointer");
  if (x == z) return fail(MRX_EINVAL, "cnn_forward: input and output must not alias");
  mrx_status st = net_ready(p, "cnn_forward");
  if (st != MRX_OK) return st;
  return cnn_fwd(p, (const float2*)x, (float2*)z, (hipStream_t)stream);
}

mrx_status mrx_cnn_backward(mrx_plan p, const float* x, const float* gz, float* gx, const mrx_cnn_grads* g,
                            int32_t accumulate, void* stream) {
  if (!p) return fail(MRX_EINVAL, "cnn_backward: null plan");
  if (!x || !gz || !gx || !g) return fail(MRX_EINVAL, "cnn_backward: null data pointer");
  for (int l = 0; l < 5; ++l)
    if (!g->w[l] || !g->b[l]) return fail(MRX_EINVAL, "cnn_backward: null gradient buffer");
  if (gx == gz) return fail(MRX_EINVAL, "cnn_backward: gx and gz must not alias");
  mrx_status st = net_ready(p, "cnn_backward");
  if (st != MRX_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  float2* z = (float2*)(p->ws + p->ws_z);
  st = cnn_fwd(p, (const float2*)x, z, s);  // recompute the activations at x
  if (st != MRX_OK) return st;
  return cnn_bwd(p, (const float2*)x, (const float2*)gz, (float2*)gx, g, accumulate, s);
}

mrx_status mrx_cnn_layer_forward(mrx_plan p, int32_t layer, const void* in, void* out, void* stream) {
  if (!p) return fail(MRX_EINVAL, "cnn_layer_forward: null plan");
  if (!in || !out || in == out) return fail(MRX_EINVAL, "cnn_layer_forward: bad data pointers");
  if (layer < 1 || layer > 3) return fail(MRX_EINVAL, "cnn_layer_forward: layer must be 1, 2 or 3");
  mrx_status st = net_ready(p, "cnn_layer_forward");
  if (st != MRX_OK) return st;
  ConvArgs m = conv_args(p);
  m.mode = CONV_FWD;
  m.in_bf16 = (const uint16_t*)in;
  m.out_bf16 = (uint16_t*)out;
  m.wpk = pk_ptr(p, 0, layer);
  m.bias = p->net_b[layer];
  hipError_t e;
  {
    KernelTimer kt(p, MRX_KERNEL_CONV_MID, (hipStream_t)stream);
    e = conv_launch(1, m, (hipStream_t)stream);
  }
  return e == hipSuccess ? MRX_OK : hip_fail(e, "cnn_layer_forward");
}

mrx_status mrx_modl_forward(mrx_plan p, const float* aHy, const float* S, const float* mask, const float* lambda,
                            int32_t T, int32_t n_cg, float* x_out, float* states, void* stream) {
  return mrx_modl_forward_from(p, aHy, aHy, S, mask, lambda, T, n_cg, x_out, states, stream);
}

mrx_status mrx_modl_forward_from(mrx_plan p, const float* x0, const float* aHy, const float* S, const float* mask,
                                 const float* lambda, int32_t T, int32_t n_cg, float* x_out, float* states,
                                 void* stream) {
  if (!p) return fail(MRX_EINVAL, "modl_forward: null plan");
  if (!x0 || !aHy || !S || !mask || !lambda || !x_out) return fail(MRX_EINVAL, "modl_forward: null data pointer");
  if (T < 0 || T > 1000 || n_cg < 0 || n_cg > 100000) return fail(MRX_EINVAL, "modl_forward: T or n_cg out of range");
  mrx_status st = net_ready(p, "modl_forward");
  if (st != MRX_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const int64_t ni = p->n_image;
  float2* z = (float2*)(p->ws + p->ws_z);
  float2* st2 = (float2*)states;
  const float2* prev = (const float2*)x0;
  if (st2) {
    hipError_t e = copy_c((const float2*)x0, st2, ni, s);
    if (e != hipSuccess) return hip_fail(e, "modl_forward: copy");
  }
  if (T == 0) {
    hipError_t e = copy_c((const float2*)x0, (float2*)x_out, ni, s);
    return e == hipSuccess ? MRX_OK : hip_fail(e, "modl_forward: copy");
  }
  for (int t = 0; t < T; ++t) {
    st = cnn_fwd(p, prev, z, s, /*fuse12=*/true);
    if (st != MRX_OK) return st;
    float2* next;
    if (t == T - 1) next = (float2*)x_out;
    else if (st2) next = st2 + (int64_t)(t + 1) * ni;
    else next = (float2*)(p->ws + p->ws_ximg[t & 1]);
    st = cg_impl(p, (const float2*)aHy, z, (const float2*)S, mask, lambda, n_cg, next, nullptr, s);
    if (st != MRX_OK) return st;
    prev = next;
  }
  if (st2) {
    hipError_t e = copy_c((const float2*)x_out, st2 + (int64_t)T * ni, ni, s);
    if (e != hipSuccess) return hip_fail(e, "modl_forward: copy");
  }
  return MRX_OK;
}

mrx_status mrx_modl_backward(mrx_plan p, const float* g_out, const float* states, const float* aHy, const float* S,
                             const float* mask, const float* lambda, int32_t T, int32_t n_cg,
                             const mrx_cnn_grads* g, float* g_lambda, float* g_aHy, int32_t accumulate,
                             void* stream) {
  if (!p) return fail(MRX_EINVAL, "modl_backward: null plan");
  if (!g_out || !states || !aHy || !S || !mask || !lambda || !g)
    return fail(MRX_EINVAL, "modl_backward: null data pointer");
  for (int l = 0; l < 5; ++l)
    if (!g->w[l] || !g->b[l]) return fail(MRX_EINVAL, "modl_backward: null gradient buffer");
  if (T < 1 || T > 1000 || n_cg < 0 || n_cg > 100000) return fail(MRX_EINVAL, "modl_backward: T or n_cg out of range");
  mrx_status st = net_ready(p, "modl_backward");
  if (st != MRX_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const int64_t ni = p->n_image;
  const float2* X = (const float2*)states;
  float2* z = (float2*)(p->ws + p->ws_z);
  float2* gcur = (float2*)(p->ws + p->ws_gimg[0]);
  float2* gz = (float2*)(p->ws + p->ws_gimg[1]);
  float2* v = (float2*)(p->ws + p->ws_vimg);
  float* part = (float*)(p->ws + p->ws_part);
  hipError_t e = copy_c((const float2*)g_out, gcur, ni, s);
  if (e != hipSuccess) return hip_fail(e, "modl_backward: copy");
  if (g_aHy && !accumulate) {
    e = fill_u32((uint32_t*)g_aHy, 0u, 2 * ni, s);
    if (e != hipSuccess) return hip_fail(e, "modl_backward: clear");
  }
  for (int t = T - 1; t >= 0; --t) {
    const float2* xt = X + (int64_t)t * ni;
    const float2* xn = X + (int64_t)(t + 1) * ni;
    st = cnn_fwd(p, xt, z, s);  // recompute z_t and the activations at x_t
    if (st != MRX_OK) return st;
    st = cg_impl(p, gcur, nullptr, (const float2*)S, mask, lambda, n_cg, v, nullptr, s);
    if (st != MRX_OK) return st;
    CgElemArgs a = elem_args(p, lambda);
    a.aHy = xn;
    a.z = z;
    a.x = v;
    e = cg_bwd_tail(a, gz, g_lambda ? part : nullptr, s);
    if (e == hipSuccess && g_lambda) e = slice_sum(a, part, g_lambda, (accumulate || t < T - 1) ? 1 : 0, s);
    if (e == hipSuccess && g_aHy) e = axpy_c(v, (float2*)g_aHy, ni, s);
    if (e != hipSuccess) return hip_fail(e, "modl_backward: dc tail");
    st = cnn_bwd(p, xt, gz, gcur, g, (accumulate || t < T - 1) ? 1 : 0, s);
    if (st != MRX_OK) return st;
  }
  if (g_aHy) {
    e = axpy_c(gcur, (float2*)g_aHy, ni, s);
    if (e != hipSuccess) return hip_fail(e, "modl_backward: tail");
  }
  return MRX_OK;
}

// out[0] (+)= sum of a[0..n) in a fixed order (per-thread strided sums, a
// fixed butterfly, the four wavefront sums in order).
__global__ void __launch_bounds__(256) k_sum_f32(const float* a, int n, float* out, int accumulate) {
  __shared__ float red[4];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) s += a[i];
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float t = ((red[0] + red[1]) + red[2]) + red[3];
    out[0] = accumulate ? out[0] + t : t;
  }
}

// ------------------------------------------------------------ soft-SENSE
// Images of soft-SENSE plans hold [2][H][W] per slice at 2 xoff.  The
// network block updates the first set's image only: it is taken out into the
// SENSE layout, denoised, and put back beside the unchanged second set.

// dst[xoff + i] = src[2 xoff + i]: the first set's image of every slice.
__global__ void k_soft_take(const SliceDesc* desc, int B, const float2* src, float2* dst) {
  const int b = blockIdx.y;
  if (b >= B) return;
  const SliceDesc d = desc[b];
  const int64_t n = (int64_t)d.H * d.W;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[d.xoff + i] = src[2 * d.xoff + i];
}
// out = (first, second's second set): out[2 xoff + i] = first[xoff + i],
// out[2 xoff + n + i] = second[2 xoff + n + i].
__global__ void k_soft_merge(const SliceDesc* desc, int B, const float2* first, const float2* second, float2* out) {
  const int b = blockIdx.y;
  if (b >= B) return;
  const SliceDesc d = desc[b];
  const int64_t n = (int64_t)d.H * d.W;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    out[2 * d.xoff + i] = first[d.xoff + i];
    out[2 * d.xoff + n + i] = second[2 * d.xoff + n + i];
  }
}
static hipError_t soft_take(mrx_plan_s* p, const float2* src, float2* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_soft_take, dim3(64, p->B), dim3(256), 0, s, p->d_desc, p->B, src, dst);
  return hipGetLastError();
}
static hipError_t soft_merge(mrx_plan_s* p, const float2* first, const float2* second, float2* out, hipStream_t s) {
  hipLaunchKernelGGL(k_soft_merge, dim3(64, p->B), dim3(256), 0, s, p->d_desc, p->B, first, second, out);
  return hipGetLastError();
}

// MSE on the coil images sum_m S_{m,c} x_m against ref (coil sized), its
// gradient g_m = sum_c conj(S_{m,c}) 2 (coil_c - ref_c) scale, and per-block
// partial sums of the squared error (block = CG_EPB pixels of a slice).
__global__ void __launch_bounds__(256) k_soft_coil_mse(const SliceDesc* desc, const float2* x, const float2* S,
                                                       const float2* ref, float2* g, float* part, int nrr,
                                                       float scale) {
  __shared__ float red[4];
  const int b = blockIdx.y;
  const SliceDesc d = desc[b];
  const int64_t n = (int64_t)d.H * d.W;
  float acc = 0.f;
  const int64_t base = (int64_t)blockIdx.x * CG_EPB;
  for (int k = threadIdx.x; k < CG_EPB; k += 256) {
    const int64_t i = base + k;
    if (i >= n) break;
    const float2 x0 = x[2 * d.xoff + i], x1 = x[2 * d.xoff + n + i];
    float2 g0 = make_float2(0.f, 0.f), g1 = make_float2(0.f, 0.f);
    for (int c = 0; c < d.C; ++c) {
      const float2 s0 = S[2 * d.soff + (int64_t)c * n + i], s1 = S[2 * d.soff + (int64_t)(d.C + c) * n + i];
      const float2 r = ref[d.soff + (int64_t)c * n + i];
      const float2 u = csub(cadd(cmul(s0, x0), cmul(s1, x1)), r);
      acc += u.x * u.x + u.y * u.y;
      g0 = cadd(g0, cmulc(s0, u));
      g1 = cadd(g1, cmulc(s1, u));
    }
    if (g) {
      g[2 * d.xoff + i] = cscale(g0, 2.f * scale);
      g[2 * d.xoff + n + i] = cscale(g1, 2.f * scale);
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) red[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)b * nrr + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

mrx_status mrx_mse_grad(mrx_plan p, const float* x, const float* ref, float* g, float* loss, void* stream) {
  if (!p) return fail(MRX_EINVAL, "mse_grad: null plan");
  if (!x || !ref) return fail(MRX_EINVAL, "mse_grad: null data pointer");
  if (!p->ws) return fail(MRX_ENOWORKSPACE, "mse_grad: workspace not set");
  hipStream_t s = (hipStream_t)stream;
  float* part = (float*)(p->ws + p->ws_part);  // B x nrr partial sums (every plan's workspace)
  const float scale = 1.0f / (float)p->n_image;
  hipLaunchKernelGGL(k_mse, dim3(p->nrr, p->B), dim3(256), 0, s, p->d_desc, p->d_all, (const float2*)x,
                     (const float2*)ref, (float2*)g, part, p->nrr, scale);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && loss) {
    hipLaunchKernelGGL(k_mse_total, dim3(1), dim3(256), 0, s, part, p->B * p->nrr, scale, loss);
    e = hipGetLastError();
  }
  return e == hipSuccess ? MRX_OK : hip_fail(e, "mse_grad");
}

mrx_status mrx_soft_modl_forward(mrx_plan p, const float* aHy, const float* S, const float* mask,
                                 const float* lambda, int32_t T, int32_t n_cg, float* x_out, float* states,
                                 void* stream) {
  if (!p) return fail(MRX_EINVAL, "soft_modl_forward: null plan");
  if (p->sets < 2) return fail(MRX_EINVAL, "soft_modl_forward: plan was created without MRX_PLAN_SOFT_SENSE");
  if (!aHy || !S || !mask || !lambda || !x_out) return fail(MRX_EINVAL, "soft_modl_forward: null data pointer");
  if (T < 0 || T > 1000 || n_cg < 0 || n_cg > 100000)
    return fail(MRX_EINVAL, "soft_modl_forward: T or n_cg out of range");
  mrx_status st = net_ready(p, "soft_modl_forward");
  if (st != MRX_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const int64_t ns = p->n_image * p->sets;
  float2* z = (float2*)(p->ws + p->ws_z);
  float2* x1 = (float2*)(p->ws + p->ws_s1[0]);
  float2* z1 = (float2*)(p->ws + p->ws_s1[1]);
  float2* st2 = (float2*)states;
  const float2* prev = (const float2*)aHy;
  hipError_t e = hipSuccess;
  if (st2) e = copy_c((const float2*)aHy, st2, ns, s);
  if (e == hipSuccess && T == 0) e = copy_c((const float2*)aHy, (float2*)x_out, ns, s);
  if (e != hipSuccess) return hip_fail(e, "soft_modl_forward: copy");
  for (int t = 0; t < T; ++t) {
    e = soft_take(p, prev, x1, s);
    if (e != hipSuccess) return hip_fail(e, "soft_modl_forward: take");
    st = cnn_fwd(p, x1, z1, s, /*fuse12=*/true);
    if (st != MRX_OK) return st;
    e = soft_merge(p, z1, prev, z, s);
    if (e != hipSuccess) return hip_fail(e, "soft_modl_forward: merge");
    float2* next;
    if (t == T - 1) next = (float2*)x_out;
    else if (st2) next = st2 + (int64_t)(t + 1) * ns;
    else next = (float2*)(p->ws + p->ws_ximg[t & 1]);
    st = cg_impl(p, cg_bufs_ws(p), (const float2*)aHy, z, (const float2*)S, mask, lambda, n_cg, next, nullptr, s,
                 /*soft=*/true);
    if (st != MRX_OK) return st;
    prev = next;
  }
  if (st2 && T > 0) {
    e = copy_c((const float2*)x_out, st2 + (int64_t)T * ns, ns, s);
    if (e != hipSuccess) return hip_fail(e, "soft_modl_forward: copy");
  }
  return MRX_OK;
}

mrx_status mrx_soft_modl_backward(mrx_plan p, const float* g_out, const float* states, const float* aHy,
                                  const float* S, const float* mask, const float* lambda, int32_t T, int32_t n_cg,
                                  const mrx_cnn_grads* g, float* g_lambda, float* g_aHy, int32_t accumulate,
                                  void* stream) {
  if (!p) return fail(MRX_EINVAL, "soft_modl_backward: null plan");
  if (p->sets < 2) return fail(MRX_EINVAL, "soft_modl_backward: plan was created without MRX_PLAN_SOFT_SENSE");
  if (!g_out || !states || !aHy || !S || !mask || !lambda || !g)
    return fail(MRX_EINVAL, "soft_modl_backward: null data pointer");
  for (int l = 0; l < 5; ++l)
    if (!g->w[l] || !g->b[l]) return fail(MRX_EINVAL, "soft_modl_backward: null gradient buffer");
  if (T < 1 || T > 1000 || n_cg < 0 || n_cg > 100000)
    return fail(MRX_EINVAL, "soft_modl_backward: T or n_cg out of range");
  mrx_status st = net_ready(p, "soft_modl_backward");
  if (st != MRX_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const int64_t ns = p->n_image * p->sets;
  const float2* X = (const float2*)states;
  float2* z = (float2*)(p->ws + p->ws_z);
  float2* gcur = (float2*)(p->ws + p->ws_gimg[0]);
  float2* gz = (float2*)(p->ws + p->ws_gimg[1]);
  float2* v = (float2*)(p->ws + p->ws_vimg);
  float2* x1 = (float2*)(p->ws + p->ws_s1[0]);
  float2* z1 = (float2*)(p->ws + p->ws_s1[1]);
  float2* gx1 = (float2*)(p->ws + p->ws_s1[2]);
  float* part = (float*)(p->ws + p->ws_part);
  hipError_t e = copy_c((const float2*)g_out, gcur, ns, s);
  if (e != hipSuccess) return hip_fail(e, "soft_modl_backward: copy");
  if (g_aHy && !accumulate) {
    e = fill_u32((uint32_t*)g_aHy, 0u, 2 * ns, s);
    if (e != hipSuccess) return hip_fail(e, "soft_modl_backward: clear");
  }
  for (int t = T - 1; t >= 0; --t) {
    const float2* xt = X + (int64_t)t * ns;
    const float2* xn = X + (int64_t)(t + 1) * ns;
    // z^t = (D(x_1^t), x_2^t), with the activations at x_1^t for the reverse pass
    e = soft_take(p, xt, x1, s);
    if (e != hipSuccess) return hip_fail(e, "soft_modl_backward: take");
    st = cnn_fwd(p, x1, z1, s);
    if (st != MRX_OK) return st;
    e = soft_merge(p, z1, xt, z, s);
    if (e != hipSuccess) return hip_fail(e, "soft_modl_backward: merge");
    st = cg_impl(p, cg_bufs_ws(p), gcur, nullptr, (const float2*)S, mask, lambda, n_cg, v, nullptr, s, true);
    if (st != MRX_OK) return st;
    CgElemArgs a = elem_args(p, lambda, cg_bufs_ws(p), /*soft=*/true);
    a.aHy = xn;
    a.z = z;
    a.x = v;
    e = cg_bwd_tail(a, gz, g_lambda ? part : nullptr, s);
    if (e == hipSuccess && g_lambda) e = slice_sum(a, part, g_lambda, (accumulate || t < T - 1) ? 1 : 0, s);
    if (e == hipSuccess && g_aHy) e = axpy_c(v, (float2*)g_aHy, ns, s);
    if (e != hipSuccess) return hip_fail(e, "soft_modl_backward: dc tail");
    // the denoiser's reverse pass on the first set; the second set's
    // gradient passes unchanged
    e = soft_take(p, gz, z1, s);
    if (e != hipSuccess) return hip_fail(e, "soft_modl_backward: take");
    st = cnn_bwd(p, x1, z1, gx1, g, (accumulate || t < T - 1) ? 1 : 0, s);
    if (st != MRX_OK) return st;
    e = soft_merge(p, gx1, gz, gcur, s);
    if (e != hipSuccess) return hip_fail(e, "soft_modl_backward: merge");
  }
  if (g_aHy) {
    e = axpy_c(gcur, (float2*)g_aHy, ns, s);
    if (e != hipSuccess) return hip_fail(e, "soft_modl_backward: tail");
  }
  return MRX_OK;
}

mrx_status mrx_soft_coil_mse_grad(mrx_plan p, const float* x, const float* S, const float* ref, float* g,
                                  float* loss, void* stream) {
  if (!p) return fail(MRX_EINVAL, "soft_coil_mse_grad: null plan");
  if (p->sets < 2) return fail(MRX_EINVAL, "soft_coil_mse_grad: plan was created without MRX_PLAN_SOFT_SENSE");
  if (!x || !S || !ref) return fail(MRX_EINVAL, "soft_coil_mse_grad: null data pointer");
  if (!p->ws) return fail(MRX_ENOWORKSPACE, "soft_coil_mse_grad: workspace not set");
  if (!(p->flags & MRX_PLAN_NETWORK))
    return fail(MRX_ENOWORKSPACE, "soft_coil_mse_grad: plan needs MRX_PLAN_NETWORK");
  hipStream_t s = (hipStream_t)stream;
  float* part = (float*)(p->ws + p->ws_loss);
  const float scale = 1.0f / (float)p->n_coil;
  hipLaunchKernelGGL(k_soft_coil_mse, dim3(p->nrr, p->B), dim3(256), 0, s, p->d_desc, (const float2*)x,
                     (const float2*)S, (const float2*)ref, (float2*)g, part, p->nrr, scale);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && loss) {
    hipLaunchKernelGGL(k_mse_total, dim3(1), dim3(256), 0, s, part, p->B * p->nrr, scale, loss);
    e = hipGetLastError();
  }
  return e == hipSuccess ? MRX_OK : hip_fail(e, "soft_coil_mse_grad");
}

mrx_status mrx_sum_f32(const float* a, int32_t n, float* out, int32_t accumulate, void* stream) {
  if (!a || !out) return fail(MRX_EINVAL, "sum_f32: null pointer");
  if (n < 0) return fail(MRX_EINVAL, "sum_f32: negative count");
  hipLaunchKernelGGL(k_sum_f32, dim3(1), dim3(256), 0, (hipStream_t)stream, a, n, out, accumulate);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MRX_OK : hip_fail(e, "sum_f32");
}

mrx_status mrx_adam_step(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                         float eps, int32_t step, void* stream) {
  if (!w || !g || !m || !v) return fail(MRX_EINVAL, "adam_step: null pointer");
  if (n < 0) return fail(MRX_EINVAL, "adam_step: negative size");
  if (step < 1) return fail(MRX_EINVAL, "adam_step: step counts from 1");
  if (n == 0) return MRX_OK;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, w, g, m, v, n,
                     lr, b1, b2, eps, c1, c2);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MRX_OK : hip_fail(e, "adam_step");
}

}  // extern "C"
