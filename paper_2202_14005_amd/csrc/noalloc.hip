// Allocation-free variant of the CG data-consistency solve (mrx_cg_dc), for
// callers that cannot allocate device memory: code under HIP graph capture,
// tight serving loops, harnesses that forbid allocation.  The CG vectors,
// partial sums, stop and status words live in `scratch`, a file-scope device
// array of NOALLOC_SCRATCH_BYTES that every GPU the library runs on holds
// until the process ends.  In host code `scratch` names a host-side stand-in,
// not device memory: its device address is taken once per device with
// hipGetSymbolAddress (with that device current, at the first call on it)
// and only that address is handed to kernels.  The kernels are those of
// mrx_cg_dc; only the buffers differ.
#include <mutex>

#include "api_internal.h"

namespace mrx {
namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

__device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
char* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on device `dev` (the current device).
mrx_status scratch_address(int dev, char** out) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(MRX_EINVAL, "cg_dc_noalloc: device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "cg_dc_noalloc: hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(MRX_EHIP, "cg_dc_noalloc: null scratch address");
    g_scratch_dev[dev] = (char*)ptr;
  }
  *out = g_scratch_dev[dev];
  return MRX_OK;
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Scratch layout of one solve for plan p with nq partial output planes;
// returns the bytes needed and, if base is non-null, the buffers.
size_t cg_scratch_layout(const mrx_plan_s* p, int nq, char* base, CgBufs* b) {
  size_t off = 0;
  auto take = [&](size_t bytes) { char* q = base ? base + off : nullptr; off += al256(bytes); return q; };
  const size_t img = sizeof(float2) * (size_t)p->n_image;
  const size_t B = (size_t)p->B;
  CgBufs t;
  t.r = (float2*)take(img);
  t.p[0] = (float2*)take(img);
  t.p[1] = (float2*)take(img);
  t.q = (float2*)take(img * (size_t)nq);
  t.pq = (float*)take(sizeof(float) * B * p->npq);
  t.rr[0] = (float*)take(sizeof(float) * B * p->nrr);
  t.rr[1] = (float*)take(sizeof(float) * B * p->nrr);
  t.stop = (int*)take(sizeof(int) * B);
  t.status = (uint32_t*)take(sizeof(uint32_t) * B);
  if (b) *b = t;
  return off;
}

__global__ void k_copy_u32(const uint32_t* src, uint32_t* dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace
}  // namespace mrx

using namespace mrx;

extern "C" mrx_status mrx_cg_dc_noalloc(mrx_plan p, const float* aHy, const float* z, const float* S,
                                        const float* mask, const float* lambda, int32_t n_iter, float* x,
                                        float* resid_hist, uint32_t* dev_flags, void* stream) {
  if (!p) return fail(MRX_EINVAL, "cg_dc_noalloc: null plan");
  if (!aHy || !S || !mask || !lambda || !x) return fail(MRX_EINVAL, "cg_dc_noalloc: null data pointer");
  if (n_iter < 0 || n_iter > 100000) return fail(MRX_EINVAL, "cg_dc_noalloc: n_iter out of range");
  if (p->toep) return fail(MRX_EINVAL, "cg_dc_noalloc: Toeplitz plans need the workspace (use mrx_cg_dc)");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "cg_dc_noalloc: hipGetDevice");
  if (dev != p->device)
    return fail(MRX_EINVAL, "cg_dc_noalloc: the current device (" + std::to_string(dev) +
                                ") is not the plan's device (" + std::to_string(p->device) + ")");
  int nq = 1;
  for (const auto& g : p->groups)
    if (g.col && g.col->kspl > nq) nq = g.col->kspl;
  const size_t need = cg_scratch_layout(p, nq, nullptr, nullptr);
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(MRX_EINVAL, "cg_dc_noalloc: the plan needs " + std::to_string(need) +
                                " bytes of scratch, more than the library's fixed " +
                                std::to_string(NOALLOC_SCRATCH_BYTES) + " (use mrx_cg_dc with a workspace)");
  char* base = nullptr;
  mrx_status st = scratch_address(dev, &base);
  if (st != MRX_OK) return st;
  CgBufs bufs;
  cg_scratch_layout(p, nq, base, &bufs);
  hipStream_t s = (hipStream_t)stream;
  // this call's status bits start at zero (a fill kernel: capture-safe)
  e = fill_u32(bufs.status, 0u, p->B, s);
  if (e != hipSuccess) return hip_fail(e, "cg_dc_noalloc: clear status");
  st = cg_impl(p, bufs, (const float2*)aHy, (const float2*)z, (const float2*)S, mask, lambda, n_iter, (float2*)x,
               resid_hist, s);
  if (st != MRX_OK || !dev_flags) return st;
  hipLaunchKernelGGL(k_copy_u32, dim3((p->B + 255) / 256), dim3(256), 0, s, bufs.status, dev_flags, p->B);
  e = hipGetLastError();
  return e == hipSuccess ? MRX_OK : hip_fail(e, "cg_dc_noalloc: status copy");
}
