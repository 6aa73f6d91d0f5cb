// C-ABI of the mrx library: plans, argument validation, schedule registry,
// and the SENSE / CG entry points.  See include/mrx.h for the contract.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mrx.h"
#include "api_internal.h"
#include "cg_kernels.h"
#include "sense_kernels.h"

namespace mrx {

static thread_local std::string g_last_error;

mrx_status fail(mrx_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

mrx_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return MRX_EHIP;
}

KernelTimer::KernelTimer(mrx_plan_s* p, int kid, hipStream_t s) : s_(s) {
  if (!p->ktime || kid < 0) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  while (p->kpool.size() < p->kpool_used + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    p->kpool.push_back(e);
  }
  hipEvent_t a = p->kpool[p->kpool_used], b = p->kpool[p->kpool_used + 1];
  if (hipEventRecord(a, s) != hipSuccess) return;
  p->kpool_used += 2;
  p->kev.push_back({a, b, kid});
  b_ = b;
}

KernelTimer::~KernelTimer() {
  if (b_) (void)hipEventRecord(b_, s_);
}

static std::vector<ColVariant>& col_registry() {
  static std::vector<ColVariant> v;
  return v;
}
static std::vector<RowVariant>& row_registry() {
  static std::vector<RowVariant> v;
  return v;
}
static std::vector<SoftVariant>& soft_registry() {
  static std::vector<SoftVariant> v;
  return v;
}
void register_soft_variant(const SoftVariant& v) { soft_registry().push_back(v); }
static std::vector<ToepVariant>& toep_registry() {
  static std::vector<ToepVariant> v;
  return v;
}
void register_toep_variant(const ToepVariant& v) { toep_registry().push_back(v); }
const ToepVariant* find_toep(int N) {
  for (auto& v : toep_registry())
    if (v.N == N) return &v;
  return nullptr;
}
const SoftVariant* find_soft(int N) {
  for (auto& v : soft_registry())
    if (v.N == N) return &v;
  return nullptr;
}
void register_col_variant(const ColVariant& v) { col_registry().push_back(v); }
void register_row_variant(const RowVariant& v) { row_registry().push_back(v); }

// Default schedule per length: the first registered one unless the tune
// cache says otherwise.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, std::string> g_tune_cache;  // (H, W, C, slices) -> column schedule name

const ColVariant* find_col(int N, const char* name) {
  for (auto& v : col_registry())
    if (v.N == N && (!name || std::strcmp(v.name, name) == 0)) return &v;
  return nullptr;
}
const RowVariant* find_row(int N) {
  for (auto& v : row_registry())
    if (v.N == N) return &v;
  return nullptr;
}
std::vector<const ColVariant*> col_variants(int N) {
  std::vector<const ColVariant*> out;
  for (auto& v : col_registry())
    if (v.N == N) out.push_back(&v);
  return out;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace mrx

using namespace mrx;

extern "C" {

const char* mrx_version(void) { return "mrx 0.1 gfx950"; }
const char* mrx_last_error(void) { return g_last_error.c_str(); }

int32_t mrx_supported_length(int32_t n) {
  return (find_col(n, nullptr) && find_row(n)) ? 1 : 0;
}

int32_t mrx_toeplitz_supported(int32_t n) {
  return (n > 0 && n <= 512 && mrx_supported_length(n) && find_toep(2 * n)) ? 1 : 0;
}

mrx_status mrx_plan_create(mrx_plan* out, int32_t B, const int32_t* H, const int32_t* W,
                           const int32_t* C, uint32_t flags) {
  if (!out) return fail(MRX_EINVAL, "plan_create: null plan pointer");
  *out = nullptr;
  if (B <= 0 || B > (1 << 20)) return fail(MRX_EINVAL, "plan_create: batch size must be in [1, 2^20]");
  if (!H || !W || !C) return fail(MRX_EINVAL, "plan_create: null shape array");
  if (flags & ~(MRX_PLAN_NETWORK | MRX_PLAN_VN | MRX_PLAN_SOFT_SENSE | MRX_PLAN_TOEPLITZ | MRX_PLAN_BATCHNORM))
    return fail(MRX_EINVAL, "plan_create: unknown flags");
  if ((flags & MRX_PLAN_BATCHNORM) && !(flags & MRX_PLAN_NETWORK))
    return fail(MRX_EINVAL, "plan_create: MRX_PLAN_BATCHNORM needs MRX_PLAN_NETWORK");
  if ((flags & MRX_PLAN_SOFT_SENSE) && (flags & MRX_PLAN_VN))
    return fail(MRX_EINVAL, "plan_create: soft-SENSE plans have no VarNet workspace");
  if ((flags & MRX_PLAN_TOEPLITZ) && (flags & (MRX_PLAN_VN | MRX_PLAN_SOFT_SENSE)))
    return fail(MRX_EINVAL, "plan_create: Toeplitz plans take neither MRX_PLAN_VN nor MRX_PLAN_SOFT_SENSE");
  auto* p = new mrx_plan_s();
  p->B = B;
  p->flags = flags;
  p->sets = (flags & MRX_PLAN_SOFT_SENSE) ? 2 : 1;
  p->toep = (flags & MRX_PLAN_TOEPLITZ) != 0;
  int64_t xo = 0, so = 0, mo = 0;
  for (int b = 0; b < B; ++b) {
    const int h = H[b], w = W[b], c = C[b];
    if (h <= 0 || w <= 0 || (h & 1) || (w & 1)) {
      delete p;
      return fail(MRX_EINVAL, "plan_create: slice " + std::to_string(b) + ": H and W must be positive and even");
    }
    if (c < 1 || c > 64) {
      delete p;
      return fail(MRX_EINVAL, "plan_create: slice " + std::to_string(b) + ": coil count must be in [1, 64]");
    }
    if (!mrx_supported_length(h) || !mrx_supported_length(w)) {
      delete p;
      return fail(MRX_EUNSUPPORTED, "plan_create: slice " + std::to_string(b) + ": no transform schedule for " +
                                        std::to_string(h) + "x" + std::to_string(w));
    }
    SliceDesc d{};
    d.H = h; d.W = w; d.C = c;
    d.xoff = xo; d.soff = so; d.moff = mo;
    xo += (int64_t)h * w;
    so += (int64_t)c * h * w;
    mo += h;
    p->desc.push_back(d);
    p->maxH = std::max(p->maxH, h);
    p->maxW = std::max(p->maxW, w);
    p->maxC = std::max(p->maxC, c);
    p->maxHW = std::max<int64_t>(p->maxHW, (int64_t)h * w);
  }
  p->n_image = xo; p->n_coil = so; p->n_mask = mo;
  // groups by (H, W)
  for (int b = 0; b < B; ++b) {
    const auto& d = p->desc[b];
    Group* g = nullptr;
    for (auto& gg : p->groups)
      if (gg.H == d.H && gg.W == d.W) g = &gg;
    if (!g) {
      p->groups.push_back(Group{});
      g = &p->groups.back();
      g->H = d.H; g->W = d.W;
    }
    g->slices.push_back(b);
    g->maxC = std::max(g->maxC, d.C);
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto& g : p->groups) {
      auto it = g_tune_cache.find({g.H, g.W, g.maxC, (int)g.slices.size()});
      g.col = find_col(g.H, it != g_tune_cache.end() ? it->second.c_str() : nullptr);
      if (!g.col) g.col = find_col(g.H, nullptr);
      g.rowW = find_row(g.W);
      g.rowH = find_row(g.H);
      g.soft = find_soft(g.H);
      if (p->toep) {
        g.toepH = find_toep(2 * g.H);
        g.toepW = find_toep(2 * g.W);
      }
    }
  }
  if (p->toep)
    for (auto& g : p->groups) {
      if (!g.toepH || !g.toepW) {
        delete p;
        return fail(MRX_EUNSUPPORTED, "plan_create: no Toeplitz kernels for " + std::to_string(g.H) + "x" +
                                          std::to_string(g.W) + " (padded lengths " + std::to_string(2 * g.H) +
                                          ", " + std::to_string(2 * g.W) + ")");
      }
      // enough workgroups for the chip: about 2048 single-wavefront row
      // workgroups and 1024 column workgroups a pass
      const int ns = (int)g.slices.size();
      const int rblk = (g.H + g.toepW->rows_wt - 1) / g.toepW->rows_wt;
      const int ctil = (2 * g.W + g.toepH->cols_wt - 1) / g.toepH->cols_wt;
      g.toep_split1 = std::max(1, std::min(g.maxC, (2048 + rblk * ns - 1) / (rblk * ns)));
      g.toep_split2 = std::max(1, std::min(g.maxC, (1024 + ctil * ns - 1) / (ctil * ns)));
      g.toep_split3 = std::max(1, std::min(std::min(g.maxC, KSPL_MAX), (2048 + rblk * ns - 1) / (rblk * ns)));
    }
  if (p->sets > 1)
    for (auto& g : p->groups)
      if (!g.soft) {
        delete p;
        return fail(MRX_EUNSUPPORTED, "plan_create: no soft-SENSE kernels for H = " + std::to_string(g.H));
      }
  refresh_desc(p, false);
  p->npq = (p->maxW + 1) / 2;  // upper bound on column tiles x coil split (tile width >= 8)
  for (auto& g : p->groups)
    if (p->toep)
      p->npq = std::max(p->npq, ((g.H + g.toepW->rows_wt - 1) / g.toepW->rows_wt) * g.toep_split3);
  p->nrr = (int)((p->sets * p->maxHW + CG_EPB - 1) / CG_EPB);
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) { delete p; return hip_fail(e, "plan_create: hipGetDevice"); }
  // device tables
  size_t tb = 2 * align256(sizeof(SliceDesc) * B) + align256(sizeof(int) * B) * (p->groups.size() + 1);
  std::vector<int> lens;
  for (auto& g : p->groups) {
    if (std::find(lens.begin(), lens.end(), g.H) == lens.end()) lens.push_back(g.H);
    if (std::find(lens.begin(), lens.end(), g.W) == lens.end()) lens.push_back(g.W);
    if (p->toep) {
      if (std::find(lens.begin(), lens.end(), 2 * g.H) == lens.end()) lens.push_back(2 * g.H);
      if (std::find(lens.begin(), lens.end(), 2 * g.W) == lens.end()) lens.push_back(2 * g.W);
    }
  }
  for (int n : lens) tb += align256(sizeof(float2) * n);
  e = hipMalloc(&p->d_tables, tb);
  if (e != hipSuccess) { delete p; return fail(MRX_ENOMEM, "plan_create: hipMalloc of plan tables failed"); }
  std::vector<char> host(tb, 0);
  size_t off = 0;
  std::memcpy(host.data() + off, p->desc.data(), sizeof(SliceDesc) * B);
  p->d_desc = (SliceDesc*)((char*)p->d_tables + off);
  off += align256(sizeof(SliceDesc) * B);
  {
    // the CG element kernels' view of a slice: sets x H x W entries at
    // sets x xoff, and the soft normal operator's partial planes
    std::vector<SliceDesc> dv(p->desc);
    for (auto& d : dv) {
      d.H *= p->sets;
      d.xoff *= p->sets;
      d.nq = SOFT_KSPL;
    }
    std::memcpy(host.data() + off, dv.data(), sizeof(SliceDesc) * B);
    p->d_desc_soft = (SliceDesc*)((char*)p->d_tables + off);
    off += align256(sizeof(SliceDesc) * B);
  }
  std::vector<int> all(B);
  for (int b = 0; b < B; ++b) all[b] = b;
  std::memcpy(host.data() + off, all.data(), sizeof(int) * B);
  p->d_all = (int*)((char*)p->d_tables + off);
  off += align256(sizeof(int) * B);
  for (auto& g : p->groups) {
    std::memcpy(host.data() + off, g.slices.data(), sizeof(int) * g.slices.size());
    g.d_slices = (int*)((char*)p->d_tables + off);
    off += align256(sizeof(int) * B);
  }
  for (int n : lens) {
    std::vector<float2> t(n);
    for (int j = 0; j < n; ++j) {
      const double a = -2.0 * M_PI * (double)j / (double)n;
      t[j] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    std::memcpy(host.data() + off, t.data(), sizeof(float2) * n);
    p->tw[n] = (float2*)((char*)p->d_tables + off);
    off += align256(sizeof(float2) * n);
  }
  e = hipMemcpy(p->d_tables, host.data(), tb, hipMemcpyHostToDevice);
  if (e != hipSuccess) { (void)hipFree(p->d_tables); delete p; return hip_fail(e, "plan_create: upload"); }
  // workspace layout
  size_t w = 0;
  auto take = [&](size_t bytes) { size_t o = w; w += align256(bytes); return o; };
  p->ws_tmp = take(sizeof(float2) * p->n_coil);
  const int64_t nimg = p->n_image * p->sets;  // CG vectors hold every set
  p->ws_r = take(sizeof(float2) * nimg);
  p->ws_p = take(sizeof(float2) * nimg);
  p->ws_p2 = take(sizeof(float2) * nimg);
  p->ws_q = take(sizeof(float2) * nimg * KSPL_MAX);
  p->ws_v = take(sizeof(float2) * nimg);
  p->ws_pq = take(sizeof(float) * B * p->npq);
  p->ws_rr0 = take(sizeof(float) * B * p->nrr);
  p->ws_rr1 = take(sizeof(float) * B * p->nrr);
  p->ws_part = take(sizeof(float) * B * p->nrr);
  p->ws_stop = take(sizeof(int) * B);
  p->ws_status = take(sizeof(uint32_t) * B);
  if (p->toep) p->ws_tbuf = take(sizeof(float2) * 2 * p->n_coil);
  p->ws_bytes_base = w;
  p->ws_bytes = w + extra_workspace_bytes(p);
  // auxiliary streams for concurrent size groups (at most 3: with the
  // caller's stream that is the four hardware queues a process gets)
  const size_t naux = std::min<size_t>(p->groups.size() > 1 ? p->groups.size() - 1 : 0, 3);
  if (naux) {
    e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
    for (size_t j = 0; j < naux && e == hipSuccess; ++j) {
      hipStream_t st = nullptr;
      e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
      if (e == hipSuccess) p->aux.push_back(st);
      hipEvent_t ev = nullptr;
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e == hipSuccess) p->ev_join.push_back(ev);
    }
    if (e != hipSuccess) {
      mrx_plan_destroy(p);
      return hip_fail(e, "plan_create: auxiliary streams");
    }
  }
  *out = p;
  return MRX_OK;
}

void mrx_plan_destroy(mrx_plan p) {
  if (!p) return;
  if (p->d_tables) (void)hipFree(p->d_tables);
  for (hipEvent_t e : p->kpool) (void)hipEventDestroy(e);
  for (hipStream_t st : p->aux) (void)hipStreamDestroy(st);
  for (hipEvent_t e : p->ev_join) (void)hipEventDestroy(e);
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  delete p;
}

mrx_status mrx_plan_kernel_timing(mrx_plan p, int32_t enable) {
  if (!p) return fail(MRX_EINVAL, "kernel_timing: null plan");
  p->ktime = enable != 0;
  p->kev.clear();
  p->kpool_used = 0;
  return MRX_OK;
}

mrx_status mrx_plan_kernel_time(mrx_plan p, int32_t kid, double* total_us, int32_t* count) {
  if (!p) return fail(MRX_EINVAL, "kernel_time: null plan");
  if (kid < 0 || kid >= MRX_KERNEL_COUNT) return fail(MRX_EINVAL, "kernel_time: unknown kernel id");
  double t = 0.0;
  int32_t n = 0;
  for (const auto& e : p->kev) {
    if (e.kid != kid) continue;
    if (hipEventSynchronize(e.b) != hipSuccess) return fail(MRX_EHIP, "kernel_time: event synchronize");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e.a, e.b) != hipSuccess) return fail(MRX_EHIP, "kernel_time: elapsed time");
    t += ms * 1e3;
    ++n;
  }
  if (total_us) *total_us = t;
  if (count) *count = n;
  return MRX_OK;
}

mrx_status mrx_plan_sizes(mrx_plan p, int64_t* ni, int64_t* nc, int64_t* nm) {
  if (!p) return fail(MRX_EINVAL, "plan_sizes: null plan");
  if (ni) *ni = p->n_image;
  if (nc) *nc = p->n_coil;
  if (nm) *nm = p->n_mask;
  return MRX_OK;
}

size_t mrx_plan_workspace_bytes(mrx_plan p) { return p ? p->ws_bytes : 0; }

mrx_status mrx_plan_set_workspace(mrx_plan p, void* ptr, size_t bytes) {
  if (!p) return fail(MRX_EINVAL, "set_workspace: null plan");
  if (!ptr) return fail(MRX_EINVAL, "set_workspace: null workspace");
  if (bytes < p->ws_bytes)
    return fail(MRX_EINVAL, "set_workspace: " + std::to_string(bytes) + " bytes given, " +
                                std::to_string(p->ws_bytes) + " needed");
  if (((uintptr_t)ptr) & 255) return fail(MRX_EINVAL, "set_workspace: pointer not 256-byte aligned");
  p->ws = (char*)ptr;
  p->ws_given = bytes;
  p->net_ready = false;  // packed weights live in the workspace
  // status words and stop flags start at zero
  hipError_t e = hipMemset(p->ws + p->ws_stop, 0, align256(sizeof(int) * p->B) + align256(sizeof(uint32_t) * p->B));
  if (e != hipSuccess) return hip_fail(e, "set_workspace: clear status");
  return MRX_OK;
}

mrx_status mrx_sense_fwd(mrx_plan p, const float* x, const float* S, const float* mask,
                         const float* noise, float* y, void* stream) {
  if (!p) return fail(MRX_EINVAL, "sense_fwd: null plan");
  if (!x || !S || !mask || !y) return fail(MRX_EINVAL, "sense_fwd: null data pointer");
  if (p->toep) return fail(MRX_EINVAL, "sense_fwd: Toeplitz plan (the forward model is mrx_nufft_fwd)");
  hipStream_t s = (hipStream_t)stream;
  for (auto& g : p->groups) {
    SenseColArgs ca{p->d_desc, g.d_slices, (int)g.slices.size(), (const float2*)S, mask,
                    (const float2*)x, (float2*)y, p->tw.at(g.H)};
    hipError_t e = g.col->fwd_col(ca, g.W, s);
    if (e != hipSuccess) return hip_fail(e, "sense_fwd: column pass");
    SenseRowArgs ra{p->d_desc, g.d_slices, (int)g.slices.size(), mask, (const float2*)y, (float2*)y,
                    (const float2*)noise, p->tw.at(g.W)};
    e = g.rowW->fwd_row(ra, g.H, g.maxC, s);
    if (e != hipSuccess) return hip_fail(e, "sense_fwd: row pass");
  }
  return MRX_OK;
}

mrx_status mrx_sense_adj(mrx_plan p, const float* y, const float* S, const float* mask, float* x,
                         void* stream) {
  if (!p) return fail(MRX_EINVAL, "sense_adj: null plan");
  if (!y || !S || !mask || !x) return fail(MRX_EINVAL, "sense_adj: null data pointer");
  if (p->toep) return fail(MRX_EINVAL, "sense_adj: Toeplitz plan (the adjoint is mrx_nufft_adj)");
  if (!p->ws) return fail(MRX_ENOWORKSPACE, "sense_adj: workspace not set");
  return sense_adj_impl(p, (const float2*)y, (const float2*)S, mask, (float2*)x, (hipStream_t)stream);
}

mrx_status mrx_sense_normal(mrx_plan p, const float* x, const float* S, const float* mask,
                            const float* lambda, float* out, void* stream) {
  if (!p) return fail(MRX_EINVAL, "sense_normal: null plan");
  if (!x || !S || !mask || !out) return fail(MRX_EINVAL, "sense_normal: null data pointer");
  if (x == out) return fail(MRX_EINVAL, "sense_normal: input and output must not alias");
  if (p->toep && !p->ws) return fail(MRX_ENOWORKSPACE, "sense_normal: workspace not set (Toeplitz plan)");
  return normal_impl(p, (const float2*)x, (const float2*)S, mask, lambda, (float2*)out, (hipStream_t)stream);
}

mrx_status mrx_cg_dc(mrx_plan p, const float* aHy, const float* z, const float* S, const float* mask,
                     const float* lambda, int32_t n_iter, float* x, float* hist, void* stream) {
  if (!p) return fail(MRX_EINVAL, "cg_dc: null plan");
  if (!aHy || !S || !mask || !lambda || !x) return fail(MRX_EINVAL, "cg_dc: null data pointer");
  if (n_iter < 0 || n_iter > 100000) return fail(MRX_EINVAL, "cg_dc: n_iter out of range");
  if (!p->ws) return fail(MRX_ENOWORKSPACE, "cg_dc: workspace not set");
  return cg_impl(p, (const float2*)aHy, (const float2*)z, (const float2*)S, mask, lambda, n_iter,
                 (float2*)x, hist, (hipStream_t)stream);
}

mrx_status mrx_cg_dc_backward(mrx_plan p, const float* gx, const float* x, const float* z,
                              const float* S, const float* mask, const float* lambda, int32_t n_iter,
                              float* g_aHy, float* g_z, float* g_lambda, int32_t accumulate,
                              void* stream) {
  if (!p) return fail(MRX_EINVAL, "cg_dc_backward: null plan");
  if (!gx || !x || !S || !mask || !lambda || !g_aHy)
    return fail(MRX_EINVAL, "cg_dc_backward: null data pointer");
  if (n_iter < 0 || n_iter > 100000) return fail(MRX_EINVAL, "cg_dc_backward: n_iter out of range");
  if (!p->ws) return fail(MRX_ENOWORKSPACE, "cg_dc_backward: workspace not set");
  hipStream_t s = (hipStream_t)stream;
  mrx_status st = cg_impl(p, (const float2*)gx, nullptr, (const float2*)S, mask, lambda, n_iter,
                          (float2*)g_aHy, nullptr, s);
  if (st != MRX_OK) return st;
  if (g_z || g_lambda) {
    CgElemArgs a = elem_args(p, lambda);
    a.aHy = (const float2*)x;
    a.z = (const float2*)z;
    a.x = (float2*)g_aHy;
    float* part = (float*)(p->ws + p->ws_part);
    hipError_t e = cg_bwd_tail(a, (float2*)g_z, g_lambda ? part : nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "cg_dc_backward: tail");
    if (g_lambda) {
      e = slice_sum(a, part, g_lambda, accumulate, s);
      if (e != hipSuccess) return hip_fail(e, "cg_dc_backward: lambda gradient");
    }
  }
  return MRX_OK;
}

static mrx_status soft_ready(mrx_plan p, const char* who) {
  if (!p) return fail(MRX_EINVAL, std::string(who) + ": null plan");
  if (p->sets < 2) return fail(MRX_EINVAL, std::string(who) + ": plan was created without MRX_PLAN_SOFT_SENSE");
  return MRX_OK;
}

mrx_status mrx_soft_sense_fwd(mrx_plan p, const float* x, const float* S, const float* mask, const float* noise,
                              float* y, void* stream) {
  mrx_status st = soft_ready(p, "soft_sense_fwd");
  if (st != MRX_OK) return st;
  if (!x || !S || !mask || !y) return fail(MRX_EINVAL, "soft_sense_fwd: null data pointer");
  return soft_fwd_impl(p, (const float2*)x, (const float2*)S, mask, (const float2*)noise, (float2*)y,
                       (hipStream_t)stream);
}

mrx_status mrx_soft_sense_adj(mrx_plan p, const float* y, const float* S, const float* mask, float* x,
                              void* stream) {
  mrx_status st = soft_ready(p, "soft_sense_adj");
  if (st != MRX_OK) return st;
  if (!y || !S || !mask || !x) return fail(MRX_EINVAL, "soft_sense_adj: null data pointer");
  if (!p->ws) return fail(MRX_ENOWORKSPACE, "soft_sense_adj: workspace not set");
  return soft_adj_impl(p, (const float2*)y, (const float2*)S, mask, (float2*)x, (hipStream_t)stream);
}

mrx_status mrx_soft_sense_normal(mrx_plan p, const float* x, const float* S, const float* mask,
                                 const float* lambda, float* out, void* stream) {
  mrx_status st = soft_ready(p, "soft_sense_normal");
  if (st != MRX_OK) return st;
  if (!x || !S || !mask || !out) return fail(MRX_EINVAL, "soft_sense_normal: null data pointer");
  if (x == out) return fail(MRX_EINVAL, "soft_sense_normal: input and output must not alias");
  return soft_normal_impl(p, (const float2*)x, (const float2*)S, mask, lambda, (float2*)out, (hipStream_t)stream);
}

mrx_status mrx_soft_cg_dc(mrx_plan p, const float* aHy, const float* z, const float* S, const float* mask,
                          const float* lambda, int32_t n_iter, float* x, float* hist, void* stream) {
  mrx_status st = soft_ready(p, "soft_cg_dc");
  if (st != MRX_OK) return st;
  if (!aHy || !S || !mask || !lambda || !x) return fail(MRX_EINVAL, "soft_cg_dc: null data pointer");
  if (n_iter < 0 || n_iter > 100000) return fail(MRX_EINVAL, "soft_cg_dc: n_iter out of range");
  if (!p->ws) return fail(MRX_ENOWORKSPACE, "soft_cg_dc: workspace not set");
  return cg_impl(p, cg_bufs_ws(p), (const float2*)aHy, (const float2*)z, (const float2*)S, mask, lambda, n_iter,
                 (float2*)x, hist, (hipStream_t)stream, /*soft=*/true);
}

mrx_status mrx_status_word(mrx_plan p, uint32_t* dev_flags, int32_t clear, void* stream) {
  if (!p) return fail(MRX_EINVAL, "status_word: null plan");
  if (!p->ws) return fail(MRX_ENOWORKSPACE, "status_word: workspace not set");
  hipStream_t s = (hipStream_t)stream;
  if (dev_flags) {
    hipError_t e = hipMemcpyAsync(dev_flags, p->ws + p->ws_status, sizeof(uint32_t) * p->B,
                                  hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "status_word: copy");
  }
  if (clear) {
    hipError_t e = clear_status(p, s);
    if (e != hipSuccess) return hip_fail(e, "status_word: clear");
  }
  return MRX_OK;
}

const char* mrx_schedule_name(int32_t n, int32_t idx) {
  auto v = col_variants(n);
  if (idx < 0 || idx >= (int)v.size()) return nullptr;
  return v[idx]->name;
}

mrx_status mrx_plan_set_schedule(mrx_plan p, int32_t n, const char* name) {
  if (!p || !name) return fail(MRX_EINVAL, "plan_set_schedule: null argument");
  const ColVariant* v = find_col(n, name);
  if (!v) return fail(MRX_EUNSUPPORTED, std::string("plan_set_schedule: no schedule ") + name);
  bool any = false;
  for (auto& g : p->groups)
    if (g.H == n) { g.col = v; any = true; }
  if (!any) return fail(MRX_EINVAL, "plan_set_schedule: no slice of the plan has that H");
  return refresh_desc(p, true);
}

const char* mrx_plan_schedule(mrx_plan p, int32_t b) {
  if (!p || b < 0 || b >= p->B) return "";
  for (auto& g : p->groups)
    for (int s : g.slices)
      if (s == b) return g.col ? g.col->name : "";
  return "";
}

}  // extern "C"
