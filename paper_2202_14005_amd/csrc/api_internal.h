// Internal plan structure and host-side operator implementations.
#pragma once
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mrx.h"
#include "cg_kernels.h"
#include "common.h"
#include "sense_kernels.h"

namespace mrx {

struct Group {
  int H = 0, W = 0, maxC = 0;
  std::vector<int> slices;
  int* d_slices = nullptr;
  const ColVariant* col = nullptr;   // transform along H (column pass)
  const RowVariant* rowW = nullptr;  // transform along W (row pass)
  const RowVariant* rowH = nullptr;
  const SoftVariant* soft = nullptr;  // soft-SENSE kernels (plans with two map sets)
  // Toeplitz plans: the padded-length kernels (2H: column pass, 2W: row
  // passes), the coil groups of the first two passes and the output planes
  // of the last in CG steps
  const ToepVariant* toepH = nullptr;
  const ToepVariant* toepW = nullptr;
  int toep_split1 = 1, toep_split2 = 1, toep_split3 = 1;
};

}  // namespace mrx

struct mrx_plan_s {
  int B = 0;
  int device = 0;
  std::vector<mrx::SliceDesc> desc;
  std::vector<mrx::Group> groups;
  int maxH = 0, maxW = 0, maxC = 0;
  int64_t maxHW = 0;
  int64_t n_image = 0, n_coil = 0, n_mask = 0;
  int npq = 0, nrr = 0;
  // coil-map sets: 1 (SENSE) or 2 (soft-SENSE, MRX_PLAN_SOFT_SENSE); image
  // vectors of the CG and of the networks then hold sets x H x W per slice,
  // described by d_desc_soft (H x sets rows, offset sets x xoff) for the
  // CG element kernels
  int sets = 1;
  mrx::SliceDesc* d_desc_soft = nullptr;
  // non-Cartesian plan (MRX_PLAN_TOEPLITZ): the normal operator is the PSF
  // convolution; ws_tbuf holds the padded per-coil spectra [C][H][2W]
  bool toep = false;
  size_t ws_tbuf = 0;
  // device tables (plan owned)
  void* d_tables = nullptr;
  mrx::SliceDesc* d_desc = nullptr;
  int* d_all = nullptr;
  std::map<int, float2*> tw;
  // borrowed workspace and its layout (byte offsets)
  char* ws = nullptr;
  size_t ws_given = 0, ws_bytes = 0, ws_bytes_base = 0;
  size_t ws_tmp = 0, ws_r = 0, ws_p = 0, ws_p2 = 0, ws_q = 0, ws_v = 0;  // ws_q: KSPL_MAX planes
  size_t ws_pq = 0, ws_rr0 = 0, ws_rr1 = 0, ws_part = 0, ws_stop = 0, ws_status = 0;
  uint32_t flags = 0;
  // network workspace (set by extra_workspace_bytes)
  size_t ws_act[4] = {0, 0, 0, 0}, ws_gact[2] = {0, 0};
  size_t ws_z = 0, ws_ximg[2] = {0, 0}, ws_gimg[2] = {0, 0}, ws_vimg = 0;
  size_t ws_pk = 0, ws_wpart = 0, ws_bpart = 0, ws_loss = 0;
  size_t ws_s1[3] = {0, 0, 0};  // soft-SENSE: first-set images in the SENSE layout (denoiser in/out)
  const float* net_b[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  // batch normalisation of the hidden layers (MRX_PLAN_BATCHNORM): gamma,
  // beta [4][64] and their gradients (device, caller owned), workspace
  size_t ws_bnpre[4] = {0, 0, 0, 0}, ws_bnstats = 0, ws_bnpart = 0, ws_bnsgz = 0, ws_bnslots = 0;
  const float* bn_gamma = nullptr;
  const float* bn_beta = nullptr;
  float* bn_ggamma = nullptr;
  float* bn_gbeta = nullptr;
  // VarNet workspace
  size_t ws_vn_kt = 0, ws_vn_wa = 0, ws_vn_wd = 0, ws_vn_u = 0, ws_vn_e = 0, ws_vn_kg = 0, ws_vn_s = 0, ws_vn_qx = 0, ws_vn_qg = 0;
  size_t ws_vn_plam = 0, ws_vn_pk = 0, ws_vn_pw = 0;
  bool net_ready = false;
  // size groups of one operator application run concurrently: groups after
  // the first on auxiliary streams (default priority) forked from and
  // joined back to the caller's stream with these events
  std::vector<hipStream_t> aux;
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
  // optional timing of the hot kernels: a pair of events around each launch
  struct KEvent {
    hipEvent_t a, b;
    int kid;
  };
  bool ktime = false;
  std::vector<hipEvent_t> kpool;  // created on demand, reused after a reset
  size_t kpool_used = 0;
  std::vector<KEvent> kev;
};

namespace mrx {

mrx_status fail(mrx_status st, const std::string& msg);

// Times one launch (constructor before, destructor after) when the plan's
// kernel timing is on and the stream is not being captured.
class KernelTimer {
 public:
  KernelTimer(mrx_plan_s* p, int kid, hipStream_t s);
  ~KernelTimer();

 private:
  hipStream_t s_;
  hipEvent_t b_ = nullptr;
};
mrx_status hip_fail(hipError_t e, const char* what);
const ColVariant* find_col(int N, const char* name);
const RowVariant* find_row(int N);
const SoftVariant* find_soft(int N);
const ToepVariant* find_toep(int N);
std::vector<const ColVariant*> col_variants(int N);

extern std::mutex g_tune_mu;
extern std::map<std::tuple<int, int, int, int>, std::string> g_tune_cache;

size_t extra_workspace_bytes(mrx_plan_s* p);
// Set desc[b].nq from the column schedule of each slice's group; with
// upload, also copy the descriptors to the device (synchronous).
mrx_status refresh_desc(mrx_plan_s* p, bool upload);
size_t vn_workspace_bytes(mrx_plan_s* p, size_t base);
// Device buffers of one CG solve: residual, the two search-direction
// buffers, the partial planes of the normal operator's output (KSPL_MAX or
// the plan's largest coil split), the <p, q> and <r, r> partial sums, the
// per-slice stop words and status words.
struct CgBufs {
  float2* r = nullptr;
  float2* p[2] = {nullptr, nullptr};
  float2* q = nullptr;
  float* pq = nullptr;
  float* rr[2] = {nullptr, nullptr};
  int* stop = nullptr;
  uint32_t* status = nullptr;
};
// The plan workspace's CG buffers.
CgBufs cg_bufs_ws(mrx_plan_s* p);
CgElemArgs elem_args(mrx_plan_s* p, const float* lam);
CgElemArgs elem_args(mrx_plan_s* p, const float* lam, const CgBufs& b, bool soft = false);
hipError_t clear_status(mrx_plan_s* p, hipStream_t s);
hipError_t fill_u32(uint32_t* dst, uint32_t value, int64_t n, hipStream_t s);

// Runs fn(group, stream) for every size group of the plan: the first group
// on s, the others on the plan's auxiliary streams, forked from s before and
// joined back into s after (parallel branches under graph capture), so that
// one group's last workgroups overlap the next group's.  With one group (or
// no auxiliary streams) everything runs on s in order.
template <class F>
hipError_t for_groups(mrx_plan_s* p, hipStream_t s, F fn) {
  const size_t G = p->groups.size();
  const size_t A = p->aux.size();
  if (G <= 1 || A == 0) {
    for (auto& g : p->groups) {
      hipError_t e = fn(g, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  hipError_t e = hipEventRecord(p->ev_fork, s);
  if (e != hipSuccess) return e;
  for (size_t j = 0; j < A && j + 1 < G; ++j) {
    e = hipStreamWaitEvent(p->aux[j], p->ev_fork, 0);
    if (e != hipSuccess) return e;
  }
  for (size_t i = 0; i < G; ++i) {
    e = fn(p->groups[i], i == 0 ? s : p->aux[(i - 1) % A]);
    if (e != hipSuccess) return e;
  }
  for (size_t j = 0; j < A && j + 1 < G; ++j) {
    e = hipEventRecord(p->ev_join[j], p->aux[j]);
    if (e != hipSuccess) return e;
    e = hipStreamWaitEvent(s, p->ev_join[j], 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

mrx_status sense_adj_impl(mrx_plan_s* p, const float2* y, const float2* S, const float* mask, float2* x,
                          hipStream_t s);
hipError_t normal_group(mrx_plan_s* p, mrx::Group& g, const float2* x, const float2* S, const float* mask,
                        const float* lam, float2* out, hipStream_t s);
mrx_status normal_impl(mrx_plan_s* p, const float2* x, const float2* S, const float* mask, const float* lam,
                       float2* out, hipStream_t s);
mrx_status cg_impl(mrx_plan_s* p, const float2* aHy, const float2* z, const float2* S, const float* mask,
                   const float* lam, int n_iter, float2* x, float* hist, hipStream_t s);
mrx_status cg_impl(mrx_plan_s* p, const CgBufs& bufs, const float2* aHy, const float2* z, const float2* S,
                   const float* mask, const float* lam, int n_iter, float2* x, float* hist, hipStream_t s,
                   bool soft = false);
// soft-SENSE (two map sets): forward, adjoint and normal operators, CG on the
// plan workspace
mrx_status soft_fwd_impl(mrx_plan_s* p, const float2* x, const float2* S, const float* mask, const float2* noise,
                         float2* y, hipStream_t s);
mrx_status soft_adj_impl(mrx_plan_s* p, const float2* y, const float2* S, const float* mask, float2* x,
                         hipStream_t s);
mrx_status soft_normal_impl(mrx_plan_s* p, const float2* x, const float2* S, const float* mask, const float* lam,
                            float2* out, hipStream_t s);
// Toeplitz plans: the three passes of the normal operator for one size
// group (a.pin .. a.stopped as for a plain application or a CG step; tw,
// split and the buffer are filled in here)
hipError_t toep_apply(mrx_plan_s* p, Group& g, ToepArgs a, hipStream_t s);

}  // namespace mrx
