// Host-side sequencing of the SENSE and CG operators on the device.
#include <algorithm>
#include <chrono>
#include <mutex>

#include "api_internal.h"

namespace mrx {

static_assert(KSPL_MAX <= CG_QPARTS_MAX && SOFT_KSPL <= CG_QPARTS_MAX, "k_cg_update must add every partial plane");

__global__ void k_fill_u32(uint32_t* d, uint32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = v;
}

hipError_t fill_u32(uint32_t* dst, uint32_t value, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, dst, value, n);
  return hipGetLastError();
}

hipError_t clear_status(mrx_plan_s* p, hipStream_t s) {
  return fill_u32((uint32_t*)(p->ws + p->ws_status), 0u, p->B, s);
}

mrx_status refresh_desc(mrx_plan_s* p, bool upload) {
  for (auto& g : p->groups)
    for (int b : g.slices)
      p->desc[b].nq = p->toep ? g.toep_split3 : (g.col && g.col->kspl > 1) ? g.col->kspl : 1;
  if (!upload) return MRX_OK;
  hipError_t e = hipMemcpy(p->d_desc, p->desc.data(), sizeof(SliceDesc) * p->B, hipMemcpyHostToDevice);
  return e == hipSuccess ? MRX_OK : hip_fail(e, "plan: descriptor upload");
}

CgBufs cg_bufs_ws(mrx_plan_s* p) {
  CgBufs b;
  b.r = (float2*)(p->ws + p->ws_r);
  b.p[0] = (float2*)(p->ws + p->ws_p);
  b.p[1] = (float2*)(p->ws + p->ws_p2);
  b.q = (float2*)(p->ws + p->ws_q);
  b.pq = (float*)(p->ws + p->ws_pq);
  b.rr[0] = (float*)(p->ws + p->ws_rr0);
  b.rr[1] = (float*)(p->ws + p->ws_rr1);
  b.stop = (int*)(p->ws + p->ws_stop);
  b.status = (uint32_t*)(p->ws + p->ws_status);
  return b;
}

CgElemArgs elem_args(mrx_plan_s* p, const float* lam, const CgBufs& b, bool soft) {
  CgElemArgs a{};
  a.desc = soft ? p->d_desc_soft : p->d_desc;
  a.slices = p->d_all;
  a.nslices = p->B;
  a.nrr = p->nrr;
  a.npq = p->npq;
  a.lam = lam;
  a.stopped = b.stop;
  a.status = b.status;
  return a;
}

CgElemArgs elem_args(mrx_plan_s* p, const float* lam) { return elem_args(p, lam, cg_bufs_ws(p)); }

mrx_status sense_adj_impl(mrx_plan_s* p, const float2* y, const float2* S, const float* mask, float2* x,
                          hipStream_t s) {
  float2* tmp = (float2*)(p->ws + p->ws_tmp);
  for (auto& g : p->groups) {
    SenseRowArgs ra{p->d_desc, g.d_slices, (int)g.slices.size(), mask, y, tmp, nullptr, p->tw.at(g.W)};
    hipError_t e = g.rowW->adj_row(ra, g.H, g.maxC, s);
    if (e != hipSuccess) return hip_fail(e, "sense_adj: row pass");
    SenseColArgs ca{p->d_desc, g.d_slices, (int)g.slices.size(), S, mask, tmp, x, p->tw.at(g.H)};
    e = g.col->adj_col(ca, g.W, s);
    if (e != hipSuccess) return hip_fail(e, "sense_adj: column pass");
  }
  return MRX_OK;
}

hipError_t toep_apply(mrx_plan_s* p, Group& g, ToepArgs a, hipStream_t s) {
  const bool cg = a.mode == 1;
  a.slices = g.d_slices;
  a.nslices = (int)g.slices.size();
  a.tbuf = (float2*)(p->ws + p->ws_tbuf);
  a.tw = p->tw.at(2 * g.W);
  a.split = g.toep_split1;
  hipError_t e = g.toepW->rows_fwd(a, g.H, s);
  if (e != hipSuccess) return e;
  a.tw = p->tw.at(2 * g.H);
  a.split = g.toep_split2;
  e = g.toepH->cols(a, 2 * g.W, s);
  if (e != hipSuccess) return e;
  a.tw = p->tw.at(2 * g.W);
  a.split = cg ? g.toep_split3 : 1;
  return g.toepW->rows_adj(a, g.H, s);
}

static mrx_status toep_normal_impl(mrx_plan_s* p, const float2* x, const float2* S, const float* psf,
                                   const float* lam, float2* out, hipStream_t s) {
  KernelTimer kt(p, MRX_KERNEL_NORMAL, s);
  hipError_t e = for_groups(p, s, [&](Group& g, hipStream_t sg) {
    ToepArgs a{};
    a.desc = p->d_desc;
    a.S = S;
    a.psf = psf;
    a.lam = lam;
    a.pin = x;
    a.qout = out;
    a.mode = 0;
    return toep_apply(p, g, a, sg);
  });
  return e == hipSuccess ? MRX_OK : hip_fail(e, "toeplitz normal operator");
}

// out = sum_{k < nparts} part[k qstride + .] over the slices of one launch,
// in plane order (the order k_cg_update adds the planes of a CG step).
__global__ void k_add_planes(const SliceDesc* desc, const int* slices, const float2* part, int nparts,
                             int64_t qstride, float2* out) {
  const SliceDesc d = desc[slices[blockIdx.y]];
  const int64_t n = (int64_t)d.H * d.W;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = d.xoff + i;
    float2 v = part[o];
    for (int k = 1; k < nparts; ++k) v = cadd(v, part[k * qstride + o]);
    out[o] = v;
  }
}

// One size group's operator application.  When the group's schedule splits
// a column tile's coils over several workgroups (the CG-step split) and the
// plan's coil-sized scratch holds that many image planes, the application
// uses the split too -- a batch with few column tiles then fills the chip --
// and a fixed-order sum adds the partial planes into out.
hipError_t normal_group(mrx_plan_s* p, Group& g, const float2* x, const float2* S, const float* mask,
                        const float* lam, float2* out, hipStream_t s) {
  NormalArgs na{};
  na.desc = p->d_desc;
  na.slices = g.d_slices;
  na.nslices = (int)g.slices.size();
  na.S = S;
  na.mask = mask;
  na.lam = lam;
  na.pin = x;
  na.qout = out;
  na.tw = p->tw.at(g.H);
  na.mode = 0;
  const int ks = g.col->kspl;
  if (ks <= 1 || !p->ws || (int64_t)ks * p->n_image > p->n_coil) return g.col->normal(na, g.W, s);
  float2* part = (float2*)(p->ws + p->ws_tmp);
  na.qout = part;
  na.qstride = p->n_image;
  na.split_plain = 1;
  hipError_t e = g.col->normal(na, g.W, s);
  if (e != hipSuccess) return e;
  const int64_t hw = (int64_t)g.H * g.W;
  const unsigned blocks = (unsigned)std::min<int64_t>((hw + 255) / 256, 1024);
  hipLaunchKernelGGL(k_add_planes, dim3(blocks, (unsigned)g.slices.size()), dim3(256), 0, s, p->d_desc,
                     g.d_slices, (const float2*)part, ks, p->n_image, out);
  return hipGetLastError();
}

mrx_status normal_impl(mrx_plan_s* p, const float2* x, const float2* S, const float* mask, const float* lam,
                       float2* out, hipStream_t s) {
  if (p->toep) return toep_normal_impl(p, x, S, mask, lam, out, s);
  KernelTimer kt(p, MRX_KERNEL_NORMAL, s);
  hipError_t e = for_groups(p, s, [&](Group& g, hipStream_t sg) {
    return normal_group(p, g, x, S, mask, lam, out, sg);
  });
  return e == hipSuccess ? MRX_OK : hip_fail(e, "sense_normal");
}

// Soft-SENSE operators: the soft column passes and the SENSE row passes.
mrx_status soft_fwd_impl(mrx_plan_s* p, const float2* x, const float2* S, const float* mask, const float2* noise,
                         float2* y, hipStream_t s) {
  for (auto& g : p->groups) {
    SenseColArgs ca{p->d_desc, g.d_slices, (int)g.slices.size(), S, mask, x, y, p->tw.at(g.H)};
    hipError_t e = g.soft->fwd_col(ca, g.W, s);
    if (e != hipSuccess) return hip_fail(e, "soft_sense_fwd: column pass");
    SenseRowArgs ra{p->d_desc, g.d_slices, (int)g.slices.size(), mask, y, y, noise, p->tw.at(g.W)};
    e = g.rowW->fwd_row(ra, g.H, g.maxC, s);
    if (e != hipSuccess) return hip_fail(e, "soft_sense_fwd: row pass");
  }
  return MRX_OK;
}

mrx_status soft_adj_impl(mrx_plan_s* p, const float2* y, const float2* S, const float* mask, float2* x,
                         hipStream_t s) {
  float2* tmp = (float2*)(p->ws + p->ws_tmp);
  for (auto& g : p->groups) {
    SenseRowArgs ra{p->d_desc, g.d_slices, (int)g.slices.size(), mask, y, tmp, nullptr, p->tw.at(g.W)};
    hipError_t e = g.rowW->adj_row(ra, g.H, g.maxC, s);
    if (e != hipSuccess) return hip_fail(e, "soft_sense_adj: row pass");
    SenseColArgs ca{p->d_desc, g.d_slices, (int)g.slices.size(), S, mask, tmp, x, p->tw.at(g.H)};
    e = g.soft->adj_col(ca, g.W, s);
    if (e != hipSuccess) return hip_fail(e, "soft_sense_adj: column pass");
  }
  return MRX_OK;
}

mrx_status soft_normal_impl(mrx_plan_s* p, const float2* x, const float2* S, const float* mask, const float* lam,
                            float2* out, hipStream_t s) {
  KernelTimer kt(p, MRX_KERNEL_NORMAL, s);
  hipError_t e = for_groups(p, s, [&](Group& g, hipStream_t sg) {
    NormalArgs na{};
    na.desc = p->d_desc;
    na.slices = g.d_slices;
    na.nslices = (int)g.slices.size();
    na.S = S;
    na.mask = mask;
    na.lam = lam;
    na.pin = x;
    na.qout = out;
    na.tw = p->tw.at(g.H);
    na.mode = 0;
    // split like a CG step when the coil-sized scratch holds the partial
    // planes of both sets (the few column tiles of a batch then fill the
    // chip); a fixed-order sum adds them into out
    const int64_t simg = p->n_image * p->sets;
    if (!p->ws || SOFT_KSPL * simg > p->n_coil) return g.soft->normal(na, g.W, sg);
    float2* part = (float2*)(p->ws + p->ws_tmp);
    na.qout = part;
    na.qstride = simg;
    na.split_plain = 1;
    hipError_t e2 = g.soft->normal(na, g.W, sg);
    if (e2 != hipSuccess) return e2;
    const int64_t n = (int64_t)p->sets * g.H * g.W;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_add_planes, dim3(blocks, (unsigned)g.slices.size()), dim3(256), 0, sg, p->d_desc_soft,
                       g.d_slices, (const float2*)part, SOFT_KSPL, simg, out);
    return hipGetLastError();
  });
  return e == hipSuccess ? MRX_OK : hip_fail(e, "soft_sense_normal");
}

mrx_status cg_impl(mrx_plan_s* p, const float2* aHy, const float2* z, const float2* S, const float* mask,
                   const float* lam, int n_iter, float2* x, float* hist, hipStream_t s) {
  return cg_impl(p, cg_bufs_ws(p), aHy, z, S, mask, lam, n_iter, x, hist, s);
}

// x = CG_n(A^H A + lam I, aHy + lam z) from x0 = 0, on the buffers bb.
mrx_status cg_impl(mrx_plan_s* p, const CgBufs& bb, const float2* aHy, const float2* z, const float2* S,
                   const float* mask, const float* lam, int n_iter, float2* x, float* hist, hipStream_t s,
                   bool soft) {
  float2* r = bb.r;
  // p_k lives in pb[k & 1]: the step that forms p_k = r_k + beta p_{k-1}
  // reads the other buffer, so workgroups splitting a tile's coils never
  // see a half-updated p
  float2* pb[2] = {bb.p[0], bb.p[1]};
  float2* pv = pb[0];
  float2* q = bb.q;
  float* pq = bb.pq;
  float* rr[2] = {bb.rr[0], bb.rr[1]};
  CgElemArgs a = elem_args(p, lam, bb, soft);
  a.aHy = aHy;
  a.z = z;
  a.x = x;
  a.r = r;
  a.p = pv;
  a.q = q;
  // partial planes of a coil split hold every coil-map set
  const int64_t qstride = p->n_image * (soft ? p->sets : 1);
  a.qstride = qstride;
  a.pq = pq;
  a.hist = hist;
  a.rr_next = rr[0];
  a.pq_clear = pq;  // cg_init also clears the <p, q> partials
  hipError_t e = cg_init(a, s);
  a.pq_clear = nullptr;
  if (e != hipSuccess) return hip_fail(e, "cg: init");
  for (int k = 0; k < n_iter; ++k) {
    float* rr_cur = rr[k & 1];
    float* rr_prev = rr[(k + 1) & 1];
    if (hist) {
      a.rr_cur = rr_cur;
      e = cg_hist(a, k, n_iter + 1, s);
      if (e != hipSuccess) return hip_fail(e, "cg: history");
    }
    // soft-SENSE: p_k = r_k + beta p_{k-1} formed once, which the operator
    // then reads as given (instead of forming it for every coil and set)
    const bool soft_form = soft && k > 0;
    if (soft_form) {
      CgElemArgs fa = a;
      fa.rr_cur = rr_cur;
      fa.rr_next = rr_prev;
      fa.p = pb[(k - 1) & 1];
      fa.x = pb[k & 1];
      e = cg_form_p(fa, s);
      if (e != hipSuccess) return hip_fail(e, "cg: search direction");
    }
    {
      KernelTimer kt(p, MRX_KERNEL_NORMAL, s);
      e = for_groups(p, s, [&](Group& g, hipStream_t sg) {
        if (p->toep) {
          ToepArgs ta{};
          ta.desc = p->d_desc;
          ta.S = S;
          ta.psf = mask;
          ta.lam = lam;
          ta.pin = pb[k == 0 ? 0 : ((k - 1) & 1)];
          ta.qout = q;
          ta.qstride = p->n_image;
          ta.mode = 1;
          ta.iter = k;
          ta.r = r;
          ta.pout = pb[k & 1];
          ta.rr_cur = rr_cur;
          ta.rr_prev = rr_prev;
          ta.nrr = p->nrr;
          ta.pq_part = pq;
          ta.npq = p->npq;
          ta.stopped = a.stopped;
          return toep_apply(p, g, ta, sg);
        }
        NormalArgs na{};
        na.desc = p->d_desc;
        na.slices = g.d_slices;
        na.nslices = (int)g.slices.size();
        na.S = S;
        na.mask = mask;
        na.lam = lam;
        // (soft: p_0 = r_0 from the initialisation, later p_k formed above)
        na.pin = soft ? pb[k & 1] : pb[k == 0 ? 0 : ((k - 1) & 1)];
        na.qout = q;
        na.qstride = qstride;
        na.tw = p->tw.at(g.H);
        na.mode = 1;
        na.iter = soft ? 0 : k;
        na.r = r;
        na.pout = soft ? nullptr : pb[k & 1];
        na.rr_cur = rr_cur;
        na.rr_prev = rr_prev;
        na.nrr = p->nrr;
        na.pq_part = pq;
        na.npq = p->npq;
        na.stopped = a.stopped;
        return soft ? g.soft->normal(na, g.W, sg) : g.col->normal(na, g.W, sg);
      });
    }
    if (e != hipSuccess) return hip_fail(e, "cg: normal operator");
    a.rr_cur = rr_cur;
    a.rr_next = rr_prev;  // rho_{k+1} overwrites rho_{k-1}
    a.p = pb[k & 1];
    {
      KernelTimer kt(p, MRX_KERNEL_CG_UPDATE, s);
      e = cg_update(a, s);
    }
    if (e != hipSuccess) return hip_fail(e, "cg: update");
  }
  if (hist) {
    a.rr_cur = rr[n_iter & 1];
    e = cg_hist(a, n_iter, n_iter + 1, s);
    if (e != hipSuccess) return hip_fail(e, "cg: history");
  }
  return MRX_OK;
}

}  // namespace mrx
