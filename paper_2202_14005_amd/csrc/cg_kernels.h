// Conjugate-gradient elementwise kernels (declarations).
#pragma once
#include "common.h"

namespace mrx {

constexpr int CG_THREADS = 256;
constexpr int CG_EPB = 512;   // elements per block and slice
constexpr int CG_QPARTS_MAX = 4;  // partial q planes k_cg_update adds (the normal operator's largest coil split)

// per-slice status bits (same values as the public MRX_FLAG_* macros)
constexpr uint32_t FLAG_NONFINITE = 1u;
constexpr uint32_t FLAG_CG_BREAKDOWN = 2u;
constexpr uint32_t FLAG_CNN_NONFINITE = 4u;
constexpr uint32_t FLAG_DC_JUDGE = 8u;

struct CgElemArgs {
  const SliceDesc* desc;
  const int* slices;
  int nslices;
  int nrr;               // blocks per slice (= partial count of rr buffers)
  int npq;               // partial count of the <p, q> buffer
  const float* lam;
  const float2* aHy;     // init: right-hand side part; bwd tail: forward x
  const float2* z;
  float2* x;             // bwd tail: the adjoint solution v
  float2* r;
  float2* p;
  const float2* q;       // q = sum of desc[b].nq partial planes, qstride apart
  int64_t qstride;
  const float* pq;       // [B][npq]
  float* pq_clear;       // cg_init: zero these [B][npq] partials first (or null)
  const float* rr_cur;   // [B][nrr]
  float* rr_next;        // [B][nrr]
  int* stopped;          // [B]
  uint32_t* status;      // [B]
  float* hist;
};

// p_out = r + beta p_in with beta = rho_k / rho_{k-1} from the rr partials
// (0 when rho_{k-1} = 0), for the slices of a.slices that have not stopped
// (a.p: p_in, a.x: p_out, a.rr_cur: rho_k, a.rr_next: rho_{k-1}).
hipError_t cg_form_p(const CgElemArgs& a, hipStream_t s);
hipError_t cg_init(const CgElemArgs& a, hipStream_t s);
hipError_t cg_update(const CgElemArgs& a, hipStream_t s);
hipError_t cg_hist(const CgElemArgs& a, int k, int stride, hipStream_t s);
hipError_t cg_bwd_tail(const CgElemArgs& a, float2* gz, float* part, hipStream_t s);
hipError_t slice_sum(const CgElemArgs& a, const float* part, float* out, int accumulate, hipStream_t s);

}  // namespace mrx
