// SENSE operator kernels for one FFT schedule (template), plus the argument
// structs and the registry through which the host picks a schedule.
//
// The SENSE model A = P F C (coil multiply, centered unitary 2-D DFT, row
// sampling) and its adjoint are computed in two passes (a column pass doing
// the transform along H and a row pass doing the transform along W).  The
// normal operator A^H A needs only the column pass: with a row mask m[h]
// constant along W, F^H P^H P F = F_H^H diag(m) F_H because the unitary
// W-transforms cancel, and the centering shifts reduce to evaluating the mask
// at (j + H/2) mod H for the uncentered frequency j.
#pragma once
#include "common.h"

namespace mrx {

struct NormalArgs {
  const SliceDesc* desc;   // all slices of the plan
  const int* slices;       // slices handled by this launch (nslices of them)
  int nslices;
  const float2* S;         // packed coil maps
  const float* mask;       // packed row masks
  const float* lam;        // per-slice lambda (device), may be null (= 0)
  const float2* pin;       // operand (image sized)
  float2* qout;            // result (image sized)
  const float2* tw;        // exp(-2 pi i j / H), j < H
  // Fused CG step (mode 1): before the operator, p = r + beta p with
  // beta = rho_k / rho_{k-1} summed from the rr partial buffers; p is written
  // back to pout and the partial sums of Re<p, q> go to pq_part.
  int mode;
  int iter;
  const float2* r;
  float2* pout;
  const float* rr_cur;     // [B][nrr] partials of rho_k
  const float* rr_prev;    // [B][nrr] partials of rho_{k-1}
  int nrr;
  float* pq_part;          // [B][npq]
  int npq;
  const int* stopped;      // [B] per-slice stop flag (CG breakdown)
  int tiles;               // column tiles per slice (set by the launcher)
  int64_t qstride;         // distance between the partial output planes (CG mode, or split_plain)
  // Operator application (mode 0) split like a CG step: a column tile's
  // coils over the schedule's KSPL workgroups, each writing its partial
  // plane at qout + k qstride (the first adds lambda p); the caller adds them.
  int split_plain;
};

struct SenseColArgs {
  const SliceDesc* desc;
  const int* slices;
  int nslices;
  const float2* S;
  const float* mask;
  const float2* in;        // fwd: image x; adj: row-pass output (coil sized)
  float2* out;             // fwd: coil-sized k-space rows; adj: image
  const float2* tw;
  int tiles;               // column tiles per slice (set by the launcher)
};

struct SenseRowArgs {
  const SliceDesc* desc;
  const int* slices;
  int nslices;
  const float* mask;
  const float2* in;        // coil sized
  float2* out;             // coil sized (may alias in for the forward pass)
  const float2* noise;     // optional additive noise on sampled rows (forward)
  const float2* tw;        // exp(-2 pi i j / W), j < W
};

using NormalFn = hipError_t (*)(const NormalArgs&, int maxW, hipStream_t);
using ColFn = hipError_t (*)(const SenseColArgs&, int maxW, hipStream_t);
using RowFn = hipError_t (*)(const SenseRowArgs&, int maxH, int maxC, hipStream_t);

struct ColVariant {
  int N, N1, N2, N3, T, WT;
  NormalFn normal;
  ColFn fwd_col;
  ColFn adj_col;
  const char* name;
  int kspl = 1;  // CG mode: workgroups per column tile (coil split), partial planes written
};
constexpr int KSPL_MAX = 4;
constexpr int SOFT_KSPL = 3;  // soft-SENSE CG steps: workgroups per column tile (coil split)
struct RowVariant {
  int N, N1, N2, N3, T, WT;
  RowFn fwd_row;
  RowFn adj_row;
  const char* name;
};

// Soft-SENSE (two coil-map sets) kernels of one length: the fused normal
// operator and the column passes; the row passes are the SENSE ones.
struct SoftVariant {
  int N;
  NormalFn normal;
  ColFn fwd_col;
  ColFn adj_col;
  const char* name;
};

// Toeplitz normal operator of non-Cartesian SENSE (kernels in toeplitz.h):
// arguments of its three passes and the kernels of one padded length.
struct ToepArgs {
  const SliceDesc* desc;
  const int* slices;
  int nslices;
  const float2* S;     // coil maps (SENSE layout)
  const float* psf;    // real [2H][2W] per slice at 4 xoff
  const float* lam;    // per-slice lambda or null
  const float2* pin;   // operand
  float2* qout;        // result (partial planes qstride apart in CG steps)
  int64_t qstride;
  float2* tbuf;        // [C][H][2W] per slice at 2 soff
  const float2* tw;    // exp(-2 pi i j / N) for the kernel's length N
  int split;           // coil groups (first two passes) / output planes (last)
  // CG step (mode 1): as NormalArgs
  int mode, iter;
  const float2* r;
  float2* pout;
  const float* rr_cur;
  const float* rr_prev;
  int nrr;
  float* pq_part;
  int npq;
  const int* stopped;
};

using ToepFn = hipError_t (*)(const ToepArgs&, int maxdim, hipStream_t);

struct ToepVariant {
  int N;             // transform length (twice an image side)
  ToepFn rows_fwd;   // first pass (N = 2W)
  ToepFn cols;       // middle pass (N = 2H)
  ToepFn rows_adj;   // last pass (N = 2W)
  int rows_wt;       // rows per workgroup of the row passes
  int cols_wt;       // columns per workgroup of the column pass
  const char* name;
};
void register_toep_variant(const ToepVariant& v);

void register_col_variant(const ColVariant& v);
void register_row_variant(const RowVariant& v);
void register_soft_variant(const SoftVariant& v);

}  // namespace mrx
