/*
 * mrx -- MI355X (gfx950) HIP library for the hot path of unrolled MRI
 * reconstruction networks (arXiv 2202.14005, "Deep, Deep Learning with BART"):
 * the multi-coil SENSE operator A = P F C, its normal operator inside a
 * conjugate-gradient data-consistency solve, the MoDL residual CNN denoiser
 * and the variational-network stage.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Complex data are interleaved float pairs (re, im) -- the memory layout of
 *   torch.complex64 -- passed as `float*` pointing at the first real part.
 * - Row-major images: a slice of H x W has the readout W contiguous and the
 *   phase-encode index h along H.  Packed batch layout, slice b at:
 *     image-sized buffers   x, p, q, z, ...   offset sum_{b'<b} H W
 *     coil-sized buffers    S, y              offset sum_{b'<b} C H W
 *       (coil c of slice b is the H x W plane at offset + c H W)
 *     masks                 mask              offset sum_{b'<b} H
 *   For an even batch this is simply [B, H, W], [B, C, H, W] and [B, H].
 * - mask[h] in {0, 1} marks sampled phase-encode lines (constant along W);
 *   P^H P = diag(mask) requires binary values.
 * - F is the centered unitary 2-D DFT (DC at (H/2, W/2)).
 * - lambda arguments are DEVICE pointers to one float per slice.
 * - All data pointers are device pointers owned by the caller; the library
 *   never frees them.  Calls enqueue work on `stream` (a hipStream_t passed
 *   as void*, NULL = default stream) and never synchronise the host, except
 *   where stated.  Inputs must not alias outputs unless stated.
 * - Errors: every call returns mrx_status.  Argument problems are detected
 *   on the host before anything is enqueued; mrx_last_error() then returns a
 *   thread-local description.  Numeric problems found on the device (non
 *   finite values, CG breakdown) set per-slice bits of the plan's status
 *   word, read with mrx_status_word().
 */
#ifndef MRX_H
#define MRX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MRX_OK = 0,
  MRX_EINVAL = -1,       /* bad argument (null pointer, bad size, ...) */
  MRX_EUNSUPPORTED = -2, /* size the library has no schedule for */
  MRX_ENOMEM = -3,       /* plan tables could not be allocated */
  MRX_EHIP = -4,         /* a HIP runtime call failed */
  MRX_ENOWORKSPACE = -5  /* operation needs a workspace that is not set */
} mrx_status;

/* Per-slice status bits (mrx_status_word). */
#define MRX_FLAG_NONFINITE 1u     /* non-finite CG scalar (NaN/Inf input) */
#define MRX_FLAG_CG_BREAKDOWN 2u  /* Re<p, S p> <= 0 with rho > 0 */
#define MRX_FLAG_CNN_NONFINITE 4u /* non-finite denoiser output */
#define MRX_FLAG_DC_JUDGE 8u      /* reserved */

typedef struct mrx_plan_s* mrx_plan;

/* Library version string and the last error of the calling thread. */
const char* mrx_version(void);
const char* mrx_last_error(void);

/*
 * Plan for a batch of B slices with per-slice matrix size H[b] x W[b] and
 * coil count C[b] (host arrays of B entries).  Requirements: H and W even,
 * each a length the library has a transform schedule for (products of
 * 2, 3 and 5 between 16 and 512 from the built list, see mrx_supported_length),
 * 1 <= C <= 64.  Creates device tables (shape table, twiddles) with hipMalloc
 * on the current device; this is the only allocating call.  Returns
 * MRX_EUNSUPPORTED for sizes without a schedule, MRX_EINVAL for bad counts.
 * flags: reserved, pass 0.
 */
mrx_status mrx_plan_create(mrx_plan* plan, int32_t B, const int32_t* H, const int32_t* W,
                           const int32_t* C, uint32_t flags);
void mrx_plan_destroy(mrx_plan plan);

/* Total element counts of the packed buffers: image-sized (sum H W),
 * coil-sized (sum C H W) and mask (sum H). */
mrx_status mrx_plan_sizes(mrx_plan plan, int64_t* n_image, int64_t* n_coil, int64_t* n_mask);

/* Bytes of device workspace needed by the operators (caller allocates). */
size_t mrx_plan_workspace_bytes(mrx_plan plan);
/* Lend a workspace of at least mrx_plan_workspace_bytes() bytes, 256-byte
 * aligned.  The plan borrows it until the next call or destruction.  Calls
 * that share one plan must not overlap in time on different streams. */
mrx_status mrx_plan_set_workspace(mrx_plan plan, void* dev_ptr, size_t bytes);

/* 1 if the library holds a transform schedule for length n, else 0. */
int32_t mrx_supported_length(int32_t n);

/*
 * Forward SENSE operator (the paper's A = P F C, Applications section):
 *   y_c = mask * (F(S_c x) + noise_c)
 * x: image-sized complex, S: coil-sized complex, mask: per slice rows,
 * noise: coil-sized complex or NULL (the Results section's training-data
 * recipe adds Gaussian noise before subsampling), y: coil-sized complex
 * output; unsampled rows are written as zeros.  No workspace needed.
 */
mrx_status mrx_sense_fwd(mrx_plan plan, const float* x, const float* S, const float* mask,
                         const float* noise, float* y, void* stream);

/*
 * Adjoint SENSE operator A^H (the adjoint reconstruction x0 = A^H y that
 * initialises MoDL and VarNet):  x = sum_c conj(S_c) F^H (mask * y_c).
 * Uses the workspace for the row-transformed k-space.
 */
mrx_status mrx_sense_adj(mrx_plan plan, const float* y, const float* S, const float* mask,
                         float* x, void* stream);

/*
 * Normal operator (A^H A + lambda I) x, the operator inverted inside the
 * MoDL data-consistency block (eq. update_modl) and applied in each VarNet
 * gradient step (eq. update_vn).  lambda: device float[B] or NULL (= 0).
 * One pass over the coil maps; no workspace needed.
 */
mrx_status mrx_sense_normal(mrx_plan plan, const float* x, const float* S, const float* mask,
                            const float* lambda, float* out, void* stream);

/*
 * Data-consistency solve of eq. update_modl:
 *   x = (A^H A + lambda I)^{-1} (aHy + lambda z)
 * by n_iter conjugate-gradient steps from x0 = 0 (fixed count, no tolerance
 * stop; a slice stops early only on breakdown, setting a status bit).
 * z: image-sized complex or NULL (= 0: plain Tikhonov CG-SENSE).
 * resid_hist: NULL or device float[B * (n_iter + 1)] receiving ||r_k||^2.
 * Uses the workspace.  x is written.
 */
mrx_status mrx_cg_dc(mrx_plan plan, const float* aHy, const float* z, const float* S,
                     const float* mask, const float* lambda, int32_t n_iter, float* x,
                     float* resid_hist, void* stream);

/*
 * Reverse-mode pass of mrx_cg_dc (derivatives of the inversion operator
 * S^{-1}: D_y S^{-1} = S^{-1}, D_lambda S^{-1} = -S^{-1} D_lambda S), with the
 * inverse applied by the same CG recipe:
 *   v = (A^H A + lambda I)^{-1} gx,  g_aHy = v,  g_z = lambda v,
 *   g_lambda[b] = Re<v, z - x>  (accumulated into g_lambda if accumulate != 0)
 * gx: upstream gradient (real part = d/dRe, imaginary = d/dIm), x: forward
 * result, z: as in the forward call (NULL = 0).  g_aHy (required), g_z and
 * g_lambda (device float[B]) may be NULL to skip.  Uses the workspace.
 */
mrx_status mrx_cg_dc_backward(mrx_plan plan, const float* gx, const float* x, const float* z,
                              const float* S, const float* mask, const float* lambda,
                              int32_t n_iter, float* g_aHy, float* g_z, float* g_lambda,
                              int32_t accumulate, void* stream);

/* Copy the per-slice status words (uint32[B]) to dev_flags (device) and, if
 * clear != 0, reset them.  Enqueued on stream. */
mrx_status mrx_status_word(mrx_plan plan, uint32_t* dev_flags, int32_t clear, void* stream);

/* Choose the fastest registered schedule per distinct length of the plan by
 * timing each on the given stream (synchronises the host).  The choice is
 * kept in the plan and in an in-process cache keyed by (H, W, C). */
mrx_status mrx_plan_autotune(mrx_plan plan, const float* S, const float* mask, float* scratch_a,
                             float* scratch_b, void* stream);
/* Name of the schedule the plan uses for slice b's column transform. */
const char* mrx_plan_schedule(mrx_plan plan, int32_t b);

#ifdef __cplusplus
}
#endif
#endif /* MRX_H */
