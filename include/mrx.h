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
#define MRX_FLAG_DC_JUDGE 8u      /* mrx_dc_judge replaced the slice by CG-SENSE */

typedef struct mrx_plan_s* mrx_plan;

/* mrx_plan_create flags */
#define MRX_PLAN_NETWORK 1u /* also reserve workspace for the CNN / MoDL calls */
#define MRX_PLAN_VN 2u      /* also reserve workspace for the VarNet stage calls */
#define MRX_PLAN_SOFT_SENSE 4u /* two sets of coil maps (soft-SENSE); see mrx_soft_* */
#define MRX_PLAN_TOEPLITZ 8u   /* non-Cartesian sampling: normal operator by the PSF; see mrx_toeplitz_psf */
#define MRX_PLAN_BATCHNORM 16u /* denoiser with batch normalisation (needs MRX_PLAN_NETWORK); see mrx_cnn_set_bn */

/*
 * Parameters of one variational-network stage (device pointers): k = 24
 * complex 11 x 11 filters, interleaved [24][11][11][re, im]; w = RBF weights
 * [24][31]; lam = the stage's step size (1 float).
 */
typedef struct {
  const float* k;
  const float* w;
  const float* lam;
} mrx_vn_params;

/*
 * Denoiser parameters: fp32 master weights of the five 3x3 convolution
 * layers, w[l] laid out [C_out][C_in][3][3] (channels 2-64-64-64-64-2) and
 * biases b[l] [C_out], all device pointers owned by the caller.
 */
typedef struct {
  const float* w[5];
  const float* b[5];
} mrx_cnn_params;

/* Gradient buffers with the same shapes as mrx_cnn_params (fp32, device). */
typedef struct {
  float* w[5];
  float* b[5];
} mrx_cnn_grads;

/* Library version string and the last error of the calling thread. */
const char* mrx_version(void);
const char* mrx_last_error(void);

/*
 * Plan for a batch of B slices with per-slice matrix size H[b] x W[b] and
 * coil count C[b] (host arrays of B entries).  Requirements: H and W even,
 * each a length the library has a transform schedule for -- every even
 * length from 8 to 1024 that factors into 2, 3 and 5, except 450, 486, 750,
 * 810, 900 and 972, whose odd parts no tile of the transform engine fits
 * (see mrx_supported_length) -- and 1 <= C <= 64.  Creates device tables (shape table, twiddles) with hipMalloc
 * on the current device; this is the only allocating call.  A plan with
 * several matrix sizes also creates up to three auxiliary streams and their
 * events: the size groups of one normal-operator application run
 * concurrently on them, forked from and joined back into the caller's
 * stream (parallel branches when the stream is being captured).  Returns
 * MRX_EUNSUPPORTED for sizes without a schedule, MRX_EINVAL for bad counts.
 * flags: 0, or MRX_PLAN_NETWORK and/or MRX_PLAN_VN to size the workspace
 * for the MoDL network calls and the VarNet stage calls; MRX_PLAN_SOFT_SENSE
 * for two coil-map sets; MRX_PLAN_TOEPLITZ for non-Cartesian sampling (with
 * MRX_PLAN_NETWORK at most; every H and W must then also satisfy
 * mrx_toeplitz_supported).  The column
 * schedule of each size group comes from the in-process tuning cache
 * (filled by mrx_plan_autotune and mrx_tune_cache_load) when it holds an
 * entry for the group's (H, W, C, slice count), else the length's default;
 * the cache is process state rather than an argument of this call.
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
 * Allocation-free variant of mrx_cg_dc, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same solve with the same kernels,
 * bit-identical x and resid_hist, but the CG vectors and partial sums live
 * in a fixed device array of the library (64 MiB per GPU, held by every GPU
 * the library runs on until the process ends) instead of the plan's
 * workspace, which need not be set.  The call allocates nothing.
 * Requirements: the current device is the plan's device; the plan's CG
 * buffers, 8 n_image (3 + k) bytes plus per-slice partial sums (k = the
 * largest coil split of the plan's column schedules, 1..4), fit in 64 MiB
 * (about 13 slices of 320 x 320 with k = 3), else MRX_EINVAL, nothing
 * enqueued.  Every call on one GPU shares that GPU's array and overwrites
 * it: calls that overlap in time on one GPU (different streams, plans or
 * threads) race.  Status bits of this call (as mrx_status_word's: non-finite
 * scalar, CG breakdown) start at zero and are copied to dev_flags (device
 * uint32[B], NULL = skip); the plan's own status word is not touched.
 * The first call on a device takes the array's device address
 * (hipGetSymbolAddress), which may load the library's code object there.
 */
mrx_status mrx_cg_dc_noalloc(mrx_plan plan, const float* aHy, const float* z, const float* S,
                             const float* mask, const float* lambda, int32_t n_iter, float* x,
                             float* resid_hist, uint32_t* dev_flags, void* stream);

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

/*
 * Non-Cartesian SENSE (Extensions to the SENSE-Model subsection) on a plan
 * created with MRX_PLAN_TOEPLITZ.  The sampling of slice b is a trajectory
 * of M points (the same M for every slice), traj[(b M + j) 2 + {0, 1}] =
 * (ky_j, kx_j) in cycles per field of view (float, device); pixel (r, s) of
 * an H x W image sits at (r - H/2, s - W/2), and the forward model is the
 * non-uniform DFT
 *   y_{c,j} = (HW)^{-1/2} sum_{r,s} S_c[r,s] x[r,s] exp(-2 pi i (ky_j (r - H/2)/H + kx_j (s - W/2)/W)),
 * evaluated exactly (no gridding), which on the Cartesian grid is the
 * centred unitary DFT of the Cartesian calls.  k-space data y: [C][M]
 * complex per slice, slices packed in order.  These three calls are the
 * one-off steps the paper precomputes for a dataset; they run a sum over
 * all samples per pixel (or pixels per sample) in fp32 with each phase
 * formed in double precision, so they cost O(H W M C) and are not part of
 * the iterations.
 *
 * mrx_nufft_fwd: y = A x (+ noise, [C][M] per slice, or NULL).
 * mrx_nufft_adj: x = A^H y (the adjoint reconstruction).
 * mrx_toeplitz_psf: psf = the real 2H x 2W spectrum of the sampling's
 *   point spread function on the twice-padded grid, row-major [2H][2W] per
 *   slice at offset 4 x (the slice's image offset):
 *     psf[ky][kx] = (HW)^{-1} sum_j D_H(ky_j - ky/2) D_W(kx_j - kx/2),
 *     D_n(u) = sum_{|d| < n} exp(2 pi i d u / n),
 *   the unnormalised 2-D DFT of h[dy, dx] = (HW)^{-1} sum_j
 *   exp(2 pi i (ky_j dy / H + kx_j dx / W)) laid out cyclically (offset
 *   (dy, dx) at (dy mod 2H, dx mod 2W), zero on row H and column W).
 *
 * On a Toeplitz plan the operator calls take psf where the Cartesian calls
 * take the row mask: mrx_sense_normal, mrx_cg_dc, mrx_dc_judge,
 * mrx_modl_forward(_from) and mrx_modl_backward then use
 *   A^H A u = sum_c conj(S_c) crop(IDFT(psf * DFT(pad(S_c u)))),
 * (pad: u into the top-left H x W of a zero 2H x 2W grid, DFT the
 * unnormalised 2-D DFT, IDFT its inverse, crop the top-left H x W), the
 * Toeplitz form of the normal operator, in three passes per application
 * through a workspace buffer of 2 x (the coil-sized count) complex values.
 * mrx_sense_fwd / mrx_sense_adj, mrx_cg_dc_noalloc and the VarNet and
 * soft-SENSE calls return MRX_EINVAL on such a plan; mrx_plan_autotune does
 * nothing.  plan_create returns MRX_EUNSUPPORTED when 2H or 2W has no
 * Toeplitz decomposition (see mrx_toeplitz_supported).  Errors: MRX_EINVAL
 * for a null pointer or M outside [1, 2^26].
 */
mrx_status mrx_nufft_fwd(mrx_plan plan, const float* traj, int32_t M, const float* x, const float* S,
                         const float* noise, float* y, void* stream);
mrx_status mrx_nufft_adj(mrx_plan plan, const float* traj, int32_t M, const float* y, const float* S,
                         float* x, void* stream);
mrx_status mrx_toeplitz_psf(mrx_plan plan, const float* traj, int32_t M, float* psf, void* stream);
/* 1 if image side n has Toeplitz kernels (a decomposition of 2n with first
 * radix 2), else 0. */
int32_t mrx_toeplitz_supported(int32_t n);

/*
 * Soft-SENSE: the SENSE model with two sets of coil maps (Extensions to the
 * SENSE-Model subsection), for objects larger than the field of view:
 *   y_c = P F (S_{0,c} x_0 + S_{1,c} x_1),  (A^H y)_m = sum_c conj(S_{m,c}) F^H P^H y_c.
 * Needs a plan created with MRX_PLAN_SOFT_SENSE (not with MRX_PLAN_VN).
 * Layout per slice b: images [2][H][W] at 2 x (the SENSE image offset),
 * maps [2][C][H][W] at 2 x (the SENSE coil offset), k-space [C][H][W] and
 * mask as for SENSE; for an even batch x is [B][2][H][W] and S
 * [B][2][C][H][W].  The calls mirror mrx_sense_fwd / _adj / _normal and
 * mrx_cg_dc on these layouts (same arguments, same workspace and status
 * rules); the CG inner products run over both sets of a slice.  The column
 * transforms use each length's default decomposition.
 */
mrx_status mrx_soft_sense_fwd(mrx_plan plan, const float* x, const float* S, const float* mask,
                              const float* noise, float* y, void* stream);
mrx_status mrx_soft_sense_adj(mrx_plan plan, const float* y, const float* S, const float* mask,
                              float* x, void* stream);
mrx_status mrx_soft_sense_normal(mrx_plan plan, const float* x, const float* S, const float* mask,
                                 const float* lambda, float* out, void* stream);
mrx_status mrx_soft_cg_dc(mrx_plan plan, const float* aHy, const float* z, const float* S,
                          const float* mask, const float* lambda, int32_t n_iter, float* x,
                          float* resid_hist, void* stream);

/*
 * Fallback and judge for a learned reconstruction.  x_cg is the plain
 * Tikhonov CG-SENSE solution (mrx_cg_dc with z = NULL), the reconstruction
 * MoDL reduces to without its denoiser (eq. update_modl with lambda z = 0).
 * Per slice b, the data-consistency residual r(x) = ||A^H A x - aHy||_2 is
 * evaluated for x_net and x_cg; out[b] = x_cg[b] (and MRX_FLAG_DC_JUDGE is
 * raised, dev_choice[b] = 1) when x_net[b] has a non-finite entry, the slice
 * already carries MRX_FLAG_NONFINITE, _CG_BREAKDOWN or _CNN_NONFINITE, or
 * r(x_net) > ratio * r(x_cg); otherwise out[b] = x_net[b], dev_choice[b] = 0.
 * x_net, x_cg, aHy, out: packed images; out may alias x_net or x_cg (the
 * selection is element-wise, after both residuals).  dev_choice: device
 * uint32[B].  ratio > 0, else MRX_EINVAL.  Uses the workspace (its CG
 * buffers), so it must not overlap a CG call of the same plan.
 */
mrx_status mrx_dc_judge(mrx_plan plan, const float* x_net, const float* x_cg, const float* aHy,
                        const float* S, const float* mask, float ratio, float* out,
                        uint32_t* dev_choice, void* stream);

/* Copy the per-slice status words (uint32[B]) to dev_flags (device; NULL
 * skips the copy) and, if clear != 0, reset them.  Enqueued on stream, with a
 * copy and a fill kernel only, so it may be captured in a graph. */
mrx_status mrx_status_word(mrx_plan plan, uint32_t* dev_flags, int32_t clear, void* stream);

/*
 * MoDL residual denoiser D(x) = x + N(x) (MoDL subsection: a residual network
 * of L = 5 convolution layers with F = 64 channels and ReLU; batch
 * normalisation only on plans created with MRX_PLAN_BATCHNORM, see
 * mrx_cnn_set_bn).  N: 3x3 convolutions with zero "same" padding
 * and bias, ReLU after layers 1-4; the complex image enters as channels
 * (real, imag).  Convolutions run on bf16 MFMA with fp32 accumulation; the
 * layer activations are stored as bf16.  Needs a plan created with
 * MRX_PLAN_NETWORK.
 *
 * The weights are plan state, not arguments of the network calls
 * (mrx_cnn_forward/backward/layer_forward, mrx_modl_forward/backward):
 * mrx_cnn_set_weights packs bf16 copies of the five weight tensors into the
 * plan's workspace and keeps the five fp32 bias pointers.  Every later
 * network call on the plan uses those packed copies, so a weight update is
 * not seen until mrx_cnn_set_weights is called again (the Python binding
 * does so whenever the weights' version counter changed); the biases are
 * read through the kept pointers at each call, so they must stay valid and
 * in-place updates of them are seen at once.  Packing is enqueued on
 * `stream`: calls on other streams must be ordered after it.
 */
mrx_status mrx_cnn_set_weights(mrx_plan plan, const mrx_cnn_params* w, void* stream);

/*
 * Batch normalisation of the denoiser (the MoDL subsection's conv + BN +
 * ReLU layers), on a plan created with MRX_PLAN_BATCHNORM | MRX_PLAN_NETWORK:
 * each hidden layer l < 4 becomes
 *   y = conv(a, W_l)  (no bias: the layer's bias is not used and its
 *                      gradient is written as zero),
 *   a' = ReLU(gamma_l (y - mu) / sqrt(var + 1e-5) + beta_l),
 * with mu, var the mean and biased variance of y per channel over every
 * pixel of the plan's batch (the statistics of the batch being processed,
 * so the slices of a batch are coupled); the last layer is unchanged.  Every
 * network call (mrx_cnn_forward/backward, mrx_modl_forward(_from)/backward,
 * the soft-SENSE MoDL calls) then normalises each application of the
 * denoiser with its own batch's statistics, and the reverse calls also
 * write (or, with accumulate, add) g_gamma and g_beta.
 * gamma, beta: device float[4][64]; g_gamma, g_beta: device float[4][64] or
 * NULL (not computed).  Kept as pointers (plan state, like the biases): they
 * must stay valid; in-place updates are seen by the next call.  The
 * statistics are reduced in a fixed order (deterministic).  Returns
 * MRX_EINVAL on a plan without MRX_PLAN_BATCHNORM; network calls on such a
 * plan before this call return MRX_EINVAL.
 */
mrx_status mrx_cnn_set_bn(mrx_plan plan, const float* gamma, const float* beta, float* g_gamma, float* g_beta);
/* z = x + N(x) (image-sized complex, must not alias). */
mrx_status mrx_cnn_forward(mrx_plan plan, const float* x, float* z, void* stream);
/*
 * Reverse mode of D at x: recomputes the activations at x, then
 * gx = gz + J_N(x)^T gz and the weight/bias gradients (written to g, or added
 * to it if accumulate != 0).  gz in the DF^H(1) convention.
 */
mrx_status mrx_cnn_backward(mrx_plan plan, const float* x, const float* gz, float* gx,
                            const mrx_cnn_grads* g, int32_t accumulate, void* stream);

/*
 * One 64 -> 64 channel layer of the denoiser (layer = 1, 2 or 3): out =
 * ReLU(conv3x3(in, W[layer]) + b[layer]) on bf16 NHWC activations
 * (n_image x 64 bf16 values each, device).  For composing or timing single
 * layers; mrx_cnn_forward runs all five.
 */
mrx_status mrx_cnn_layer_forward(mrx_plan plan, int32_t layer, const void* in, void* out, void* stream);

/*
 * MoDL unrolled network, eq. update_modl with shared weights:
 *   x^0 = aHy,  x^{t+1} = (A^H A + lambda I)^{-1} (aHy + lambda D(x^t)),  t < T,
 * each inverse by n_cg CG steps (as mrx_cg_dc).  x_out receives x^T.
 * states: NULL or device buffer of (T + 1) image-sized arrays receiving
 * x^0 .. x^T (what mrx_modl_backward needs).
 */
mrx_status mrx_modl_forward(mrx_plan plan, const float* aHy, const float* S, const float* mask,
                            const float* lambda, int32_t T, int32_t n_cg, float* x_out,
                            float* states, void* stream);

/*
 * mrx_modl_forward from a given start image x^0 = x0 (image-sized, device)
 * instead of aHy: the non-Cartesian networks start from the SENSE
 * reconstruction x^0 = (A^H A + lambda I)^{-1} A^H y (Extensions to the
 * SENSE-Model subsection; mrx_cg_dc with z = NULL computes it).  states[0]
 * receives x0, so mrx_modl_backward applies unchanged to the weights and
 * lambda; its g_aHy then holds the gradient through the data-consistency
 * blocks plus the one reaching x^0 (the latter is the caller's to route
 * through its x0).  x0 may alias x_out.
 */
mrx_status mrx_modl_forward_from(mrx_plan plan, const float* x0, const float* aHy, const float* S,
                                 const float* mask, const float* lambda, int32_t T, int32_t n_cg,
                                 float* x_out, float* states, void* stream);

/*
 * Reverse mode of mrx_modl_forward from the stored states x^0..x^T: for
 * t = T-1 .. 0 the denoiser activations at x^t are recomputed, the data
 * consistency block is differentiated by a second CG solve
 * (v = (A^H A + lambda I)^{-1} g, g_z = lambda v, g_lambda += Re<v, z^t - x^{t+1}>)
 * and the denoiser by its reverse pass.  g_out: gradient w.r.t. x^T.
 * Weight gradients go to g (summed over the unrolls; added to g if
 * accumulate != 0).  g_lambda (device float[B]) and g_aHy (image-sized) may
 * be NULL.
 */
mrx_status mrx_modl_backward(mrx_plan plan, const float* g_out, const float* states, const float* aHy,
                             const float* S, const float* mask, const float* lambda, int32_t T,
                             int32_t n_cg, const mrx_cnn_grads* g, float* g_lambda, float* g_aHy,
                             int32_t accumulate, void* stream);

/*
 * MoDL with the soft-SENSE operator (two map sets, plan created with
 * MRX_PLAN_SOFT_SENSE | MRX_PLAN_NETWORK): as mrx_modl_forward/backward, but
 * the network block updates the first set's image only,
 *   z^t = (D(x_0^t), x_1^t),  x^{t+1} = (A^H A + lambda I)^{-1} (aHy + lambda z^t),
 * with images in the soft layout ([2][H][W] per slice) and the CG over both
 * sets; the reverse pass differentiates the soft CG blocks by a second soft
 * CG solve and the denoiser on the first set.  states: (T + 1) soft images.
 * Same weight, workspace and error rules as the SENSE calls.
 */
mrx_status mrx_soft_modl_forward(mrx_plan plan, const float* aHy, const float* S, const float* mask,
                                 const float* lambda, int32_t T, int32_t n_cg, float* x_out,
                                 float* states, void* stream);
mrx_status mrx_soft_modl_backward(mrx_plan plan, const float* g_out, const float* states,
                                  const float* aHy, const float* S, const float* mask,
                                  const float* lambda, int32_t T, int32_t n_cg,
                                  const mrx_cnn_grads* g, float* g_lambda, float* g_aHy,
                                  int32_t accumulate, void* stream);
/*
 * The training loss of the soft-SENSE networks: the MSE on the coil images
 * (they do not depend on how the map sets split the object),
 *   loss = mean over all coil pixels |S_{0,c} x_0 + S_{1,c} x_1 - ref_c|^2,
 *   g_m = sum_c conj(S_{m,c}) 2 (S_{0,c} x_0 + S_{1,c} x_1 - ref_c) / n_coil_pixels.
 * x, g: soft images; S: soft maps; ref: coil images (coil sized, the SENSE
 * k-space layout).  g and loss (device float[1]) may be NULL.
 */
mrx_status mrx_soft_coil_mse_grad(mrx_plan plan, const float* x, const float* S, const float* ref,
                                  float* g, float* loss, void* stream);

/*
 * MSE loss of eq. network_optimize over all packed pixels:
 *   loss = mean |x - ref|^2,  g = 2 (x - ref) / n_image  (DF^H(1) form).
 * g (image-sized) and loss (device float[1]) may be NULL.
 */
mrx_status mrx_mse_grad(mrx_plan plan, const float* x, const float* ref, float* g, float* loss,
                        void* stream);

/*
 * out[0] = sum of the n floats a[0..n) (+ out[0] if accumulate != 0), in a
 * fixed order; device pointers.  Reduces MoDL's per-slice lambda gradients
 * to the gradient of the one shared, trainable lambda.
 */
mrx_status mrx_sum_f32(const float* a, int32_t n, float* out, int32_t accumulate, void* stream);

/*
 * One Adam step (the training algorithm named in the Methods section) on n
 * fp32 parameters: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * w -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).  step >= 1.
 * All arrays are device arrays of n floats.
 */
mrx_status mrx_adam_step(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                         float b2, float eps, int32_t step, void* stream);

/*
 * One variational-network stage (Variational Network subsection, eq.
 * update_vn):
 *   x_next = x - sum_i K_i^T Phi'_i(Re(k_i * x)) - lambda (A^H A x - aHy)
 * with 24 complex 11 x 11 filters (cross-correlation, zero "same" padding),
 * Phi'_i(s) = sum_j w_ij exp(-(s - mu_j)^2 / (2 sigma^2)), 31 knots mu_j on
 * [-1, 1], sigma = the knot spacing.  fp32 throughout.  Needs a plan created
 * with MRX_PLAN_VN.  x, aHy, x_next image-sized complex; x_next must not
 * alias x.
 */
mrx_status mrx_vn_stage(mrx_plan plan, const float* x, const float* aHy, const float* S,
                        const float* mask, const mrx_vn_params* p, float* x_next, void* stream);
/*
 * Reverse mode of mrx_vn_stage at x with upstream gradient g:
 *   g_x = g - K^T(Phi''(Kx) * Kg) - lambda A^H A g,
 *   g_k (complex [24][11][11]), g_w ([24][31]) and g_lam (1 float) written,
 *   or added to if accumulate != 0.  Gradients in the DF^H(1) convention.
 */
mrx_status mrx_vn_stage_backward(mrx_plan plan, const float* g, const float* x, const float* aHy,
                                 const float* S, const float* mask, const mrx_vn_params* p,
                                 float* g_x, float* g_k, float* g_w, float* g_lam,
                                 int32_t accumulate, void* stream);

/*
 * iPALM, the training algorithm named for VarNet (Iterative Training
 * Algorithms; Variational Network subsection), on n fp32 parameters (complex
 * parameters as interleaved pairs).  Step k = 1, 2, ...: extrapolate
 *   y = theta + alpha (theta - theta_prev)          (alpha = (k - 1)/(k + 2)),
 * evaluate the loss gradient g at y, then
 *   theta_prev = theta;  theta = y - tau g          (mrx_ipalm_update),
 * and apply the proximal map, here mrx_vn_project.  All device arrays of n
 * floats; y may not alias theta or theta_prev.
 */
mrx_status mrx_ipalm_extrapolate(const float* theta, const float* theta_prev, float* y, int64_t n,
                                 float alpha, void* stream);
mrx_status mrx_ipalm_update(float* theta, float* theta_prev, const float* y, const float* g, int64_t n,
                            float tau, void* stream);
/*
 * The VarNet constraints as a projection: each of n_filters complex filters
 * of `taps` taps (interleaved, consecutive; taps <= 256) to zero mean and unit
 * Euclidean norm (a filter that is zero after removing its mean stays zero),
 * and each of n_lam step sizes to lambda >= 0.  In place on the device.
 */
mrx_status mrx_vn_project(float* k, int32_t n_filters, int32_t taps, float* lam, int32_t n_lam,
                          void* stream);
/*
 * The VarNet training option that scales the data so that max|x^0| = 1, per
 * slice: s_b = 1 / max_i |x_b[i]| (1 for an all-zero slice), x (image sized)
 * and, where not NULL, y (coil sized k-space) and ref (image sized) of slice
 * b multiplied by s_b in place; scale_out: device float[B] receives s_b.
 * Uses the workspace.
 */
mrx_status mrx_normalize_max(mrx_plan plan, float* x, float* y, float* ref, float* scale_out, void* stream);

/* Choose the fastest registered column schedule for each (H, W) group of the
 * plan by timing each on the given stream (synchronises the host): four CG
 * iterations over the plan when its workspace is set (scratch_a is the
 * right-hand side, scratch_b the solution; both image-sized and
 * overwritten), else, and for plans created with MRX_PLAN_VN, five
 * normal-operator applications of the group (scratch_a in, scratch_b out).  The
 * choice is kept in the plan and in an in-process cache keyed by (H, W, C,
 * number of slices of the group); plans created later with a matching group
 * start from the cached choice. */
mrx_status mrx_plan_autotune(mrx_plan plan, const float* S, const float* mask, float* scratch_a,
                             float* scratch_b, void* stream);
/* Kernel timing (measurement aid): with timing on, every launch of the
 * kernels below made through this plan on a stream that is not being
 * captured is bracketed by a pair of HIP events on that stream.
 * mrx_plan_kernel_timing(plan, enable) switches it on or off and drops the
 * records so far (the events are kept for reuse and freed with the plan).
 * mrx_plan_kernel_time synchronises with the recorded launches of kernel
 * `kid` and returns their summed duration in microseconds and their number.
 * Timing adds two event records to each timed launch. */
enum {
  MRX_KERNEL_NORMAL = 0,     /* normal operator (plain and CG-fused): one record per application,
                                spanning the launches of all size groups */
  MRX_KERNEL_CG_UPDATE = 1,  /* CG update of x, r and the residual partials */
  MRX_KERNEL_CONV_MID = 2,   /* 64 -> 64 denoiser layer (forward and input gradient) */
  MRX_KERNEL_WGRAD_MID = 3,  /* weight gradient of a 64 -> 64 layer */
  MRX_KERNEL_VN_FILTER = 4,  /* variational-network stage: filter responses + activation (forward) */
  MRX_KERNEL_VN_FILTER_REV = 5,  /* the same in the reverse pass (also K g and the activation's derivative) */
  MRX_KERNEL_VN_ADJOINT = 6, /* transposed filters + stage update (forward and reverse) */
  MRX_KERNEL_VN_KGRAD = 7,   /* filter gradients of a stage */
  MRX_KERNEL_COUNT = 8
};
mrx_status mrx_plan_kernel_timing(mrx_plan plan, int32_t enable);
mrx_status mrx_plan_kernel_time(mrx_plan plan, int32_t kid, double* total_us, int32_t* count);
/* Name of the schedule the plan uses for slice b's column transform. */
const char* mrx_plan_schedule(mrx_plan plan, int32_t b);
/* Name of the idx-th registered column schedule for length n, or NULL. */
const char* mrx_schedule_name(int32_t n, int32_t idx);
/* Force the column schedule `name` for the slices of the plan with H = n. */
mrx_status mrx_plan_set_schedule(mrx_plan plan, int32_t n, const char* name);
/* Write the in-process tuning cache to a text file, one "H W C slices name"
 * entry a line.  MRX_EINVAL if the file cannot be written. */
mrx_status mrx_tune_cache_save(const char* path);
/* Merge the entries of a file written by mrx_tune_cache_save into the
 * in-process cache; plans created afterwards use them.  Every entry is checked
 * first (known schedule for its H, positive W, C and slices): on a bad entry nothing is
 * merged and MRX_EINVAL names the line.  n_loaded (nullable) receives the
 * number of entries. */
mrx_status mrx_tune_cache_load(const char* path, int32_t* n_loaded);

#ifdef __cplusplus
}
#endif
#endif /* MRX_H */
