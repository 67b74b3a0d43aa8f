/*
 * dlx.h -- C ABI of the MI355X differentiable PSF library (libdlx.so).
 *
 * The library evaluates the forward model of Desdoigts et al., "Differentiable
 * optics with dLux I" (arXiv 2406.08703), and its gradient:
 *
 *   Section 3 (aperture listing): pupil OPD = sum_j c_j Z_j (+ an optional
 *     bicubic pixel-phase map B C B^T), on a grey transmission normalised to
 *     unit power;
 *   Section 3 (propagation paragraph): Fraunhofer propagation to an
 *     oversampled focal grid by a two-sided matrix Fourier transform, |E|^2
 *     summed over wavelengths and stars, binned to detector pixels, times the
 *     per-pixel response (flat field);
 *   Section 4: per-pixel Poisson log-likelihood plus a chi-squared prior on
 *     the pixel response, differentiated with respect to star positions,
 *     fluxes, Zernike coefficients and every pixel-response value.
 *
 * Conventions used throughout:
 *   - Every array argument is a DEVICE pointer owned by the caller, contiguous
 *     and row-major, unless marked "host".
 *   - Pupil arrays are [n_pupil][n_pupil] indexed [y][x]; detector arrays are
 *     [n_det][n_det] with n_det = n_focal / oversample; frames are outermost.
 *   - Grids are pixel-centred: sample i of an n-point grid of pitch p sits at
 *     (i - (n-1)/2) p. The pupil pitch is diameter / n_pupil; the focal pitch
 *     is focal_pixel_rad; a detector pixel is oversample focal pixels.
 *   - The MFT kernel is exp(-2 pi i x u / lambda); a star at angular offset
 *     (alpha, beta) tilts the pupil by exp(+2 pi i (x alpha + y beta)/lambda),
 *     placing its image at +alpha, +beta. The focal field carries the factor
 *     dx du / lambda, so that a full-period focal grid holds unit power.
 *   - Calls are asynchronous on the HIP stream passed in (NULL = default
 *     stream). A plan must not be used from two streams at once.
 *   - Argument and shape errors are returned synchronously before any launch.
 *     Conditions detected on the device (non-finite values; model <= 0 where
 *     the data are positive, which is clamped) set a status word in the plan,
 *     returned by dlx_plan_sync. The library never aborts the process.
 *   - forward, loss_grad and backward allocate nothing; the plan owns all
 *     workspaces, allocated once by dlx_plan_create.
 */
#ifndef DLX_H
#define DLX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DLX_OK = 0,
  DLX_ERR_INVALID_ARG = 1, /* null pointer, non-positive size, bad enum value */
  DLX_ERR_SHAPE = 2,       /* inconsistent sizes (n_focal % oversample != 0, ...) */
  DLX_ERR_OOM = 3,         /* workspace does not fit the device or the given limit */
  DLX_ERR_HIP = 4,         /* a HIP runtime call failed (no device, launch failure) */
  DLX_ERR_NONFINITE = 5,   /* device saw a NaN or Inf in the model or data */
  DLX_ERR_DOMAIN = 6,      /* model <= 0 where the Poisson loss needs m > 0 (clamped to 1e-30) */
  DLX_ERR_UNSUPPORTED = 7  /* valid request the library does not implement */
} dlx_status;

/* Arithmetic of the matrix Fourier transforms. DLX_FP32: FP32 MFMA with FP32
 * accumulation. DLX_BF16X3: each FP32 operand split as hi = bf16(x),
 * lo = bf16(x - hi); products hi*hi + hi*lo + lo*hi on BF16 MFMA, FP32
 * accumulation. DFT-matrix phases and tilt phases are always generated in
 * FP64; the loss and the flat-field gradient are always reduced in FP64. */
typedef enum { DLX_FP32 = 0, DLX_BF16X3 = 1 } dlx_precision;

/* Data term of the loss (Section 4). POISSON: m - d ln m (ln d! dropped).
 * CHI2: (m - d)^2 / (2 max(d, 1)). Both add the prior
 * sum_p (F_p - mu)^2 / (2 sigma^2) on the pixel response F. */
typedef enum { DLX_LOSS_POISSON = 0, DLX_LOSS_CHI2 = 1 } dlx_loss_kind;

/* One forward+gradient problem (the sizes of Section 3's optical system). */
typedef struct {
  int32_t n_pupil;       /* N_i: pupil samples per side, >= 2 */
  int32_t n_focal;       /* N_o: focal samples per side, multiple of oversample */
  int32_t oversample;    /* Q: focal samples per detector pixel per side, >= 1 */
  int32_t n_wavelengths; /* >= 1 */
  int32_t n_sources;     /* stars per frame, >= 1 */
  int32_t n_frames;      /* images (dithers), >= 1 */
  int32_t n_zernike;     /* basis terms, >= 0 */
  int32_t n_map;         /* bicubic map nodes per side, 0 = no map */
  double diameter_m;     /* D: pupil side length in metres, > 0 */
  double focal_pixel_rad;/* focal-grid pitch in radians, > 0 */
  const double* wavelengths_m;    /* host [n_wavelengths], each > 0 */
  const double* spectral_weights; /* host [n_wavelengths] */
  /* Integer-dither mode (the paper's own run, Section 3): NULL for frames
   * with independent sources. Otherwise host int32 [n_frames][2], the shift
   * (dx, dy) of the scene in each frame in whole detector pixels, with
   * |dx|, |dy| <= dither_margin. The frames then share one set of stars
   * (sources and grad_sources are [S][3]); every (star, wavelength) PSF is
   * computed once on an enlarged focal grid of Q (N_det + 2 dither_margin)
   * samples per side, and frame f is the N_det x N_det window of its binned
   * image whose pixel p is enlarged-plane pixel p + dither_margin - d_f.
   * The result equals independent frames with d_f added to every star's
   * position, at 1/n_frames of the propagation work. The array is copied at
   * plan creation. */
  const int32_t* frame_dithers;
  int32_t dither_margin;          /* >= 0; ignored when frame_dithers is NULL */
} dlx_problem_desc;

typedef struct dlx_plan dlx_plan;

/* Check a problem description without touching the device.
 * Returns DLX_OK, DLX_ERR_INVALID_ARG or DLX_ERR_SHAPE. */
dlx_status dlx_validate(const dlx_problem_desc* probs, int32_t n_probs);

/* Plan flags. By default dlx_plan_create autotunes: for each MFT stage it
 * times every compiled output-tile shape on the plan's own (zeroed)
 * workspace for the first frame chunk and keeps the fastest (for the last
 * adjoint product also its split of the contraction and the number of PSFs
 * each workgroup sums over).
 * DLX_FLAG_NO_AUTOTUNE keeps the built-in size heuristic instead. Tuned
 * tiles are kept per problem shape and device for the process; when the
 * environment variable DLX_TUNE_CACHE names a file, that file is the cache
 * instead (looked up at plan creation, one line appended per newly tuned
 * shape, naming the device by its architecture and compute-unit count), so
 * tuning carries across processes. Lines that do not parse, or whose tiles
 * are not compiled for their stage, are ignored.
 * The adjoint seed w phi G E is formed inside the first adjoint product's
 * operand loader; a plan with DLX_FLAG_DENSE_MFT forms it in a separate
 * elementwise pass instead when a frame's seed weights G exceed 4 MiB, and
 * DLX_FLAG_SEED_PASS forces the separate pass (same results, bit for bit). */
enum {
  DLX_FLAG_NO_AUTOTUNE = 1,
  DLX_FLAG_SEED_PASS = 2,
  DLX_FLAG_STORE_FIELDS = 4,
  DLX_FLAG_PIXEL_KERNEL = 8,
  DLX_FLAG_DENSE_MFT = 16,
  DLX_FLAG_GROUPED = 32
};

/* DLX_FLAG_GROUPED (plans of several problems): dlx_eval runs each stage as
 * ONE launch over every problem -- the OPD and tilts, the pupil fields, the
 * four MFT products, the binning with the loss, and the three final
 * reductions -- instead of each problem's own launch sequence on the plan's
 * concurrent streams. A device table maps every workgroup of a launch to its
 * problem and its tile; the per-problem arguments live in device memory, and
 * a call passes only its packed arrays' base pointers, so the launches
 * replay from a captured graph. The MFT tile of each stage (shared by all
 * problems) and B4's split and PSFs per group are tuned over the whole batch
 * at plan creation. It applies when every problem has one frame, no bicubic
 * map and no integer dithers, with the symmetric fold and without
 * DLX_FLAG_SEED_PASS, DLX_FLAG_STORE_FIELDS or DLX_FLAG_PIXEL_KERNEL, and to
 * calls without grad_intrapixel; otherwise the problems run on the streams.
 * dlx_psf_forward, dlx_loss_grad and dlx_psf_backward always run per problem.
 * Results equal the per-problem form's up to the order of partial sums in
 * the gradient reductions (the images are the same bits). */

/* The MFT products use the symmetry of the pixel-centred grids (Section 3's
 * coordinates are centred on the optical axis, so every sample x has a
 * partner -x): the DFT matrix equals its own conjugate under reversal of
 * either index, and each product is computed from the pair sums and
 * differences of its data over half the depth and half the output rows, a
 * quarter of the multiply-adds of the dense complex product, with the same
 * results up to rounding. DLX_FLAG_DENSE_MFT selects the dense products
 * instead (for comparison; same results up to rounding). */

/* DLX_FLAG_PIXEL_KERNEL gives every detector pixel its own intra-pixel kernel
 * (Section 6: intra-pixel sensitivity, recoverable at this sampling): every
 * `intrapixel` argument is then [Nd][Nd][Q][Q] (pixel p's kernel K_p[a][b])
 * and `grad_intrapixel` receives dL/dK_p[a][b] as [Nd][Nd][Q][Q] (FP64, Q <= 4),
 * the per-pixel terms of the shared kernel's gradient. Not available in
 * integer-dither mode (DLX_ERR_UNSUPPORTED at plan creation), where one
 * binned plane serves frames whose pixels see it through different windows. */

/* DLX_FLAG_STORE_FIELDS keeps the focal fields E of every PSF (and the
 * per-star binned images) in the plan from one dlx_psf_forward to the next
 * dlx_psf_backward, which then runs only the adjoint products: 2 MFTs per
 * PSF for a forward + backward pair instead of 3 (the choice between
 * recomputing and storing E). The whole problem is then one frame chunk:
 * the workspace holds every PSF's T, E and U^T (for 4096 PSFs of 768^2
 * focal samples from a 512^2 pupil, about 45 GB); without workspace_limit_bytes the plan
 * may use up to 80% of the free device memory, and DLX_ERR_OOM is returned
 * if the problem does not fit. The backward call must receive the same
 * parameter arrays, unchanged, as the forward call it follows; any other
 * call on the plan in between (dlx_eval, dlx_graph_launch, another
 * backward) discards the stored fields and the backward recomputes them. */

/* Create a plan: validates, picks kernel tiles, allocates every workspace on
 * the current device and builds the DFT matrices of each wavelength (FP64
 * phase; FP32, or bf16 hi/lo planes for DLX_BF16X3).
 * n_probs > 1 makes one plan for several independent problems (fits of
 * uneven size): every per-call array of dlx_psf_forward / dlx_loss_grad /
 * dlx_psf_backward / dlx_eval then packs the problems' arrays one after the
 * other, problem k starting at the element offsets dlx_plan_offsets reports
 * (loss_out holds one loss per problem). flags: an OR of DLX_FLAG_NO_AUTOTUNE,
 * DLX_FLAG_SEED_PASS, DLX_FLAG_STORE_FIELDS, DLX_FLAG_PIXEL_KERNEL,
 * DLX_FLAG_DENSE_MFT and DLX_FLAG_GROUPED (other bits: DLX_ERR_INVALID_ARG). Results do not depend on the tiles chosen
 * except for the order of FP32/FP64 partial sums in the gradient
 * reductions. workspace_limit_bytes: 0 = no limit;
 * otherwise the frame-chunk size is reduced until the workspace fits, and
 * DLX_ERR_OOM is returned if even one frame does not.
 * On success *out owns the device memory until dlx_plan_destroy. */
dlx_status dlx_plan_create(const dlx_problem_desc* probs, int32_t n_probs, dlx_precision precision,
                           int32_t flags, size_t workspace_limit_bytes, dlx_plan** out);

/* Free the plan and its device memory (synchronises the device first). NULL is a no-op. */
dlx_status dlx_plan_destroy(dlx_plan* plan);

/* Device bytes the plan holds. */
size_t dlx_plan_workspace_bytes(const dlx_plan* plan);

/* Element offsets of problem k's arrays in the packed arrays of a plan made
 * for several problems (all zero for k = 0). Sizes per problem:
 * transmission Ni^2, zernike_basis Nz Ni^2, map_basis Ni n_map,
 * zernike_coeffs / grad_zernike Nz, phase_map / grad_map n_map^2,
 * sources / grad_sources 3 F S (3 S in integer-dither mode), flat /
 * grad_flat Nd^2, intrapixel Q^2 (Nd^2 Q^2 with DLX_FLAG_PIXEL_KERNEL),
 * images (data, binned, model, dloss_dmodel) F Nd^2, loss 1. */
typedef struct {
  int64_t transmission, zernike_basis, map_basis, zernike_coeffs, phase_map, sources, flat, intrapixel, images,
      loss;
} dlx_offsets;
dlx_status dlx_plan_offsets(const dlx_plan* plan, int32_t problem, dlx_offsets* out);

/* Number of problems of the plan. */
int32_t dlx_plan_problems(const dlx_plan* plan);

/* Output-tile shape of each MFT stage (autotuned or heuristic): tiles[2k],
 * tiles[2k+1] = rows/32 and columns/32 of a workgroup's tile for stage
 * k = F1, F2, B3, B4 (host int32_t[8]). */
dlx_status dlx_plan_tiles(const dlx_plan* plan, int32_t* tiles);

/* Static pupil phase screen of one problem (Section 3, the optical layers: the
 * paper's system carries a fixed phase optic, the Toliman pupil's binary phase
 * plate, after the Zernike aperture). `screen` is a device array [Ni][Ni] of
 * phases in radians, row-major on the pupil grid, applied to every wavelength
 * (achromatic) on top of the OPD's 2 pi OPD / lambda; NULL clears it. The plan
 * copies the values on `stream` (the caller may free its array once the stream
 * has passed the copy); they hold for every later forward, backward and fused
 * call, including graph replays captured before or after. The screen is a fixed
 * input: no gradient is returned for it. Every plan starts with a zero screen.
 * `problem` is 0 for a one-problem plan. Errors: DLX_ERR_INVALID_ARG for a
 * null plan or a problem index out of range. */
dlx_status dlx_plan_set_phase_screen(dlx_plan* plan, int32_t problem, const float* screen, void* stream);

/* Synchronise `stream`, then return and clear the plan's device status word
 * (DLX_OK, DLX_ERR_NONFINITE or DLX_ERR_DOMAIN). */
dlx_status dlx_plan_sync(dlx_plan* plan, void* stream);

/* Forward model (Section 3).
 *   transmission [Ni][Ni]        grey pupil transmission A (>= 0)
 *   zernike_basis [Nz][Ni][Ni]   Z_j in metres of OPD per unit coefficient
 *   map_basis [Ni][n_map]        bicubic matrix B (NULL iff n_map == 0)
 *   zernike_coeffs [Nz]          c (metres)
 *   phase_map [n_map][n_map]     C (metres; NULL iff n_map == 0)
 *   sources [F][S][3]            per frame and star: alpha, beta (radians,
 *                                dither included), photons phi; [S][3] in
 *                                integer-dither mode (positions of frame 0)
 *   flat [Nd][Nd]                pixel response F
 *   intrapixel [Q][Q]            intra-pixel kernel K, NULL = all ones
 *                                ([Nd][Nd][Q][Q] with DLX_FLAG_PIXEL_KERNEL)
 * Outputs (may not alias inputs):
 *   binned_out [F][Nd][Nd]       B_f = bin_Q(K * sum_s sum_l w_l phi_s |E|^2)
 *   model_out  [F][Nd][Nd]       m_f = F * B_f */
dlx_status dlx_psf_forward(dlx_plan* plan, const float* transmission, const float* zernike_basis,
                           const float* map_basis, const float* zernike_coeffs, const float* phase_map,
                           const float* sources, const float* flat, const float* intrapixel,
                           float* binned_out, float* model_out, void* stream);

/* Loss, residual and flat-field gradient (Section 4), all reductions FP64.
 *   model, binned, data [F][Nd][Nd]; flat [Nd][Nd]; prior_sigma > 0.
 * Outputs:
 *   loss_out       device double[1]      L
 *   dloss_dmodel   [F][Nd][Nd] float     r = dL/dm
 *   grad_flat      [Nd][Nd] double       dL/dF_p = sum_f r_fp B_fp + (F_p - mu)/sigma^2 */
dlx_status dlx_loss_grad(dlx_plan* plan, const float* model, const float* binned, const float* data,
                         const float* flat, dlx_loss_kind kind, double prior_mu, double prior_sigma,
                         double* loss_out, float* dloss_dmodel, double* grad_flat, void* stream);

/* Largest frame, in pixels (n_det^2), that dlx_loss_grad_noalloc accepts. */
#define DLX_NOALLOC_MAX_PIXELS 4194304

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc: dlx_loss_grad
 * without a plan. Arguments, outputs and arithmetic are those of
 * dlx_loss_grad for n_frames images of n_det x n_det pixels (the same
 * kernels: the results equal, bit for bit, dlx_loss_grad's on a plan of that
 * many frames and pixels), with n_det^2 <= DLX_NOALLOC_MAX_PIXELS.
 * It allocates nothing. Its FP64 per-block loss partials and its status word
 * sit in a fixed library array of 128 KiB + 256 B on each device it runs on,
 * held until the process ends; every call on a device shares that device's
 * array, so calls that overlap on one device (two streams or two threads)
 * race and must be serialised by the caller. The status word is left zero by
 * every call.
 *   status_out  device int32[1] receiving this call's device flags, or NULL:
 *               0, or bit 0 (a non-finite model or data value,
 *               DLX_ERR_NONFINITE) | bit 1 (model <= 0 where the Poisson loss
 *               needs m > 0, clamped to 1e-30: DLX_ERR_DOMAIN).
 * Asynchronous on `stream`, which must belong to the current device.
 * Errors, returned before any device work: DLX_ERR_INVALID_ARG (a null
 * pointer other than status_out, n_frames or n_det < 1, a bad loss kind or
 * prior), DLX_ERR_UNSUPPORTED (n_det^2 > DLX_NOALLOC_MAX_PIXELS); DLX_ERR_HIP
 * if a launch fails. */
dlx_status dlx_loss_grad_noalloc(int32_t n_frames, int32_t n_det, const float* model, const float* binned,
                                 const float* data, const float* flat, dlx_loss_kind kind, double prior_mu,
                                 double prior_sigma, double* loss_out, float* dloss_dmodel, double* grad_flat,
                                 int32_t* status_out, void* stream);

/* Gradient through the optics given r = dL/dm (Sections 3-4). The inputs are
 * those of dlx_psf_forward; the focal fields are recomputed (one chunk of
 * frames at a time in the plan's workspace), unless the plan was created with
 * DLX_FLAG_STORE_FIELDS and this call directly follows dlx_psf_forward with
 * the same inputs, in which case that call's fields are used.
 * Outputs (double, FP64-reduced):
 *   grad_zernike [Nz]              dL/dc
 *   grad_map [n_map][n_map]        dL/dC (NULL iff n_map == 0)
 *   grad_sources [F][S][3]         dL/dalpha, dL/dbeta, dL/dphi per frame and star
 *                                  ([S][3], summed over frames, in integer-dither mode)
 *   grad_intrapixel [Q][Q]         dL/dK of the intra-pixel kernel, [Nd][Nd][Q][Q] with
 *                                  DLX_FLAG_PIXEL_KERNEL (fitting it is the
 *                                  extension Section 6 proposes); NULL = not computed.
 *                                  Needs Q <= 4 (else DLX_ERR_UNSUPPORTED). */
dlx_status dlx_psf_backward(dlx_plan* plan, const float* transmission, const float* zernike_basis,
                            const float* map_basis, const float* zernike_coeffs, const float* phase_map,
                            const float* sources, const float* flat, const float* intrapixel,
                            const float* dloss_dmodel, double* grad_zernike, double* grad_map,
                            double* grad_sources, double* grad_intrapixel, void* stream);

/* Every pointer of one full evaluation (forward, loss, backward); the
 * meanings, shapes and NULL rules are those of dlx_psf_forward,
 * dlx_loss_grad and dlx_psf_backward. */
typedef struct {
  const float* transmission;
  const float* zernike_basis;
  const float* map_basis;
  const float* zernike_coeffs;
  const float* phase_map;
  const float* sources;
  const float* flat;
  const float* intrapixel;
  const float* data;
  dlx_loss_kind loss_kind;
  double prior_mu;
  double prior_sigma;
  float* binned;        /* [F][Nd][Nd] */
  float* model;         /* [F][Nd][Nd] */
  float* dloss_dmodel;  /* [F][Nd][Nd] */
  double* loss;         /* [1] */
  double* grad_flat;    /* [Nd][Nd] */
  double* grad_zernike; /* [Nz] */
  double* grad_map;     /* [n_map][n_map] */
  double* grad_sources; /* [F][S][3] */
  double* grad_intrapixel; /* [Q][Q], NULL = not computed */
} dlx_eval_args;

/* Value and gradient of Section 4's objective in one call: dlx_psf_forward,
 * dlx_loss_grad and dlx_psf_backward enqueued on `stream`. */
dlx_status dlx_eval(dlx_plan* plan, const dlx_eval_args* args, void* stream);

/* Record dlx_eval with these pointers into a HIP graph owned by the plan
 * (replacing any earlier one). Nothing runs; the pointers must stay valid
 * while the graph is used. Capture happens on a plan-owned stream. */
dlx_status dlx_graph_capture(dlx_plan* plan, const dlx_eval_args* args);

/* Replay the captured evaluation on `stream` (DLX_ERR_INVALID_ARG if none). */
dlx_status dlx_graph_launch(dlx_plan* plan, void* stream);

/* Stages of one evaluation, for per-stage timing. PREP builds the OPD, the
 * pupil field and the tilt vectors; F1/F2 are the two MFT products of the
 * forward pass (F2 stores the focal fields E); BIN forms the intensity, the
 * intra-pixel weighting and the binning (per source, and the model with the
 * flat); LOSS is the loss and residual (in dlx_eval also the adjoint seed
 * weights G = K flat r and the flux-gradient partials); SEED forms those in
 * dlx_psf_backward, and the separate seed pass w phi G E where it runs; B3/B4 are the two
 * adjoint MFT products (B3 forms w phi G E in its loader, B4 has the
 * phase-gradient epilogue); GRAD reduces dL/dOPD and projects it onto the
 * Zernike basis, the map, positions and fluxes. */
typedef enum {
  DLX_STAGE_PREP = 0, DLX_STAGE_F1, DLX_STAGE_F2, DLX_STAGE_BIN, DLX_STAGE_LOSS,
  DLX_STAGE_SEED, DLX_STAGE_B3, DLX_STAGE_B4, DLX_STAGE_GRAD, DLX_N_STAGES
} dlx_stage;

/* Diagnostics: while enabled (enable != 0), each stage launch is bracketed
 * by HIP events recorded on the stream of the call, adding a few event
 * records per stage. Disabling discards pending records. */
dlx_status dlx_plan_profile(dlx_plan* plan, int32_t enable);

/* Diagnostics: synchronise on the recorded events and return, per stage
 * (arrays of DLX_N_STAGES, host memory), the summed device time in ms, the
 * number of launches and the number of PSFs those launches processed since
 * profiling was enabled or these counters were last read; then reset them. */
dlx_status dlx_plan_stage_times(dlx_plan* plan, double* total_ms, int64_t* launches, int64_t* psfs);

/* Static string naming a status code. */
const char* dlx_status_string(dlx_status status);

#ifdef __cplusplus
}
#endif

#endif /* DLX_H */
