/*
 * combgpu.h -- C ABI of the MI355X (gfx950) comb-spectroscopy hot path.
 *
 * Method (paper, "Data Capture and Processing"): raw integer digitizer samples
 * are cast to floating point, cut into frames of consecutive samples, each
 * frame is Fourier transformed, the bins of the comb teeth are picked out in
 * optical order, each spectrum is divided by an averaged reference spectrum,
 * a 7x7 median filter over the (frame, tooth) image gives the starting centre,
 * and a Levenberg-Marquardt fit of the cavity resonance returns its centre
 * (the proof-mass displacement proxy) per frame.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns a cg_status; nothing throws or aborts across the
 *   ABI.  CG_ERR_HIP carries a thread-local detail string, see
 *   cg_last_error_detail().
 * - "device" pointers are HIP device allocations (e.g. torch tensors on the
 *   GPU); "host" pointers are ordinary CPU memory.  The caller owns every
 *   buffer it passes in and keeps device buffers alive until the stream work
 *   has completed.
 * - `stream` is a hipStream_t passed as void*; NULL is HIP's null (default)
 *   stream.  Work is only enqueued on that stream: the call returns before the
 *   GPU finishes, and stream order is the only ordering with the caller's work.
 * - Arrays are row-major and contiguous: frames [n_frames][frame_len] of the
 *   plan's sample type (int16, or int8 for a plan made with
 *   CG_SAMPLES_INT8), passed as void*;
 *   spectra float32 [n_frames][n_teeth]; parameters float32 [n_frames][4] in
 *   the order (centre, width, depth, baseline).
 * - Centre and width are in units of the tooth index (0 .. n_teeth-1, optical
 *   order); width is the full width at half depth of the Lorentzian dip
 *   y(x) = baseline * (1 - depth / (1 + (2 (x - centre) / width)^2)).
 * - n_frames == 0 is a no-op returning CG_OK; n_frames < 0 is
 *   CG_ERR_INVALID_ARG.
 * - A plan may be used from one host thread at a time.
 */
#ifndef COMBGPU_H
#define COMBGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cg_plan cg_plan;
typedef int32_t cg_status;

/* Return codes. */
#define CG_OK               0
#define CG_ERR_INVALID_ARG (-1) /* a size, count or flag is out of range        */
#define CG_ERR_UNSUPPORTED (-2) /* frame_len or n_teeth outside what is built   */
#define CG_ERR_BAD_REF     (-3) /* reference spectrum not finite and > 0        */
#define CG_ERR_NULL        (-4) /* a required pointer is NULL                   */
#define CG_ERR_OOM         (-5) /* device allocation failed                     */
#define CG_ERR_HIP         (-6) /* HIP runtime / launch error (see detail)      */
#define CG_ERR_WORKSPACE   (-7) /* caller workspace smaller than required       */
#define CG_ERR_STATE       (-8) /* operation needs state the plan lacks         */
#define CG_ERR_RING_FULL   (-9) /* pipeline: no free slot; the burst was not taken */

/* Per-frame fit status written to out_status. */
#define CG_FIT_CONVERGED 0 /* accepted step lowered chi2 by <= 1e-6 chi2        */
#define CG_FIT_MAX_ITER  1 /* iteration cap reached; last accepted point kept  */
#define CG_FIT_SINGULAR  2 /* damped normal matrix not positive definite       */
#define CG_FIT_FALLBACK  3 /* warm start rejected, cold-start fit used         */

/* Flags of cg_process_batch_ex: one DFT form ... */
#define CG_DFT_FFT         0x0u /* FP32 real FFT (default)                       */
#define CG_DFT_MFMA_BF16X3 0x1u /* tooth DFT on BF16 MFMA, hi/lo split, 3 terms  */
#define CG_DFT_MFMA_FP16   0x2u /* tooth DFT on FP16 MFMA, one term              */
#define CG_DFT_MFMA_FP16X2 0x3u /* tooth DFT on FP16 MFMA, split samples, 2 terms*/
#define CG_DFT_MASK        0xFu
/* ... and one start-point form. */
#define CG_FIT_COLD      0x00u /* 7x7 median start point, full LM (default)     */
#define CG_FIT_WARM_MLP  0x10u /* learned warm start + 2-iteration polish       */
#define CG_FIT_NONE      0x20u /* stop after the normalised spectra             */
#define CG_FIT_FANO      0x30u /* the paper's boxed Fano fit (cg_set_fano)      */
#define CG_FIT_MASK      0xF0u

/* Supported sizes. */
#define CG_MIN_FRAME_LEN 512
#define CG_MAX_FRAME_LEN 8192
#define CG_PAPER_FRAME_LEN 2200 /* the paper's rows: 1 us at 2.2 GS/s          */

/* Sample types of cg_create_plan_ex. */
#define CG_SAMPLES_INT16 0
#define CG_SAMPLES_INT8  1 /* the paper's 8-bit digitiser samples            */
#define CG_MAX_TEETH     440
#define CG_MAX_ITER      64

/*
 * Create a plan for frames of `frame_len` int16 samples (a power of two in
 * 512..8192, or 2200) and `n_teeth` comb teeth (1..min(440, frame_len/2+1)).
 *   fs            sample rate in Hz (> 0, finite); metadata only: bin k is
 *                 k*fs/frame_len Hz and frame f starts at f*frame_len/fs s.
 *   tooth_bins    host int32[n_teeth]: DFT bin of each tooth in optical
 *                 order; each in [0, frame_len/2], all distinct.
 *   ref_spectrum  host float32[n_teeth]: averaged reference amplitudes in the
 *                 units of |X[k]| of the unnormalised forward DFT of the raw
 *                 int16 frame; finite and > 0 (paper: average reference
 *                 spectrum recorded at the start of the experiment).
 *   out_plan      receives the plan; set to NULL on failure.
 * Arguments are validated on the host before any HIP call.  The plan owns its
 * device tables (bins, reference, twiddles) and a workspace; release it with
 * cg_destroy_plan.
 * Errors: CG_ERR_NULL, CG_ERR_UNSUPPORTED, CG_ERR_INVALID_ARG, CG_ERR_BAD_REF,
 * CG_ERR_OOM, CG_ERR_HIP.
 */
cg_status cg_create_plan(int32_t frame_len, double fs, const int32_t* tooth_bins,
                         int32_t n_teeth, const float* ref_spectrum, cg_plan** out_plan);

/*
 * As cg_create_plan for frames of `sample_type` samples (paper, Data Capture
 * and Processing: 8-bit integer samples cast to single precision on the GPU,
 * rows of 2200 samples = 1 us at 2.2 GS/s).  frame_len is a power of two in
 * 512..8192 for CG_SAMPLES_INT16, or CG_PAPER_FRAME_LEN (2200) for either
 * type; 2200-sample frames go through a mixed-radix (4, 5, 5, 11) FFT of
 * 1100 complex points.  The matrix-core DFT forms take int16 frames of a
 * power-of-two length only (CG_ERR_UNSUPPORTED otherwise).  Errors as for
 * cg_create_plan, CG_ERR_INVALID_ARG for an unknown sample type.
 */
cg_status cg_create_plan_ex(int32_t frame_len, double fs, const int32_t* tooth_bins,
                            int32_t n_teeth, const float* ref_spectrum, int32_t sample_type,
                            cg_plan** out_plan);

/* Bytes per sample of the plan's frames (2 or 1). */
cg_status cg_plan_sample_bytes(const cg_plan* plan, int32_t* bytes);

/* Release a plan and everything it owns (NULL is allowed).  Synchronises the
 * device first. */
cg_status cg_destroy_plan(cg_plan* plan);

/* Replace the plan's reference spectrum (host float32[n_teeth], finite, > 0);
 * synchronises the device first so no queued work sees a partial update. */
cg_status cg_set_reference(cg_plan* plan, const float* ref_spectrum);

/* Read back the plan's geometry (any output pointer may be NULL). */
cg_status cg_plan_info(const cg_plan* plan, int32_t* frame_len, int32_t* n_teeth, double* fs);

/*
 * Bytes of device workspace cg_process_batch_ex needs for `n_frames` frames
 * when the caller supplies one: the float32 [n_frames][n_teeth] normalised
 * spectra and the float32 [n_frames][4] start points, each 256-byte aligned.
 * The workspace must be 256-byte aligned.
 */
cg_status cg_workspace_bytes(const cg_plan* plan, int64_t n_frames, size_t* bytes);

/*
 * Whole hot path for one batch: cast + frame, real FFT, tooth gather,
 * amplitude, division by the reference, 7x7 median start point and the
 * Levenberg-Marquardt fit (at most 20 iterations, tolerance 1e-6).
 *   frames      device [n_frames][frame_len] samples (int16, or int8 for a
 *               CG_SAMPLES_INT8 plan).
 *   out_params  device float32[n_frames][4] (centre, width, depth, baseline).
 * Uses the plan's internal workspace, grown on demand (the first call for a
 * larger batch allocates).  The 7x7 median window replicates the first and
 * last frame of the batch at its edges, so results depend on how a stream is
 * cut into batches only within three frames of a cut.
 */
cg_status cg_process_batch(cg_plan* plan, const void* frames, int64_t n_frames,
                           float* out_params, void* stream);

/*
 * As cg_process_batch, with optional outputs (each NULL = not written):
 *   out_iters   device int32[n_frames]  LM iterations used.
 *   out_status  device int32[n_frames]  CG_FIT_* code.
 *   out_chi2    device float32[n_frames] final sum of squared residuals.
 *   out_teeth   device float32[n_frames][n_teeth] raw amplitudes |X[k_i]|.
 *   out_y       device float32[n_frames][n_teeth] normalised spectra.
 *   flags       one CG_DFT_* form OR one CG_FIT_* form (CG_FIT_FANO: the
 *               paper's boxed Fano fit, see cg_set_fano).
 *   workspace   device buffer of >= cg_workspace_bytes() bytes, or NULL to use
 *               the plan's own (then workspace_bytes is ignored).
 * out_params may be NULL only with CG_FIT_NONE.
 * The CG_DFT_MFMA_* forms evaluate the DFT at the tooth bins directly as the
 * product frames [n][frame_len] x basis [frame_len][2 n_teeth] on the matrix
 * cores (FP32 accumulation) instead of the FFT; they need 16-byte aligned
 * frames, and the first call with a form builds its basis (device allocation).
 * Errors: CG_ERR_WORKSPACE if workspace_bytes is too small; CG_ERR_STATE for
 * CG_FIT_WARM_MLP before cg_set_mlp; CG_ERR_INVALID_ARG for unknown flags.
 */
cg_status cg_process_batch_ex(cg_plan* plan, const void* frames, int64_t n_frames,
                              float* out_params, int32_t* out_iters, int32_t* out_status,
                              float* out_chi2, float* out_teeth, float* out_y, uint32_t flags,
                              void* workspace, size_t workspace_bytes, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the whole
 * path of cg_process_batch_ex with its workspace (normalised spectra, start
 * points, chi2, fallback flags, list and count) in a fixed device array that
 * the library carries, CG_STATIC_SCRATCH_BYTES bytes on each GPU it runs on,
 * held until the process ends.  The call allocates nothing: no hipMalloc, no
 * hipFree, no allocating library routine.
 *   frames, out_params, out_iters, out_status, out_chi2, flags, stream as for
 *   cg_process_batch_ex (out_teeth / out_y are not offered); flags must name
 *   the FFT form (CG_DFT_FFT) with CG_FIT_COLD, CG_FIT_WARM_MLP or
 *   CG_FIT_FANO (the matrix-core forms build a basis on first use, which
 *   allocates).
 * Needs cg_workspace_bytes(plan, n_frames) <= CG_STATIC_SCRATCH_BYTES (for
 * 220 teeth: up to 72 000 frames); larger batches get CG_ERR_WORKSPACE and
 * nothing is enqueued.  The array's address on a device is resolved when a
 * plan is created there.
 * Every call on one GPU shares that GPU's array, which keeps the contents of
 * the last call; nothing in it needs to start at zero (the fallback count is
 * cleared by the kernels).  Calls that overlap on one GPU (on different
 * streams, or from different threads) race on the array: the caller orders
 * them.
 */
#define CG_STATIC_SCRATCH_BYTES (64u << 20)
cg_status cg_process_batch_static(cg_plan* plan, const void* frames, int64_t n_frames,
                                  float* out_params, int32_t* out_iters, int32_t* out_status,
                                  float* out_chi2, uint32_t flags, void* stream);

/*
 * Transform stage only: amplitudes at the tooth bins and/or normalised
 * spectra (either output may be NULL, not both).  `flags` selects the DFT form
 * (CG_DFT_*).  frames device int16[n_frames][frame_len]; outputs device
 * float32[n_frames][n_teeth].
 */
cg_status cg_teeth(cg_plan* plan, const void* frames, int64_t n_frames, float* out_teeth,
                   float* out_y, uint32_t flags, void* stream);

/*
 * Averaged reference spectrum (paper: pre-calculated average reference
 * spectrum): out_ref[i] = mean over the n reference frames of |X[k_i]|,
 * accumulated in FP64 in frame order.  ref_frames device int16[n][frame_len];
 * out_ref device float32[n_teeth].  The plan's own reference is not changed;
 * copy the result to the host and pass it to cg_set_reference to install it.
 */
cg_status cg_reference_from_frames(cg_plan* plan, const void* ref_frames, int64_t n,
                                   float* out_ref, void* stream);

/*
 * Cold-start initial guess on normalised spectra y (device float32
 * [n_frames][n_teeth]): M = 7x7 median of y over (frame, tooth) with edge
 * replication inside the batch; per frame centre = first index of min M,
 * baseline = lower median of the row of M, depth = clip(1 - M[centre] /
 * baseline, 0.05, 0.95) (0.05 if baseline <= 0), width = max(2, count of teeth
 * with M < baseline (1 - depth/2)), all decisions in float32.
 *   out_p0      device float32[n_frames][4].
 *   out_median  device float32[n_frames][n_teeth] or NULL (then M stays on
 *               chip); must not alias y.
 * y is taken to be finite (as normalised spectra from cg_teeth always are):
 * the median network does not order NaNs, so a NaN in y leaves the affected
 * filtered values and start points unspecified (never an error).
 */
cg_status cg_init_spectra(cg_plan* plan, const float* y, int64_t n_frames, float* out_p0,
                          float* out_median, void* stream);

/*
 * Start points for listed frames only (paper, Data Capture and Processing, as
 * cg_init_spectra; the learned warm start re-runs this cold start for the
 * frames whose network fit it rejects).  listed: device int32[n_frames];
 * row f of out_p0 is written when listed[f] != 0 and left untouched
 * otherwise.  The 7x7 median still reads the neighbouring frames of a listed
 * one, listed or not, so its values are those cg_init_spectra gives.  Errors
 * as for cg_init_spectra (CG_ERR_NULL for a NULL listed with n_frames > 0).
 */
cg_status cg_init_spectra_listed(cg_plan* plan, const float* y, int64_t n_frames,
                                 const int32_t* listed, float* out_p0, void* stream);

/*
 * The start centres alone (paper, Data Capture and Processing: the lowest
 * value of each row of the 7x7-median image): column 0 of out_p0 (device
 * float32 [n_frames][4]) receives the same centre cg_init_spectra writes;
 * columns 1..3 are left untouched.  The boxed Fano fit starts from these
 * (its extent and scale start at the plan's averages).  Only the columns
 * whose window bounds (smallest and largest median of a window's row
 * segments) leave room for a row's minimum are filtered exactly, so spectra
 * with a dip take less time than cg_init_spectra; the centres are the same.
 * Errors as for cg_init_spectra.
 */
cg_status cg_start_centres(cg_plan* plan, const float* y, int64_t n_frames, float* out_p0,
                           void* stream);

/*
 * The two kernels of cg_init_spectra, callable on their own:
 * cg_median_filter writes out_median = 7x7 median image of y (both device
 * float32 [n_frames][n_teeth], distinct buffers); cg_start_points turns a
 * median image into start points out_p0 (device float32 [n_frames][4]) by the
 * rules of cg_init_spectra.
 */
cg_status cg_median_filter(cg_plan* plan, const float* y, int64_t n_frames, float* out_median,
                           void* stream);
cg_status cg_start_points(cg_plan* plan, const float* median, int64_t n_frames, float* out_p0,
                          void* stream);

/*
 * Levenberg-Marquardt fit of the Lorentzian dip to each row of y from p0
 * (device float32 [n_frames][n_teeth] and [n_frames][4]).  Damped normal
 * equations (A + lam diag A) d = J^T r solved by an FP64 Cholesky; lam starts
 * at 1e-3, /10 on accept, *10 on reject; a step is accepted when chi2 does not
 * increase, width stays > 0 and all values are finite; converged when an
 * accepted step lowers chi2 by <= 1e-6 chi2 (or chi2 <= 1e-30).  Residuals,
 * Jacobian and sums are FP32, the chi2 decrease of a step taken from the
 * model's change so that it is exact to FP32 rounding of itself; a spectrum
 * the model reproduces exactly stops at chi2 <= K (2^-19 b0)^2 (b0: the start
 * baseline), the FP32 counterpart of 1e-30, and is reported converged.
 * max_iter in 1..CG_MAX_ITER (the paper uses 20).  Outputs as in
 * cg_process_batch_ex.
 */
cg_status cg_fit_spectra(cg_plan* plan, const float* y, const float* p0, int64_t n_frames,
                         int32_t max_iter, float* out_params, int32_t* out_iters,
                         int32_t* out_status, float* out_chi2, void* stream);

/*
 * The paper's own fit (CG_FIT_FANO; paper, Data Capture and Processing: a
 * five-parameter asymmetric Fano lineshape, only the centre free, scale and
 * extent held within about +-10 % of pre-computed averages, asymmetry and
 * width fixed to values measured for the device, <= 20 iterations,
 * tolerance 1e-6):
 *   y(x) = scale * (1 - extent * (1 + u/asymmetry)^2 / (1 + u^2)),
 *   u = 2 (x - centre) / width,
 * fitted by Levenberg-Marquardt over (centre, extent, scale) with extent in
 * [0.9, 1.1] * depth_avg and scale in [0.9, 1.1] * scale_avg: a boxed
 * parameter on a bound whose gradient points out of the box is held for the
 * step and every trial point is clipped into the box.  Start point: the
 * centre of the 7x7-median initializer (cg_init_spectra), extent and scale
 * at their averages.  Schedule, statuses and arithmetic as the Lorentzian
 * fit (FP32 per tooth, the chi2 decrease of a step from the model's change,
 * the same resolution floor; FP64 Cholesky).  Output parameters (centre,
 * width (the fixed value), extent, scale).
 * cg_set_fano: width > 0, |asymmetry| >= 1e-3, averages > 0, all finite
 * (host doubles; CG_ERR_INVALID_ARG otherwise).  cg_fit_fano: the fit alone
 * on normalised spectra y (device float32 [n_frames][n_teeth]) from start
 * points p0 (device float32 [n_frames][4], column 0 used), outputs as
 * cg_fit_spectra; CG_ERR_STATE before cg_set_fano.
 */
cg_status cg_set_fano(cg_plan* plan, double width, double asymmetry, double depth_avg,
                      double scale_avg);
cg_status cg_fit_fano(cg_plan* plan, const float* y, const float* p0, int64_t n_frames,
                      int32_t max_iter, float* out_params, int32_t* out_iters,
                      int32_t* out_status, float* out_chi2, void* stream);

/*
 * Learned warm start (CG_FIT_WARM_MLP).  A network 220 -> 256 -> 256 -> 4 with
 * GELU maps a normalised tooth vector to standardised start parameters
 * (c, w, d, b); bfloat16 matrix-product operands, FP32 accumulation, biases and
 * GELU (exact erf) in FP32.  Spectra with K != 220 teeth are resampled
 * linearly onto 220 points and the predicted centre and width scaled by
 * (K-1)/219.  The start point is polished by 2 LM iterations; a frame whose
 * RMS residual sqrt(chi2/(K-4)) then exceeds 2 * noise_floor (or is not
 * finite) is re-fitted from the cold-start (7x7 median) point with the full
 * LM and reported with status CG_FIT_FALLBACK.
 *
 * Parameters are one host float32 array of CG_MLP_NPARAMS values in the order
 * W1[256][220], b1[256], W2[256][256], b2[256], W3[4][256], b3[4] (row-major,
 * out x in).
 */
#define CG_MLP_NPARAMS 123396

/* Install trained weights in a plan.  out_mean/out_std (host float32[4]):
 * p = z * std + mean per output (c, w, d, b).  noise_floor > 0: typical RMS
 * residual of a converged cold-start fit of this stream. */
cg_status cg_set_mlp(cg_plan* plan, const float* params, const float* out_mean,
                     const float* out_std, float noise_floor);

/* Levenberg-Marquardt iterations run from the network's start point before
 * the residual test (paper's learned part: a short polish of one or two
 * iterations).  iters in 1..CG_MAX_ITER; the default is 2.  With 20, the
 * cold start's cap, the polish is a full fit from the network's start point.
 * Errors: CG_ERR_INVALID_ARG out of range. */
cg_status cg_set_polish_iters(cg_plan* plan, int32_t iters);

/* Network start points only: y device float32 [n_frames][n_teeth] -> out_p0
 * device float32 [n_frames][4] (CG_ERR_STATE before cg_set_mlp). */
cg_status cg_mlp_infer(cg_plan* plan, const float* y, int64_t n_frames, float* out_p0,
                       void* stream);

/* Training state: FP32 master weights, Adam moments and the buffers of one
 * mini-batch of `batch` samples (1..65536), on the current device. */
typedef struct cg_mlp_trainer cg_mlp_trainer;
cg_status cg_mlp_trainer_create(int32_t batch, const float* init_params /* host */,
                                cg_mlp_trainer** out);
cg_status cg_mlp_trainer_destroy(cg_mlp_trainer* trainer);

/*
 * One Adam step on the mini-batch rows idx[0..batch) (device int32) of
 *   x        device float32 [*][220] inputs,
 *   targets  device float32 [*][4] standardised labels,
 *   weights  device float32 [*] per-sample loss weights (NULL = all 1).
 * Loss: sum_s w_s sum_j (out_sj - t_sj)^2 / (4 sum_s w_s).  Adam with bias
 * correction (lr, beta1, beta2, eps).  loss: device float32 [1] or NULL.
 */
cg_status cg_mlp_train_step(cg_mlp_trainer* trainer, const float* x, const float* targets,
                            const float* weights, const int32_t* idx, float lr, float beta1,
                            float beta2, float eps, float* loss, void* stream);

/* Same forward/backward without the update: grads device float32
 * [CG_MLP_NPARAMS] (flat layout), loss device float32 [1] or NULL. */
cg_status cg_mlp_gradients(cg_mlp_trainer* trainer, const float* x, const float* targets,
                           const float* weights, const int32_t* idx, float* grads, float* loss,
                           void* stream);

/* Copy the FP32 master weights to the host (synchronises the device). */
cg_status cg_mlp_get_params(cg_mlp_trainer* trainer, float* params);

/*
 * Tuning knobs of a plan (launch shapes only).  Spectra per wavefront and the
 * FFT grid do not change any result; lanes per spectrum changes the order in
 * which each spectrum's sums are reduced, so results move by rounding only.
 *   CG_TUNE_LM_CHUNK    spectra per wavefront in the fit kernel: 0 = chosen
 *                       from the batch size (default), else a multiple of 4 in
 *                       4..256.
 *   CG_TUNE_LM_LANES    lanes per spectrum in the fit kernel: 0 = 8 up to 224
 *                       teeth, else 16 (default); 8 (only up to 224 teeth) or
 *                       16.
 *   CG_TUNE_FFT_BLOCKS  cap on the persistent FFT kernel's grid: 0 = every
 *                       block that fits on the device at once (default), else
 *                       at most that many blocks.
 * cg_get_tuning reads a knob back.
 * Errors: CG_ERR_INVALID_ARG for an unknown knob or value out of range.
 */
#define CG_TUNE_LM_CHUNK   1
#define CG_TUNE_LM_LANES   2
#define CG_TUNE_FFT_BLOCKS 3
cg_status cg_set_tuning(cg_plan* plan, int32_t knob, int32_t value);
cg_status cg_get_tuning(const cg_plan* plan, int32_t knob, int32_t* value);

/*
 * Multi-stream ring pipeline (paper: ring buffer between digitiser and GPU,
 * asynchronous batches across threads, out-of-order completion re-sorted into
 * time order; indefinite streaming only while consumption keeps up, otherwise
 * the buffer overflows).
 *
 * Each of n_streams streams (<= CG_PIPE_MAX_STREAMS) has its own plan (frame
 * length, teeth, reference, network) and fit form (CG_FIT_COLD or
 * CG_FIT_WARM_MLP) and slots_per_stream device slots of max_burst_frames
 * frames.  Each slot's processing chain is captured once as a hipGraph; a
 * persistent dispatcher thread launches published bursts in publish order on
 * one HIP stream per stream (default priority); it is the only thread that
 * enqueues on those streams (the copies cg_pipeline_put asks for included).
 * Latency from publish to results is recorded on the host clock (until the
 * dispatcher sees the burst complete) and on the GPU's wall clock (until the
 * results are in host memory; the publish time is mapped onto the GPU clock
 * by the smallest launch-to-start gap seen in the last 0.1-0.2 s).  Plans
 * must outlive the pipeline and must not change while it exists.
 *
 * options: CG_PIPE_KEEP_RESULTS keeps each completed burst's results (and its
 * slot) until cg_pipeline_read; without it slots are recycled on completion.
 * CG_PIPE_DRY_RUN simulates the bookkeeping without a device (plans and
 * fit_flags may be NULL): a burst completes dry_us_per_frame * n us after it
 * was published and acquire returns no frame buffer.
 */
typedef struct cg_pipeline cg_pipeline;
#define CG_PIPE_MAX_STREAMS  64
#define CG_PIPE_MAX_LANES    8
#define CG_PIPE_KEEP_RESULTS 0x1u
#define CG_PIPE_DRY_RUN      0x2u
#define CG_PIPE_HOST_RING    0x4u
cg_status cg_pipeline_create(int32_t n_streams, cg_plan* const* plans, const uint32_t* fit_flags,
                             int32_t slots_per_stream, int32_t max_burst_frames,
                             uint32_t options, double dry_us_per_frame, cg_pipeline** out);
/*
 * As cg_pipeline_create, with lanes_per_stream (1..CG_PIPE_MAX_LANES) compute
 * lanes (HIP streams) per stream: consecutive bursts of a stream go to the
 * lanes in turn and can run at the same time and complete out of order
 * (cg_pipeline_read still hands them out in publish order).  fit_flags may
 * also be CG_FIT_FANO (after cg_set_fano on the plan).
 * CG_PIPE_HOST_RING (paper, Data Capture and Processing: digitiser -> ring
 * buffer in host memory -> GPU): every slot also owns a pinned host frame
 * buffer; cg_pipeline_acquire returns that host buffer, and the dispatcher
 * copies each published burst host -> device on the stream's own copy
 * stream, the burst's graph waiting for the copy, so copies of later bursts
 * overlap the kernels of earlier ones; cg_pipeline_put then copies src (host
 * memory) into the slot on the calling thread.  The throughput counters then
 * include the PCIe transfer.
 */
cg_status cg_pipeline_create_ex(int32_t n_streams, cg_plan* const* plans,
                                const uint32_t* fit_flags, int32_t slots_per_stream,
                                int32_t max_burst_frames, uint32_t options,
                                int32_t lanes_per_stream, double dry_us_per_frame,
                                cg_pipeline** out);
/* Stops the dispatcher after the queued bursts completed, frees everything. */
cg_status cg_pipeline_destroy(cg_pipeline* pipe);
/* Take a free slot of `stream` for writing: *frames receives its device buffer
 * int16 [max_burst_frames][frame_len] (with CG_PIPE_HOST_RING: its pinned
 * host buffer).  CG_ERR_RING_FULL (counted as an
 * overflow) when every slot is queued, running or holding unread results. */
cg_status cg_pipeline_acquire(cg_pipeline* pipe, int32_t stream, int32_t* slot,
                              void** frames);
/* Hand a written slot to the dispatcher: n_frames in 1..max_burst_frames,
 * seq the caller's sequence number for this stream (increasing). */
cg_status cg_pipeline_publish(cg_pipeline* pipe, int32_t stream, int32_t slot, int32_t n_frames,
                              int64_t seq);
/* Acquire + copy + publish in one call: src holds n_frames frames of the
 * stream's frame length in host or device memory (any address HIP can copy
 * from).  The dispatcher queues the copy on the stream's HIP stream just
 * before the burst's graph, so src must stay valid and unchanged until the
 * burst completes; a host source is best pinned (a pageable one makes the
 * dispatcher wait for the copy).  CG_ERR_RING_FULL as for
 * cg_pipeline_acquire.  out_slot (may be NULL) receives the slot taken, so
 * the caller can keep src alive until that slot is handed out again. */
cg_status cg_pipeline_put(cg_pipeline* pipe, int32_t stream, const void* src, int32_t n_frames,
                          int64_t seq, int32_t* out_slot);
/* Pop the next burst of `stream` in publish order (CG_PIPE_KEEP_RESULTS),
 * once it has completed: bursts that complete before an earlier burst of
 * their stream are held until it has (the paper's re-sort of out-of-order
 * batches).  params host float32 [n][4], status host int32 [n] (either may be
 * NULL), capacity in frames.  CG_ERR_STATE with *n_frames = 0 when the next
 * burst is not ready (or none is queued); CG_ERR_STATE with the burst
 * dropped when its seq is not above the previous one read. */
cg_status cg_pipeline_read(cg_pipeline* pipe, int32_t stream, float* params, int32_t* status,
                           int32_t capacity, int32_t* n_frames, int64_t* seq);
/* Wait until every published burst has completed (CG_ERR_STATE on timeout). */
cg_status cg_pipeline_drain(cg_pipeline* pipe, int32_t timeout_ms);
/* Counters since creation, out[CG_PIPE_NSTATS]: bursts, frames, bytes of
 * int16 input, overflows, seconds from first publish to last completion,
 * host-clock latency p50, p99, max (ms), bytes/s, frames/s, GPU-clock
 * latency publish -> results p50, p99, max (ms), GPU-clock span graph start
 * -> results p50 (ms), bursts that completed ahead of an earlier burst of
 * their stream (re-sorted on read).  In dry-run mode the GPU-clock figures
 * are the host clock's.  Percentiles come from a uniform sample of at most
 * 2^20 bursts of the whole run, maxima from every burst.  With n_out >=
 * CG_PIPE_NSTATS_EX two more: the longest single burst launch on the
 * dispatcher thread (ms) and its longest pass over launches and completion
 * polling (ms). */
#define CG_PIPE_NSTATS 15
#define CG_PIPE_NSTATS_EX 17
cg_status cg_pipeline_stats(cg_pipeline* pipe, double* out, int32_t n_out);

/*
 * Autotuner: times the whole path (flags as for cg_process_batch_ex) on the
 * given frames for each launch shape -- fit-kernel lanes per spectrum (8 when
 * the teeth allow it, 16) x spectra per wavefront (1, 2, 4, 8 per lane group)
 * x FFT grid (every resident block, half of them) -- installs the fastest in
 * the plan (read it back with cg_get_tuning) and returns its spectra per
 * wavefront (*chosen) and its time per batch (*best_ms, may be NULL).
 * Timing: the plan's current shape first runs for at least 100 ms of device
 * time (an idle device starts at a low clock that rises over its first
 * milliseconds of work), then every candidate is timed once per round over
 * three rounds and keeps its fastest time; a timing covers passes over about
 * 64 Ki frames (at most 16 passes).  The plan's current shape is kept unless
 * a candidate is at least 3 % faster.  Synchronises the device; allocates a
 * parameter buffer for the timing.
 */
cg_status cg_autotune(cg_plan* plan, const void* frames, int64_t n_frames, uint32_t flags,
                      void* workspace, size_t workspace_bytes, int32_t* chosen, float* best_ms);

/*
 * Displacement power spectral density and the mechanical resonance fit
 * (paper, Experimental Results and the figure of the power spectral density:
 * the fitted centres form a displacement series; its PSD averaged over 1 s,
 * 10 s and 10 min shows the thermomechanical resonance near 24 kHz, whose fit
 * gives the resonance frequency f and quality factor Q).
 *
 * cg_psd_band: the bins k_lo .. k_lo + n_bins - 1 of segments of seg_len
 * samples that cover [f_lo, f_hi] Hz at sample rate fs (bin k is k fs /
 * seg_len Hz; clipped at seg_len / 2).
 * cg_psd_welch: Welch's averaged periodogram of `series` (device float32
 * [n], e.g. the centres of consecutive frames, fs = frame rate): segments of
 * seg_len (16384, 32768, 65536 or 131072) samples overlapping by half,
 * segment mean removed, periodic Hann window, one-sided density (units^2 /
 * Hz; factor 1 instead of 2 at DC and Nyquist), averaged over the segments;
 * out_psd device float64 [n_bins] for the band bins.  FP32 transforms (the
 * half-length complex FFT of even/odd-packed samples, split 128-point
 * columns x rows), FP64 averages.  Needs n >= seg_len, an 8-byte aligned
 * series and a 256-byte aligned device workspace of
 * cg_psd_workspace_bytes() bytes (segments are processed in chunks of up to
 * CG_PSD_CHUNK).
 * cg_resonance_fit: fits S(f) = A / ((f0^2 - f^2)^2 + (f0 f / Q)^2) + B to
 * a band of the PSD (device float64 [n_bins], n_bins 8..CG_PSD_MAX_FIT_BINS,
 * bin b at f_first + b df Hz) by Levenberg-Marquardt on ln S in FP64 (lam0
 * 1e-3, /10 on accept, *10 on reject, converged when an accepted step lowers
 * chi2 by at most tol chi2; at most max_iter iterations), starting from the
 * peak bin, the half-width of the peak above the floor (the median of the
 * band's lowest quarter) and the peak height.  out: device float64 [7] =
 * ln A, f0 (Hz), Q, ln B, chi2, iterations, status (CG_FIT_*).
 */
#define CG_PSD_CHUNK 1024
#define CG_PSD_MAX_FIT_BINS 2048
cg_status cg_psd_band(int32_t seg_len, double fs, double f_lo, double f_hi, int32_t* k_lo,
                      int32_t* n_bins);
cg_status cg_psd_workspace_bytes(int64_t n, int32_t seg_len, int32_t n_bins, size_t* bytes);
cg_status cg_psd_welch(const float* series, int64_t n, double fs, int32_t seg_len, int32_t k_lo,
                       int32_t n_bins, double* out_psd, void* workspace, size_t workspace_bytes,
                       void* stream);
cg_status cg_resonance_fit(const double* psd, int32_t n_bins, double f_first, double df,
                           int32_t max_iter, double tol, double* out, void* stream);

/* Static description of a status code. */
const char* cg_status_string(cg_status status);

/* Thread-local detail of the last CG_ERR_HIP / CG_ERR_OOM raised on this
 * thread ("" if none). */
const char* cg_last_error_detail(void);

/* Library version string. */
const char* cg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* COMBGPU_H */
