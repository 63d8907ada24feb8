/*
 * uvmem.h -- C ABI of the MI355X (gfx950) non-gridding maximum-entropy
 * imaging hot path (Carcamo et al., "Multi-GPU maximum entropy image
 * synthesis for radio astronomy").
 *
 * What it computes (paper Sec. 2.2-2.5):
 *   V^m_k   = sum_{i,j} A_ij I_ij exp(-2 pi i (u_k x_j + v_k y_i))  (Eq. fft,
 *             discretised exactly at the measured, ungridded (u_k, v_k))
 *   R_k     = V^m_k - V^o_k                                       (Alg. 2)
 *   chi^2   = 1/2 sum_k w_k |R_k|^2, w_k = 1/sigma_k^2             (Eq. phi2)
 *   S       = sum_p I_p ln(I_p / M)        (regulariser; Eq. Sgradient is its
 *                                           gradient ln(I/M) + 1)
 *   Phi     = chi^2 + lambda S                                     (Eq. phi3)
 *   grad chi^2_ij = A_ij sum_k Re(w_k R_k exp(+2 pi i (u_k x_j + v_k y_i)))
 *                                            (Eq. chi2gradient, Alg. 3; the
 *                                            A_ij factor is the exact derivative)
 *   grad Phi = grad chi^2 + lambda (ln(I/M) + 1)
 * and a positively-constrained projected conjugate-gradient step minimising
 * Phi over I >= M (Eq. minproblem; M plays the role of the paper's G).
 *
 * Geometry: image side N (even), pixel (i, j) at x_j = (j - N/2) cell,
 * y_i = (i - N/2) cell (Alg. 3 with the phase centre at pixel (N/2, N/2));
 * linear pixel index N*i + j (row i <-> y).  u, v in wavelengths, cell in
 * radians.  Every channel has its own visibilities, weights and primary
 * beam.  In cube mode the channels are independent problems, each with its
 * own image; in shared mode one image is seen by all channels and chi^2 is
 * the sum over channels (Eq. chi2-multi).
 *
 * Conventions for every entry point:
 *  - Return value: UVMEM_OK (0) or a negative uvmem_status.  On error the
 *    context keeps a message readable with uvmem_last_error(); no C++
 *    exception crosses the ABI.  A context is used by one host thread at a
 *    time.
 *  - Pointers named *_dev are device pointers on the context's device; the
 *    caller owns them.  set_* calls accept host or device pointers and copy
 *    the data into buffers the context owns (the caller may free its copy).
 *  - Image-like arrays are [n_img][N][N] row-major (n_img = n_chan in cube
 *    mode, 1 in shared mode; beam images are per channel), element type double for
 *    UVMEM_FP64 and float for every other precision.  Visibility arrays are
 *    the concatenation of the channels in channel order.
 *  - Hot entry points (phi_and_grad, forward, adjoint, cg_step, cg_run) only
 *    enqueue work on the context's stream and never synchronise; the
 *    results are valid once that stream has reached them.  They allocate no
 *    buffers: uvmem_finalize allocates every one (cg_run's first graph
 *    capture on an image leaves the instantiation to the HIP runtime).
 */
#ifndef UVMEM_H
#define UVMEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct uvmem_ctx uvmem_ctx;

typedef enum uvmem_status {
    UVMEM_OK = 0,
    UVMEM_EINVAL = -1,   /* bad argument (null pointer, size, index)          */
    UVMEM_ENOMEM = -2,   /* device or host allocation failed                  */
    UVMEM_EDEVICE = -3,  /* a HIP runtime call failed                         */
    UVMEM_EDOMAIN = -4,  /* an image pixel was <= 0 or NaN (from uvmem_check) */
    UVMEM_ESTATE = -5,   /* call out of order (e.g. set_* after finalize)     */
    UVMEM_ETOOBIG = -6   /* sizes need more than an allocation-free entry
                            point's fixed scratch (UVMEM_NOALLOC_SCRATCH_BYTES) */
} uvmem_status;

/* Precision of the DFT contractions (the chi^2, entropy and line-search sums
 * are FP64 in every mode, and so are the model visibilities and residuals). */
typedef enum uvmem_precision {
    UVMEM_FP64 = 0,      /* FP64 operands, FP64 matrix cores                  */
    UVMEM_FP32 = 1,      /* FP32 operands on FP32 matrix cores                */
    UVMEM_BF16X3 = 2,    /* bf16 hi+lo split, three products, FP32 accumulate */
    UVMEM_FP16X3 = 3     /* fp16 hi+lo split (power-of-two scaled), three products */
} uvmem_precision;

/* Image model.  n_img below is the number of image planes: n_chan in cube
 * mode, 1 in shared mode.  Images, gradients, the CG state and the scalar
 * records have one plane / record per image; visibilities, weights and
 * beams stay per channel. */
typedef enum uvmem_mode {
    UVMEM_CUBE = 0,      /* one image per channel, channels independent       */
    UVMEM_SHARED = 1     /* one image seen by every channel through its own
                            uv scale and beam A_c (Eq. chi2-multi):
                            chi^2 = sum_c chi^2_c, grad chi^2 = sum_c A_c o
                            Re F_c^H (w_c R_c), S and the CG over the one image */
} uvmem_mode;

/* Forward model of the objective.  UVMEM_FWD_DFT (the default) is the exact
 * direct DFT above.  UVMEM_FWD_GRIDDED is the paper's GPU approximation
 * (Sec. 2.4 items 1-4, Alg. 1): B_c = A_c o I zero-padded to an L x L grid,
 * L = oversample * N; its 2-D DFT on the uniform grid du = 1/(L cell);
 * modulation by e^{+2 pi i (u x_c + v y_c)} (phase centre at pixel N/2);
 * then bilinear interpolation at (u_k/du, v_k/du), wrapping modulo L.  The
 * transforms run in FP64 for UVMEM_FP64 and in FP32 for every other
 * precision.  The chi^2 gradient is chosen by uvmem_gradient_model. */
typedef enum uvmem_forward_model {
    UVMEM_FWD_DFT = 0,
    UVMEM_FWD_GRIDDED = 1
} uvmem_forward_model;

typedef enum uvmem_gradient_model {
    UVMEM_GRAD_ADJOINT = 0,  /* the exact adjoint of the forward model in use:
                                grad Phi is the gradient of Phi               */
    UVMEM_GRAD_DFT = 1       /* Eq. chi2gradient with the exact DFT at the
                                gridded residuals (the paper's combination;
                                with the gridded model Phi and grad Phi then
                                belong to different operators)                */
} uvmem_gradient_model;

/* Per-image scalar slots, FP64, layout [n_img][UVMEM_NSCAL]. */
enum {
    UVMEM_S_PHI = 0,     /* Phi = chi^2 + lambda S                            */
    UVMEM_S_CHI2 = 1,    /* chi^2                                             */
    UVMEM_S_S = 2,       /* S                                                 */
    UVMEM_S_ALPHA = 3,   /* CG step length of the last step                   */
    UVMEM_S_BETA = 4,    /* Polak-Ribiere beta of the last step               */
    UVMEM_S_GNORM2 = 5,  /* squared norm of the projected gradient            */
    UVMEM_S_ALPHA_MAX = 6, /* largest feasible step of the last line search   */
    UVMEM_S_ITER = 7,    /* CG iterations taken so far (stops count)          */
    UVMEM_NSCAL = 8
};

/* Create a context for images of side n (even, 2..8192), n_chan >= 1
 * channels and image model `mode` (uvmem_mode).  hip_stream is a hipStream_t
 * (NULL = the null stream) on the current device; all work is enqueued
 * there. */
int uvmem_create(uvmem_ctx **out, int n, int n_chan, int mode, int precision, void *hip_stream);
int uvmem_destroy(uvmem_ctx *ctx);

/* Visibility coordinates of channel `chan` (Sec. 2.1): nvis >= 0 points,
 * u, v in wavelengths (double[nvis]).  cell_rad is the pixel size Delta x in
 * radians and must be the same for every channel (one pixel grid).  nvis = 0
 * is legal: the channel then contributes chi^2 = 0 and grad chi^2 = 0.
 * UVMEM_EINVAL for non-finite u, v or |u| cell_rad, |v| cell_rad above 4096
 * cycles per pixel (8192 times the grid's Nyquist limit). */
int uvmem_set_uv(uvmem_ctx *ctx, int chan, int64_t nvis, const double *u, const double *v,
                 double cell_rad);
/* Observed visibilities V^o of the channel: float[nvis][2] (re, im). */
int uvmem_set_vis(uvmem_ctx *ctx, int chan, const float *vis);
/* Weights w_k = 1/sigma_k^2 >= 0 of the channel: float[nvis]; 0 = flagged. */
int uvmem_set_weights(uvmem_ctx *ctx, int chan, const float *w);
/* Gaussian primary beam of the given FWHM (radians), centred on the phase
 * centre (Sec. 2.4 item 1): A_ij = exp(-4 ln2 (x_j^2 + y_i^2) / fwhm^2). */
int uvmem_set_beam(uvmem_ctx *ctx, int chan, double fwhm_rad);
/* General attenuation image A for the channel: float[N][N]. */
int uvmem_set_beam_image(uvmem_ctx *ctx, int chan, const float *A);
/* Pointing of channel `chan` in a mosaic (Sec. 1, mosaic support; Sec. 2.4
 * items 1 and 3): the channel's Gaussian primary beam (uvmem_set_beam) is
 * centred at (x0, y0) radians from the image centre, and its visibilities
 * are phase-referenced to (x0, y0), so that its model is
 *   V_k = e^{+2 pi i (u_k x0 + v_k y0)} sum_ij A_ij I_ij e^{-2 pi i (u_k x_j + v_k y_i)}.
 * At finalize the library rotates the channel's observed visibilities by
 * e^{-2 pi i (u_k x0 + v_k y0)} (FP64, phase reduced mod 1); chi^2 and all
 * gradients are unchanged by it, but the channel's residuals
 * (uvmem_get_residual) and model visibilities (uvmem_forward) are then
 * referenced to the image centre.  A beam image from uvmem_set_beam_image is
 * used as given.  Fitting one image to all pointings is shared mode.
 * Default (0, 0).  UVMEM_EINVAL for a bad channel or a non-finite centre,
 * UVMEM_ESTATE after finalize. */
int uvmem_set_phase_centre(uvmem_ctx *ctx, int chan, double x0_rad, double y0_rad);
/* Choose the forward model (uvmem_forward_model) before finalize.  For
 * UVMEM_FWD_GRIDDED, oversample >= 1 and L = oversample * N must be a power
 * of two in [16, 8192] ([16, 4096] for UVMEM_FP64); grad is a
 * uvmem_gradient_model and also selects what uvmem_adjoint computes.  The
 * gridded model sorts the visibilities by grid cell at finalize (so the
 * adjoint's sums have a fixed order) and holds per channel an L x L complex
 * spectrum, an L x N row-pass buffer and L^2 + 1 cell offsets; it needs fewer
 * than 2^31 visibilities.  For UVMEM_FWD_DFT, oversample and grad are
 * ignored.  UVMEM_EINVAL on bad values, UVMEM_ESTATE after finalize. */
int uvmem_set_forward_model(uvmem_ctx *ctx, int model, int oversample, int grad);
/* Focus of attention (Sec. 6: reconstruction restricted to a region the
 * user selects, fewer free parameters): mask of image plane `img`,
 * uint8[N][N] (host or device; nonzero = free pixel).  NULL (the default)
 * makes every pixel free.  Pixels outside the mask are not free parameters:
 * the CG keeps them at their current value and uvmem_phi_and_grad reports
 * grad Phi = 0 there; Phi, chi^2 and S still cover every pixel.  With the
 * exact DFT, the CG's direction forward model visits only the image blocks
 * that meet a mask, and gradients only the pixel tiles that meet one
 * (work lists built at finalize for the union of the planes' masks).  Call before
 * finalize; UVMEM_EINVAL for a bad plane, UVMEM_ESTATE after finalize. */
int uvmem_set_mask(uvmem_ctx *ctx, int img, const uint8_t *mask);
/* Image floor M > 0 (the paper's G, Eq. minproblem) and entropy weight
 * lambda >= 0 (Eq. phi2). */
int uvmem_set_prior(uvmem_ctx *ctx, double M, double lambda);
/* Validate, upload, build the work tables and allocate every buffer.  After
 * it, set_* return UVMEM_ESTATE and the hot entry points allocate nothing. */
int uvmem_finalize(uvmem_ctx *ctx);

/* One evaluation of Phi and grad Phi at I_dev ([n_img][N][N]).  grad_dev
 * receives grad Phi ([n_img][N][N]); scal_dev (may be NULL) receives Phi,
 * chi^2 and S per image in slots UVMEM_S_PHI..UVMEM_S_S of
 * double[n_img][UVMEM_NSCAL].  The residuals R are kept in the context. */
int uvmem_phi_and_grad(uvmem_ctx *ctx, const void *I_dev, void *grad_dev, double *scal_dev);
/* Model visibilities V^m = F(I) (Eq. fft) of every channel: vis_dev is
 * double[sum Z][2]; I_dev is [n_img][N][N]. */
int uvmem_forward(uvmem_ctx *ctx, const void *I_dev, void *vis_dev);
/* Adjoint A o Re F^H c of complex coefficients c (double[sum Z][2], e.g. the
 * weighted residual w R): img_dev is [n_img][N][N] (shared mode: the sum
 * over channels).  F is the exact DFT, or the gridded model when that model
 * is in use with UVMEM_GRAD_ADJOINT. */
int uvmem_adjoint(uvmem_ctx *ctx, const void *coef_dev, void *img_dev);
/* Copy the current residuals R = V^m - V^o (double[sum Z][2]) to res_dev. */
int uvmem_get_residual(uvmem_ctx *ctx, void *res_dev);

/* Natural-weight dirty image and point spread function (App. A, Eq. dirty
 * and Eq. PSF) of every image plane, without attenuation:
 *   dirty_ij = Re sum_k w_k V^o_k e^{+2 pi i (u_k x_j + v_k y_i)} / sum_k w_k
 *   psf_ij   = sum_k w_k cos(2 pi (u_k x_j + v_k y_i)) / sum_k w_k
 * with the sums over the channels of the plane (shared mode: all channels;
 * mosaic pointings contribute in the image-centre frame).  They are
 * computed with the adjoint in use (the exact DFT, or the gridded model
 * under UVMEM_GRAD_ADJOINT).  Outputs [n_img][N][N] in the precision's real
 * type; either may be NULL.  Enqueued on the stream; the direction
 * visibilities and split-K partials serve as scratch (no CG state is
 * touched). */
int uvmem_dirty_image(uvmem_ctx *ctx, void *dirty_dev, void *psf_dev);
/* Thermal noise of the dirty image, sigma_D = 1 / sqrt(sum_k w_k) per image
 * plane (App. B), into host double[n_img]; INFINITY for a plane without
 * weight.  UVMEM_ESTATE before finalize. */
int uvmem_noise(const uvmem_ctx *ctx, double *sigma_d);
/* Clean beam (App. A): an elliptical Gaussian fitted to the main lobe of
 * each PSF plane psf_dev ([n_img][N][N] from uvmem_dirty_image): the pixels
 * with PSF >= 1/2 connected to the centre pixel, least squares of -ln PSF as
 * a quadratic form in the pixel offsets.  bmaj, bmin: full widths at half
 * maximum along the major and minor axes (radians); bpa: angle of the major
 * axis from +y towards +x in degrees, in (-90, 90]; host double[n_img] each.
 * Synchronises the stream; UVMEM_EDOMAIN if a lobe cannot be fitted. */
int uvmem_fit_beam(uvmem_ctx *ctx, const void *psf_dev, double *bmaj, double *bmin, double *bpa);

/* Projected CG (positively constrained, Sec. 2.6).  cg_init evaluates Phi at
 * I_dev (first setting I_dev to M everywhere if init_to_floor) and sets the
 * first direction.  cg_step performs one iteration in place on I_dev (which
 * must be the same buffer as in cg_init) and writes the per-image scalars
 * (all UVMEM_NSCAL slots) to scal_dev (may be NULL).  An image whose line
 * search stalls (no descent, or zero projected gradient) stops: later steps
 * leave it unchanged.  cg_run performs `iters` steps, writing scalars to
 * scal_hist_dev (double[iters][n_img][UVMEM_NSCAL], may be NULL); with
 * use_graph != 0 it replays one step captured as a HIP graph.  The first
 * use_graph call on an image captures that step on a stream the context
 * owns and instantiates the graph (the HIP runtime allocates the executable
 * graph there); later calls only launch it on the context's stream.  No
 * call synchronises. */
int uvmem_cg_init(uvmem_ctx *ctx, void *I_dev, int init_to_floor);
int uvmem_cg_step(uvmem_ctx *ctx, void *I_dev, double *scal_dev);
int uvmem_cg_run(uvmem_ctx *ctx, void *I_dev, int iters, double *scal_hist_dev, int use_graph);
/* Checkpoint of the CG state (direction, projected gradients, residuals,
 * scalars, iteration count) to/from host memory.  With host_blob == NULL,
 * get_state only reports the size in *bytes.  Both synchronise the stream.
 * Blob layout (native byte order, parts back to back): a 48-byte header
 * (uint64 magic; int32 image side, channel count, precision, mode, forward
 * model, grid side, gradient model, pad; int64 total visibilities), then the
 * direction d, the projected gradient and the gradient, each n_img x N x N
 * values of the context's real type (double for UVMEM_FP64, else float),
 * the residuals R (complex128 per visibility), the UVMEM_NSCAL scalars of
 * each image (double) and eight double CG flags per image.  set_state
 * refuses a blob whose header does not match the context. */
int uvmem_cg_get_state(uvmem_ctx *ctx, void *host_blob, size_t *bytes);
int uvmem_cg_set_state(uvmem_ctx *ctx, const void *host_blob, size_t bytes);

/* Synchronise the stream; return UVMEM_EDOMAIN if any evaluated image had a
 * pixel <= 0 or NaN since the last check (and clear the flag), else the
 * first asynchronous HIP error, else UVMEM_OK. */
int uvmem_check(uvmem_ctx *ctx);

/* Kernel timing (benchmarking): when enabled, the forward and adjoint
 * launches of every hot call are bracketed by HIP events on the context's
 * stream.  which = 0 forward, 1 adjoint; total_ms and count accumulate over
 * completed launches (reading synchronises the stream); reset clears them. */
int uvmem_timing_enable(uvmem_ctx *ctx, int enable);
int uvmem_timing_read(uvmem_ctx *ctx, int which, double *total_ms, int64_t *count, int reset);

/* Introspection.  uvmem_info writes up to nout of, in order: N, padded side
 * Np, channels, precision, total visibilities, forward image blocks, adjoint
 * tile side, adjoint split-K slots, forward workgroups, adjoint workgroups,
 * visibility items, device bytes held, pixel blocks per channel, pixels per
 * pixel block, visibilities per visibility item, image planes n_img, forward
 * model, gridded-model grid side L (0 for the DFT), gradient model,
 * forward and adjoint workgroups of the focus-of-attention region's work
 * lists (0 without a region).  uvmem_chan_range gives a channel's offset into the concatenated
 * visibility arrays and its count. */
int uvmem_info(const uvmem_ctx *ctx, int64_t *out, int nout);
int uvmem_chan_range(const uvmem_ctx *ctx, int chan, int64_t *offset, int64_t *nvis);

/* Allocation-free forward model, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same result as uvmem_forward of an FP32 context with
 * one channel whose beam image is `beam`, on the same FP32 matrix-core
 * kernels, but without a context:
 *   vis_k = sum_ij A_ij I_ij exp(-2 pi i (u_k x_j + v_k y_i)),
 * x_j = (j - n/2) cell_rad, y_i = (i - n/2) cell_rad.
 * Arguments: n even in [2, 8192]; nvis >= 0; u, v: device double[nvis]
 * (wavelengths; not validated -- non-finite values or |u| cell_rad, |v|
 * cell_rad beyond 4096 cycles per pixel give meaningless visibilities);
 * beam: device float[n][n] or NULL (A = 1); I: device float[n][n]; vis:
 * device double[nvis][2] (re, im), written; hip_stream: a hipStream_t of the
 * current device (NULL = null stream).  Enqueues on hip_stream and returns
 * without synchronising; calls no allocating routine.  Scratch: one fixed
 * device array of UVMEM_NOALLOC_SCRATCH_BYTES per GPU, held until the
 * process ends, shared by every call on that GPU -- calls that overlap on
 * one GPU (different streams, or host threads) race; calls on one stream
 * are ordered.  Returns UVMEM_EINVAL for bad sizes or null pointers,
 * UVMEM_ETOOBIG when the sizes need more than the scratch
 * (8 nvis + 8 nvis + 4 Np^2 + 16 nvis B Np^2 / (IB JB) + tables, each part
 * rounded up to 256 bytes; Np = n rounded up to a multiple of 64, IB x JB =
 * 128 x 256, 128 x 128 or 64 x 64 by Np), UVMEM_EDEVICE on a launch error. */
#define UVMEM_NOALLOC_SCRATCH_BYTES (64u << 20)
int uvmem_forward_noalloc(int n, double cell_rad, int64_t nvis, const double *u_dev, const double *v_dev,
                          const float *beam_dev, const float *I_dev, double *vis_dev, void *hip_stream);

const char *uvmem_last_error(const uvmem_ctx *ctx);
const char *uvmem_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* UVMEM_H */
