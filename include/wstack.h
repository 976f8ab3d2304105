/*
 * wstack.h - C ABI of the MI355X w-stacking imaging library (libwstack.so).
 *
 * The calls follow the paper's statement of the problem (Gheller, Taffoni &
 * Goz, "High Performance W-stacking for Imaging Radio Astronomy Data",
 * Sec. 2): visibilities with baseline coordinates (u, v, w) and weights are
 * convolved with a Gaussian kernel onto a Cartesian mesh of N_u x N_v x N_w
 * cells (Eq. 3, the nearest w-plane taking each visibility), every w-plane
 * is Fourier transformed (Eq. 2, inner integral), and a w-dependent phase
 * screen is applied to each transformed plane before the planes are summed
 * into the dirty image (Eq. 2, outer integral).  Degridding, the adjoint
 * map from an image back to visibilities, is the paper's future work
 * (Sec. 5) and is provided as the exact conjugate transpose.
 *
 * Conventions (the paper leaves them open; these are the library's):
 *   - u, v, w in wavelengths; fov_l, fov_m are the full image widths in
 *     radians.  Cell size du = 1/fov_l, dv = 1/fov_m; pixel size
 *     dl = fov_l/nu, dm = fov_m/nv.  Zero spacing at cell (nu/2, nv/2).
 *   - Visibility position x = u fov_l + nu/2, y = v fov_m + nv/2 (FP64);
 *     the K x K kernel is centred on the nearest cell floor(x + 1/2),
 *     floor(y + 1/2); tap weight c g(i - x) g(j - y) with
 *     g(d) = exp(-d^2/(2 sigma^2)), c = 1/(2 pi sigma^2).
 *   - Plane k = clamp(floor((w - w_min)/dw), 0, nw - 1), dw = (w_max -
 *     w_min)/nw, plane centre w_k = w_min + (k + 1/2) dw (nw = 1: one plane
 *     at (w_min + w_max)/2).
 *   - Transform: F[q][p] = sum_{j,i} P[j][i] exp(+2 pi i [(i - nu/2)(p -
 *     nu/2)/nu + (j - nv/2)(q - nv/2)/nv]) (direction +1), unnormalised.
 *   - Screen: exp(+2 pi i w_k (n - 1)), n - 1 = -r^2/(1 + sqrt(1 - r^2)),
 *     r^2 = l^2 + m^2, l_p = (p - nu/2) dl, m_q = (q - nv/2) dm.
 *
 * Layouts: complex values are interleaved (re, im) - complex64 on the FP32
 * path, complex128 on the FP64 path.  The plane stack is row-major
 * [k][j][i] (i along u, fastest), the image [q][p] (p along l, fastest).
 * uvw is float64 [m][3]; weights float32 [m] (NULL means unit weights).
 *
 * Memory: every device array is owned by the caller (for example torch
 * tensors); the library never allocates device memory.  A plan owns only a
 * small host structure.  All work is enqueued asynchronously on the plan's
 * HIP stream; pointers must stay valid until that work completes.
 *
 * Errors: every call returns a ws_status; WS_OK is 0 and errors are
 * negative.  Nothing is enqueued when a call fails its argument checks.
 * ws_last_error() returns a thread-local description of the last failure.
 * Kernel faults are asynchronous and surface at a later call or ws_sync().
 * Threading: one plan must not be used from two threads at once; distinct
 * plans are independent.
 */
#ifndef WSTACK_H
#define WSTACK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ws_status;
#define WS_OK 0
#define WS_INVALID_ARG (-1)          /* null pointer, bad enum, bad range */
#define WS_UNSUPPORTED_SIZE (-2)     /* grid or support outside the limits */
#define WS_WORKSPACE_TOO_SMALL (-3)  /* a caller buffer is too small */
#define WS_HIP_ERROR (-4)            /* a HIP runtime call failed */
#define WS_BAD_STATE (-5)            /* call not allowed in the plan's state */

#define WS_FP32 0 /* complex64 data and plane stack; FP32 kernel taps, FFT
                     and screen; FP64 positions, plane index, phase argument
                     and in-tile sums (FP64 LDS adds, rounded to FP32 once) */
#define WS_FP64 1 /* complex128 data, everything in FP64 (the paper's
                     precision, Sec. 4.2 memory model) */

/* Gridding kernels (Sec. 2, the paragraph after Eq. 3).  WS_KERNEL_GAUSS is
 * the paper's Gaussian: phi(d) = exp(-d^2/(2 sigma^2)), c = 1/(2 pi sigma^2).
 * WS_KERNEL_ES is the exponential of a semicircle, the analytic
 * approximation of the production (prolate-spheroidal) kernels the paper
 * names as the better choice at the same cost: phi(d) = exp(beta
 * (sqrt(1 - z^2) - 1)), z = 2 d / K, over the same K x K support, with c = 1 /
 * (integral of phi over |d| <= K/2)^2 so that the 2-D kernel integrates to
 * one.  Either kernel enters as G = c phi(i - x) phi(j - y). */
#define WS_KERNEL_GAUSS 0
#define WS_KERNEL_ES 1

/* Imaging geometry and kernel.
 *   nu, nv   grid size, each a power of two in [16, 32768] (65536 would
 *            overflow the 16-bit cell fields of the binned records, and a
 *            single FP32 plane of it is 34 GB)
 *   nw       number of w-planes, >= 1
 *   fov_l, fov_m  full field of view in radians, > 0, with
 *            (fov_l/2)^2 + (fov_m/2)^2 < 1
 *   w_min, w_max  w range in wavelengths covered by the planes;
 *            w_max > w_min when nw > 1
 *   support  kernel support K in cells, odd, 1..15 (the paper uses 7)
 *   sigma    Gaussian width in cells; <= 0 selects K/7
 *   precision  WS_FP32 or WS_FP64
 *   tile     gridding tile edge in cells (power of two, 16..64, > K - 1);
 *            0 = automatic
 *   chunk    most visibilities one gridding work item accumulates before a
 *            split tile is merged; 0 = automatic (4096)
 *   kernel   WS_KERNEL_GAUSS or WS_KERNEL_ES (sigma applies to the
 *            Gaussian only)
 *   beta     ES kernel shape; <= 0 selects 2.3 K; at most 200
 *   correct  1: grid correction - the image is divided by the kernel's 2-D
 *            Fourier transform c psi(f_p) psi(f_q), psi(f) the transform of
 *            the 1-D kernel truncated to |d| <= K/2 and f_p = (p - nu/2)/nu
 *            cycles per cell (the factor that undoes the kernel's taper of
 *            the image); degridding multiplies its input image by the same
 *            real factor, which keeps it the exact adjoint.  Refused
 *            (WS_INVALID_ARG) when psi is not positive for |f| <= 1/2.
 *            0: no correction (the dirty image of Eq. 2 as gridded).
 *   binning  how visibilities are grouped by (plane, tile, edge region)
 *            before gridding (the records and their order per key are the
 *            same): WS_BINNING_PARTITION - two-level partition by (plane,
 *            tile rows), then by (tile column, region), with per-workgroup
 *            histograms and no global atomics; WS_BINNING_HASHED - one
 *            counting sort with LDS-hashed counts and global atomics;
 *            WS_BINNING_AUTO - the partition whenever its histograms fit
 *            (at most 16384 buckets of at most 16384 keys), else hashed.
 *            Requesting WS_BINNING_PARTITION where it does not fit is
 *            WS_UNSUPPORTED_SIZE. */
#define WS_BINNING_AUTO 0
#define WS_BINNING_PARTITION 1
#define WS_BINNING_HASHED 2
typedef struct ws_params {
  int32_t nu, nv, nw;
  double fov_l, fov_m;
  double w_min, w_max;
  int32_t support;
  double sigma;
  int32_t precision;
  int32_t tile;
  int32_t chunk;
  int32_t kernel;
  double beta;
  int32_t correct;
  int32_t binning;
} ws_params;

typedef struct ws_plan ws_plan;

/* Check a parameter set without touching the GPU (host only). */
ws_status ws_validate_params(const ws_params* params);

/* Sizes in bytes of the two caller-owned device buffers a plan needs:
 * the plane stack (nw * nv * nu complex cells) and the workspace for
 * batches of up to max_vis visibilities (1 <= max_vis < 2^31).  For FP32
 * plans with nv = 4096, 512 <= nu <= 4096 and tile edge 64, the workspace
 * includes the one-call path's store of the tiles with records (at most
 * half the stack's size; tiles beyond it stay in the stack).  Host only;
 * needs no GPU.  Either output pointer may be NULL. */
ws_status ws_workspace_bytes(const ws_params* params, int64_t max_vis,
                             size_t* planes_bytes, size_t* work_bytes);

/* The kernel's 1-D Fourier transform and norm, as the library uses them
 * (host only; needs no GPU): psi[i] = integral over |d| <= K/2 of phi(d)
 * cos(2 pi f[i] d) dd for i < n (f in cycles per cell; FP64 tanh-sinh
 * quadrature), and *cnorm = c.  f, psi: host arrays of n doubles (may be
 * NULL when n = 0); cnorm may be NULL. */
ws_status ws_kernel_transform(const ws_params* params, int64_t n,
                              const double* f, double* psi, double* cnorm);

/* Build a plan over caller-owned device buffers (Sec. 2: the Cartesian
 * mesh of N_u x N_v x N_w cells).  planes and work must be device
 * pointers of at least the sizes ws_workspace_bytes() returns, 256-byte
 * aligned.  hip_stream is a hipStream_t (NULL = the null stream).  The
 * stack starts empty: it is cleared lazily by the first call that needs
 * it, so no work is enqueued here except the small twiddle tables.
 * *out receives a host handle to release with ws_plan_destroy(). */
ws_status ws_grid_init(const ws_params* params, int64_t max_vis, void* planes,
                       size_t planes_bytes, void* work, size_t work_bytes,
                       void* hip_stream, ws_plan** out);

/* Convolutional gridding (Eq. 3) of m visibilities onto the plane stack,
 * each to its nearest w-plane.  Additive: the first call after init or
 * reset writes every cell of the stack exactly once (zeros included);
 * later calls add to it, like the paper's slab-by-slab accumulation
 * (Sec. 3.2).  uvw: device float64 [m][3]; vis: device complex64 (FP32
 * path) or complex128 (FP64 path) [m]; weight: device float32 [m] or NULL.
 * n_dropped_taps: device int64 that the number of kernel taps falling off
 * the grid is ADDED to, or NULL.  A visibility with a non-finite
 * coordinate drops all of its taps; non-finite values propagate.
 * 0 <= m <= max_vis.  Fails with WS_BAD_STATE after ws_fft_planes(). */
ws_status ws_grid_visibilities(ws_plan* plan, int64_t m, const double* uvw,
                               const void* vis, const float* weight,
                               int64_t* n_dropped_taps);

/* In-place, unnormalised, centred 2-D FFT of every plane (Eq. 2, inner
 * integral); direction +1 = exp(+2 pi i ...) (imaging), -1 = exp(-2 pi i
 * ...) (its adjoint).  The stack then holds transforms. */
ws_status ws_fft_planes(ws_plan* plan, int32_t direction);

/* w-correction and plane reduction (Eq. 2, outer integral):
 * image[q][p] += sum_k F_k[q][p] exp(+2 pi i w_k (n_pq - 1)), reading the
 * transformed stack.  image: device [nv][nu] complex, same precision as the
 * plan.  The caller zeroes the image before the first accumulation.
 * Needs a transformed stack (after ws_fft_planes): on an empty plan it adds
 * nothing and returns WS_OK; on gridded, untransformed planes it fails with
 * WS_BAD_STATE. */
ws_status ws_wcorrect_accumulate(ws_plan* plan, void* image);

/* Fused form of ws_fft_planes(+1) followed by ws_wcorrect_accumulate():
 * the last FFT stage, the screen and the plane sum run in one pass that
 * never writes the transformed planes back.  Same result to rounding.  It
 * images the stack as the gridding calls since the last reset left it:
 * column strips (tile-wide column ranges of one plane) that none of those
 * calls reached hold zeros and are not transformed or read (a caller that
 * writes into the stack itself uses ws_fft_planes and
 * ws_wcorrect_accumulate instead).  It consumes the stack: afterwards the
 * plan is reset (empty).  Fails with WS_BAD_STATE after ws_fft_planes(). */
ws_status ws_image_accumulate(ws_plan* plan, void* image);

/* Gridding (Eq. 3) and imaging (Eq. 2) in one call, with the stack as
 * scratch: the same image as ws_grid_visibilities() followed by
 * ws_image_accumulate(), to rounding.  Because no caller observes the
 * stack in between, tiles that receive no visibility are not zeroed when
 * the imaging pass can take them as zero by itself (tile edge 64, nu in
 * [512, 4096], nv <= 4096); otherwise the call does exactly the two steps.
 * Arguments as for those two calls; the plan must be empty (after init or
 * ws_plan_reset(), else WS_BAD_STATE) and is empty afterwards, with the
 * stack's contents unspecified. */
ws_status ws_grid_image(ws_plan* plan, int64_t m, const double* uvw,
                        const void* vis, const float* weight, void* image,
                        int64_t* n_dropped_taps);

/* Baseline-major gridding (Sec. 2, data structures: (u, v, w) per baseline
 * and measurement time, several visibilities per baseline from the
 * frequency channels and polarisations, a weight per measurement and
 * polarisation; Sec. 3.4.2: one GPU thread per measurement convolves all
 * of its frequencies and polarisations; Sec. 5: full multi-wavelength and
 * polarisation support as future work).  The same gridding as
 * ws_grid_visibilities over m = nrows * nchan visibilities, entry
 * r * nchan + c for row r (one baseline at one time) and channel c:
 *   uvw_m     device float64 [nrows][3], baseline coordinates in METRES;
 *             the visibility of channel c sits at uvw_m[r] * (freq_hz[c] /
 *             c0) wavelengths, c0 = 299792458 m/s (the scale formed first,
 *             then one product per coordinate, in FP64);
 *   freq_hz   device float64 [nchan], channel frequencies;
 *   vis       device complex64 (FP32 path) or complex128 (FP64 path)
 *             [nrows][nchan][npol], the npol correlations;
 *   weight    device float32 [nrows][npol] or NULL (unit);
 *   pol_coeff HOST float64 [npol][2] (re, im): coefficients a_p of the
 *             gridded value sum_p a_p weight[r][p] vis[r][c][p], formed in
 *             FP64 and rounded to the path precision (a Stokes parameter
 *             from linear or circular correlations, e.g. I = (XX + YY)/2:
 *             a = (1/2, 0, 0, 1/2)); copied before the call returns;
 *   1 <= npol <= 4, nchan >= 1, 0 <= nrows * nchan <= max_vis.
 * n_dropped_taps: as for ws_grid_visibilities. */
ws_status ws_grid_rows(ws_plan* plan, int64_t nrows, int32_t nchan,
                       int32_t npol, const double* uvw_m,
                       const double* freq_hz, const void* vis,
                       const float* weight, const double* pol_coeff,
                       int64_t* n_dropped_taps);

/* Baseline-major input through the one-call path: the image of
 * ws_grid_image for the visibilities ws_grid_rows defines.  Arguments as
 * for those two calls; the plan must be empty and is empty afterwards. */
ws_status ws_grid_image_rows(ws_plan* plan, int64_t nrows, int32_t nchan,
                             int32_t npol, const double* uvw_m,
                             const double* freq_hz, const void* vis,
                             const float* weight, const double* pol_coeff,
                             void* image, int64_t* n_dropped_taps);

/* Degridding (Sec. 5 future work): the exact adjoint of gridding, FFT(+1)
 * and w-correction.  vis_out[m] = w_m sum_taps c g g Q_k(m)[j][i] with
 * Q_k = FFT(-1)(conj(screen_k) * X).  image: device [nv][nu], complex in the
 * plan's precision, or real (float32 on the FP32 path, float64 on the FP64
 * path) when image_is_real != 0.  vis_out: device [m] complex, every entry
 * overwritten; a visibility with no tap on the grid (a non-finite
 * coordinate, or a footprint wholly off the grid) gets 0.
 * Uses the plane stack as scratch and leaves the plan reset (empty). */
ws_status ws_degrid(ws_plan* plan, const void* image, int32_t image_is_real,
                    int64_t m, const double* uvw, const float* weight,
                    void* vis_out);

/* ---- imaging major cycle --------------------------------------------------
 * Deconvolution follows imaging in the processing chain of Sec. 1: CLEAN
 * (Hogbom's image-plane loop) inside the major / minor cycle split of Clark
 * and Schwab, where the model is subtracted from the visibilities between
 * minor cycles.  These calls run one such cycle on the plan's kernels;
 * images here are REAL (float32 on the FP32 path, float64 on the FP64
 * path), [nv][nu]; the visibilities should be Hermitian-paired so that the
 * images they give are real (the imaginary parts are dropped).  A caller
 * loops: ws_dirty_beam once, then per major cycle ws_residual_image and
 * ws_clean_minor (the Python driver is paper_2301_06061_amd.clean). */

/* Dirty beam: beam = Re(I(1)) / beta, I(1) the image (ws_grid_image) of unit
 * visibilities with the given weights, beta its value at the centre pixel
 * (nv/2, nu/2), written to the device double *beta.  image_scratch: device
 * complex [nv][nu] of the plan precision, overwritten.  The plan must be
 * empty and is empty afterwards. */
ws_status ws_dirty_beam(ws_plan* plan, int64_t m, const double* uvw,
                        const float* weight, void* image_scratch, void* beam,
                        double* beta);

/* Residual image of a model: residual = Re(I(V - A model)) / beta, with A
 * model = ws_degrid(model, unit weights) (the prediction of the sky model's
 * visibilities) and I the image with the given weights (ws_grid_image).
 * model: device real [nv][nu]; beta: device double (from ws_dirty_beam);
 * vis_scratch: device complex [m] (receives V - A model); image_scratch:
 * device complex [nv][nu]; residual: device real [nv][nu], overwritten.
 * The plan is empty afterwards. */
ws_status ws_residual_image(ws_plan* plan, int64_t m, const double* uvw,
                            const void* vis, const float* weight,
                            const void* model, const double* beta,
                            void* vis_scratch, void* image_scratch,
                            void* residual);

/* Hogbom minor cycle on device real images: up to niter steps, each taking
 * the pixel of largest |residual| (the lowest index q * nu + p on ties;
 * non-finite pixels are never taken), stopping before a peak below
 * threshold; a step adds gain * peak to model at that pixel and subtracts
 * gain * peak times the beam centred there (beam[q - q* + nv/2][p - p* +
 * nu/2] where that index lies on the grid) from the residual.  beam is
 * normalised (1 at its centre); residual and model are updated in place.
 * picks: device int32 [niter] receiving the pixel index of each step, or
 * NULL; n_done: device int32 receiving the number of steps, or NULL.
 * 0 < gain <= 1, threshold >= 0.  All decisions stay on the device (no
 * host synchronisation inside the cycle); the state lives in the plan's
 * workspace, so the plan's other calls must not run concurrently. */
ws_status ws_clean_minor(ws_plan* plan, void* residual, const void* beam,
                         void* model, int32_t niter, double gain,
                         double threshold, int32_t* picks, int32_t* n_done);

/* ---- allocation-free imaging ---------------------------------------------
 * For callers that cannot allocate device memory at all: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same dirty image as ws_grid_init + ws_grid_image (same kernels, same
 * arguments), with no plan and no caller buffers besides the inputs and the
 * image: the plane stack and the workspace live in a static device array of
 * WS_NOALLOC_SCRATCH_BYTES bytes inside the library (one per GPU, held until
 * the process ends).  The call allocates nothing, host or device.
 *   params, m, uvw, vis, weight, n_dropped_taps: as for ws_grid_image;
 *   image: device [nv][nu] complex of the plan precision, ADDED to;
 *   hip_stream: the stream to enqueue on (NULL = the null stream).
 * A problem whose stack plus workspace (ws_workspace_bytes with max_vis =
 * m, the stack rounded up to 256 bytes) exceeds WS_NOALLOC_SCRATCH_BYTES is
 * refused with WS_WORKSPACE_TOO_SMALL before any device work.  Every call
 * on one GPU shares that GPU's scratch: calls that overlap in time on one
 * GPU (two streams, two threads) race and give wrong images; serialise
 * them.  The scratch keeps the last call's contents; each call clears what
 * it needs. */
#define WS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
ws_status ws_grid_image_noalloc(const ws_params* params, int64_t m,
                                const double* uvw, const void* vis,
                                const float* weight, void* image,
                                int64_t* n_dropped_taps, void* hip_stream);

/* Start a new image: the stack counts as empty again (cleared lazily). */
ws_status ws_plan_reset(ws_plan* plan);

/* Replace the stream later calls enqueue on (a hipStream_t, NULL = null). */
ws_status ws_set_stream(ws_plan* plan, void* hip_stream);

/* Wait for all work the plan enqueued; reports asynchronous HIP errors. */
ws_status ws_sync(ws_plan* plan);

/* Work counts of the last call that binned visibilities on this plan
 * (ws_grid_visibilities, ws_grid_image, ws_degrid, or the plan's part of a
 * batch): out[0] the tile edge in cells, out[1] tiles (of all planes) that
 * received records, out[2] tiles that received none, out[3] tiles split
 * into several work items, out[4] the further items of split tiles, out[5]
 * the column strips (tile-wide column ranges of one plane) marked as
 * holding records since the last reset (gridding; unspecified after
 * ws_degrid), out[6] the records read by all work items together (a
 * record is read by its own tile and by each neighbouring tile its
 * footprint reaches; degridding: one read per record).  Waits for the
 * plan's stream.  Diagnostics of the binning (Sec. 3.4); before any such
 * call the counts are unspecified. */
ws_status ws_tile_stats(ws_plan* plan, int64_t out[7]);

/* Per-kernel timing: when enabled, every kernel launch of the plan is
 * bracketed by HIP events on the plan's stream and its duration is added
 * to a per-kernel total.  ws_kernel_times() waits for the plan's stream,
 * then fills up to cap entries of names (static strings), total ms and
 * launch counts, and returns the number of kernels in *n; it also resets
 * the totals when reset != 0. */
ws_status ws_set_profiling(ws_plan* plan, int32_t enable);
ws_status ws_kernel_times(ws_plan* plan, int32_t cap, const char** names,
                          double* total_ms, int64_t* launches, int32_t* n,
                          int32_t reset);

/* ---- batches: many independent images in one launch sequence ----------
 * Many frequency channels or observations, each with its own plan (grid
 * size, planes, w range, visibility count), imaged together: every plan's
 * binning kernels, then ONE persistent gridding kernel draining a single
 * queue that holds the (tile, chunk) work items of all plans, then each
 * plan's FFT, w-screen and plane sum.  The paper's GPU thread loops over
 * the channels of one baseline (Sec. 3.4.2); here channels are separate
 * records of separate plans sharing one gridding launch.  All plans of a
 * batch share precision, kernel support and device; the batch runs on the
 * stream of plans[0], which every plan then uses. */
typedef struct ws_batch ws_batch;

/* Device workspace of a batch of n plans (1 <= n <= 64).  Host only. */
ws_status ws_batch_workspace_bytes(int32_t n, size_t* work_bytes);

/* Build a batch over n existing plans and a caller-owned, 256-byte aligned
 * device workspace (copies a small job table into it).  The plans and the
 * workspace must outlive the batch. */
ws_status ws_batch_create(int32_t n, ws_plan* const* plans, void* work,
                          size_t work_bytes, ws_batch** out);

/* One dirty image per plan: images[i] += image of the m[i] visibilities
 * uvw[i], vis[i], weight[i] (weight may be NULL, or any weight[i] NULL).
 * The arrays are host arrays of n entries holding device pointers.  The
 * plans are reset before and after, and their stacks are scratch: when
 * every plan meets the conditions of ws_grid_image for leaving tiles
 * without visibilities unwritten, the batch leaves them unwritten too. */
ws_status ws_batch_image(ws_batch* batch, const int64_t* m,
                         const double* const* uvw, const void* const* vis,
                         const float* const* weight, void* const* images);

/* Record ws_batch_image with exactly these arguments into a HIP graph by
 * stream capture (the batch stream must not be the null stream); nothing
 * runs until ws_batch_replay.  The buffers must stay allocated; their
 * contents may change between replays (m[i] and the pointers may not). */
ws_status ws_batch_capture(ws_batch* batch, const int64_t* m,
                           const double* const* uvw, const void* const* vis,
                           const float* const* weight, void* const* images);

/* Launch the captured graph once on the batch stream. */
ws_status ws_batch_replay(ws_batch* batch);

void ws_batch_destroy(ws_batch* batch);

void ws_plan_destroy(ws_plan* plan);
const char* ws_status_string(ws_status status);
const char* ws_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* WSTACK_H */
