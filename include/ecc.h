/*
 * libecc — spatially adaptive ("extended") correlation and convolution on one MI355X
 * (gfx950) GPU, after "Efficient Spatially Adaptive Convolution and Correlation"
 * (arXiv 2006.13188).
 *
 * Problem statement (Sec. 2): a signal H, a filter F and a transformation field T that
 * says how F is transformed at every pixel. Extended correlation (Sec. 2.1, eq.
 * Def-ECorr) gathers: y(p) = sum_q H(q) conj((T(p)F)(q - p)). Extended convolution
 * (Sec. 2.2, eq. Def-EConv) scatters: y(p) = sum_q H(q) (T(q)F)(p - q).
 * For 2D rotation the filter is split into angular components F_k(r, phi) =
 * f_k(r) e^{i k phi}, k = -K..K (Sec. 4.1, band-limited as in Sec. 4.3); rotating by
 * theta multiplies F_k by e^{-i k theta}, so the correlation is
 * sum_k e^{i k theta(p)} (H star F_k)(p) and the convolution is
 * sum_k (H e^{-i k theta}) * F_k. For the scale group (Sec. 8) the components are
 * Fourier modes in log r.
 *
 * Conventions shared by every call:
 *  - Images are row-major float32, ny rows by nx columns, row stride `ld` elements
 *    (ld >= nx); x = column (right), y = row (down); angles are atan2(dy, dx) radians.
 *  - Components are complex64 stored as interleaved (re, im) float pairs, layout
 *    [k][row][col] with k = 0..K and an S x S window centred at (R, R), R = (S-1)/2.
 *  - Filters are real, so F_{-k} = conj(F_k) and only k = 0..K are stored.
 *  - Zero boundary: H is zero outside the image; outputs have the image's size.
 *  - Every pointer marked "device" is a HIP device pointer owned by the caller; it must
 *    stay valid until the work enqueued on `stream` has completed. `stream` is a
 *    hipStream_t (NULL = the null stream). Calls enqueue work and return without
 *    waiting, except plan creation, which may wait for its own set-up.
 *  - Every call returns an ecc_status. Arguments are validated before anything is
 *    enqueued, so a failed call leaves outputs untouched; ecc_last_error gives the
 *    message (thread-local). No call aborts, throws or prints.
 */
#ifndef ECC_H
#define ECC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ECC_OK = 0,
  ECC_ERR_INVALID_ARGUMENT = 1,
  ECC_ERR_UNSUPPORTED = 2,
  ECC_ERR_OUT_OF_MEMORY = 3,
  ECC_ERR_HIP = 4,
  ECC_ERR_PLAN_MISMATCH = 5,
  ECC_ERR_INTERNAL = 6
} ecc_status;

typedef enum {
  ECC_GROUP_ROTATION = 0,
  ECC_GROUP_SCALE = 1,
  ECC_GROUP_ROTATION_SCALE = 2   /* joint rotation and scale fields: ecc_joint_convolution */
} ecc_group;
typedef enum { ECC_CORRELATION = 0, ECC_CONVOLUTION = 1 } ecc_op;
typedef enum {
  ECC_PREC_FP32 = 0,
  ECC_PREC_MFMA_FP16_HILO = 1,
  ECC_PREC_MFMA_BF16_HILO = 2
} ecc_precision;

/* How extended correlations are evaluated (both reach the same result up to rounding).
 * TWO_PASS: the paper's form (Sec. 4): one zero-padded FFT correlation per component over
 * the whole image, P >= n + R (ecc_fft_size), with the per-pixel combination fused into
 * the last inverse pass. TILED: overlap-save blocks: each T x T block of outputs is computed from
 * an N x N window (N - 2R >= T) entirely on chip, per component, then combined per
 * pixel (block shapes exist for R <= 56). AUTO takes TILED when a block shape with side
 * T >= 2R exists, choosing among those by a cost model (measured when the autotuner is
 * on). Correlation, convolution, scale smoothing, matching and the adjoint have both
 * forms (ecc_extended_save writes the two-pass stack and so always runs TWO_PASS).
 * DIRECT: ecc_extended (both ops, and batch instances) evaluated as spatial sums without
 * transforms, G_c(p) = sum_x H(p + x) conj(F_c(x)) for the correlation and
 * sum_x (H e^{-i c alpha})(p - x) F_c(x) for the convolution: 2 U S^2 multiply-adds per
 * pixel, for filter sides S = 3..15 (UNSUPPORTED for larger filters); every other call
 * treats DIRECT as AUTO. AUTO takes DIRECT when its estimated time is below the block
 * path's (the smallest filters and band limits). */
typedef enum {
  ECC_STRATEGY_AUTO = 0,
  ECC_STRATEGY_TWO_PASS = 1,
  ECC_STRATEGY_TILED = 2,
  ECC_STRATEGY_DIRECT = 3
} ecc_strategy;

typedef struct ecc_context_s* ecc_context;
typedef struct ecc_filter_plan_s* ecc_filter_plan;
typedef struct ecc_batch_plan_s* ecc_batch_plan;

/* Parameters of the transformation group. Zero fields take the defaults shown. */
typedef struct {
  int angular_samples;        /* rotation: angular samples M per radius; 0 = smallest power
                                 of two >= max(8(2K+1), 4 ceil(2 pi R))                   */
  double sigma0;              /* scale: base Gaussian width in pixels at s = 1 (1.0)       */
  double scale_min;           /* scale: smallest per-pixel scale (1.0)                     */
  double scale_max;           /* scale: largest per-pixel scale (8.0)                      */
  int scale_components;       /* scale: number of log-radial Fourier modes n (24)          */
  double scale_period_factor; /* scale: period of the log-radial expansion relative to the
                                 range of ln|x| - ln s met on the grid (1.5)              */
} ecc_group_params;

/* ---------------------------------------------------------------- context */

/* Creates a context bound to HIP device `hip_device` (made current for the call).
 * The context owns twiddle tables, scratch workspace and size choices. One context
 * must not be used by two host threads at once. One host thread may use it on several
 * streams: a call that uses the workspace on a stream other than the previous such
 * call's first waits (on the device) for that call's last kernel. Errors:
 * INVALID_ARGUMENT (bad device or NULL out), HIP. */
ecc_status ecc_create(int hip_device, ecc_context* out);
/* Waits for the device, then frees everything the context owns, including filter plans
 * made from it that are still alive (their handles must not be used afterwards). NULL
 * is accepted. */
ecc_status ecc_destroy(ecc_context ctx);
const char* ecc_status_string(ecc_status s);
/* Message of the last failed call on this host thread ("" if none). The text is kept
 * per host thread, not per context: `ctx` may be NULL (as after a failed ecc_create) and
 * does not select among contexts; the pointer stays valid until the thread's next failed
 * call. */
const char* ecc_last_error(ecc_context ctx);

/* FFT size of the two-pass path for an image side n and filter radius R: the smallest
 * 7-smooth integer >= max(n + R, 2R + 1, 16) (zero-boundary linear correlation needs
 * >= n + R; the filter window of 2R + 1 taps is placed without wrapping onto itself; the
 * floor of 16 keeps every transform at two passes or more) whose transforms every
 * two-pass kernel takes (a length with more butterflies per pass than they handle is
 * passed over for the next, up to 4096; beyond that the smallest). With the autotuner on
 * (ecc_set_autotune), the fastest of the 7-smooth sizes from that one up to 1/8 above it
 * (at most four), timed once per context and (n, R) as the two-pass form's forward
 * transform of an n x n signal; the first call for a pair may enqueue that timing. */
ecc_status ecc_fft_size(ecc_context ctx, int n, int R, int* P);
/* Enables (1) or disables (0) the autotuner. When enabled, the next forward call (or
 * ecc_describe) first times every compiled block shape of the tiled path on this device
 * (once per context, a few milliseconds); block shapes are then chosen from the measured
 * per-block costs instead of an operation count. */
ecc_status ecc_set_autotune(ecc_context ctx, int enable);
/* The autotuner's measurements as JSON text, to be kept between processes:
 *   {"device": "<architecture name>", "tile_cost": [[N, TV, a, b], ...],
 *    "fft_size": [[n, R, P], ...]}
 * with the time of one full wave of blocks of shape (N, TV) modelled as a + b U ms, and the
 * two-pass FFT sizes chosen so far (see ecc_fft_size; the list is optional on import).
 * ecc_autotune_export writes the text and its terminating NUL to buf (cap bytes) and the
 * text's length to *len; buf may be NULL to ask for the length. INVALID_ARGUMENT if the
 * context has not calibrated yet (enable the autotuner and make one call, or
 * ecc_describe) or buf is too small. ecc_autotune_import takes such text, checks that it
 * was measured on the same architecture and covers every compiled block shape, and marks
 * the context calibrated, so no measurement runs (INVALID_ARGUMENT otherwise; the
 * context is then unchanged). Neither call enqueues GPU work. */
ecc_status ecc_autotune_export(ecc_context ctx, char* buf, size_t cap, size_t* len);
ecc_status ecc_autotune_import(ecc_context ctx, const char* json);
/* Sets the evaluation strategy of later ecc_extended correlations on this context.
 * TILED with a filter radius that has no block shape fails with UNSUPPORTED at the call. */
ecc_status ecc_set_strategy(ecc_context ctx, ecc_strategy strategy);
/* Reports how ecc_extended(op, plan, ny x nx) would run on this context (for a
 * rotation-and-scale plan, op = ECC_CONVOLUTION only: how ecc_joint_convolution would run):
 * the strategy, the transform length (TILED: N; TWO_PASS: the column-direction size P_y;
 * DIRECT: 0) and the block side T (0 for TWO_PASS and DIRECT). Any output pointer may be NULL. Nothing is
 * enqueued, except the autotuner's one-time calibration when it is enabled and has not
 * run yet. */
ecc_status ecc_describe(ecc_context ctx, ecc_op op, ecc_filter_plan plan, int ny, int nx,
                        ecc_strategy* strategy, int* fft_size, int* block);

/* Measurement hook: while set, every forward call (ecc_extended, ecc_scale_smooth,
 * ecc_match_rotations) records events[0] on its stream before its first kernel and
 * events[i + 1] after its i-th kernel, for i + 1 < n. `events` holds n hipEvent_t
 * handles created by the caller and must stay valid while set; n = 0 or NULL clears
 * the hook. Kernel order: correlation = row FFT, column FFT, component column
 * transforms, row transforms + combination; convolution = modulated row FFTs, column
 * transforms + component sum, row transforms; matching as correlation with the angle
 * search in the last kernel. */
ecc_status ecc_set_stage_events(ecc_context ctx, void* const* events, int n);

/* ---------------------------------------------------------------- workspace */

/* The calls whose device workspace ecc_workspace_size reports. The first two values are
 * those of ecc_op (ecc_extended with that op). */
typedef enum {
  ECC_WS_EXTENDED_CORRELATION = 0, /* ecc_extended(ECC_CORRELATION, ...)                 */
  ECC_WS_EXTENDED_CONVOLUTION = 1, /* ecc_extended(ECC_CONVOLUTION, ...)                 */
  ECC_WS_SCALE_SMOOTH = 2,         /* ecc_scale_smooth (batch = 1)                       */
  ECC_WS_MATCH_ROTATIONS = 3,      /* ecc_match_rotations (batch = 1)                    */
  ECC_WS_BACKWARD_CONVOLUTION = 4, /* ecc_extended_backward(ECC_CONVOLUTION), no saved stack */
  ECC_WS_BACKWARD_CORRELATION = 5, /* ecc_extended_backward(ECC_CORRELATION)             */
  ECC_WS_NORMALIZED_CONVOLUTION = 6, /* ecc_normalized_convolution                       */
  ECC_WS_JOINT_CONVOLUTION = 7      /* ecc_joint_convolution (the normalised form's size) */
} ecc_ws_call;

/* Every context owns one device workspace, shared by its calls and grown on demand (a
 * call that needs more than is allocated waits for the device, frees it and allocates
 * the larger size). ecc_workspace_size reports, without enqueueing or allocating
 * anything, the bytes that `call` (an ecc_ws_call; ECC_CORRELATION and ECC_CONVOLUTION
 * mean ecc_extended with that op) needs for `batch` images of ny x nx with `plan` under
 * the context's current strategy: 0 for the on-chip block paths of the correlation and
 * of the convolution with 64- and 96-point blocks; the overlap-add regions of the
 * convolution with 128-point blocks, the normalised convolution and the scale smoothing;
 * the component stack of matching; the two-pass stacks otherwise. (The adjoints also allocate a temporary image when grad_signal is NULL.)
 * When the autotuner is enabled and has not run, this call runs it first (the choice of
 * block shape depends on it). Errors: INVALID_ARGUMENT, HIP. */
ecc_status ecc_workspace_size(ecc_context ctx, int call, ecc_filter_plan plan, int batch, int ny,
                              int nx, size_t* bytes);
/* Grows the context's workspace to at least `bytes` now (waiting for the device first if
 * a smaller workspace exists), so that later calls needing at most that much allocate
 * nothing. Errors: OUT_OF_MEMORY, HIP. */
ecc_status ecc_workspace_reserve(ecc_context ctx, size_t bytes);
/* Bytes of workspace the context currently holds. */
ecc_status ecc_workspace_allocated(ecc_context ctx, size_t* bytes);

/* ---------------------------------------------------------------- filter plans */

/* Rotation (Sec. 4.1, "Filter Decomposition"): `filter` is a device S x S float32 array
 * (S odd, 3 <= S <= 255), centre at (R, R). The plan samples it bilinearly (zero outside
 * the array) on every distinct grid radius 0 < rho <= R at M equispaced angles, takes
 * the angular DFT f_k(rho) = (1/M) sum_m F(rho, phi_m) e^{-i k phi_m} for k = 0..K
 * (0 <= K <= M/2 - 1), and stores F_k(x) = f_k(|x|) e^{i k phi(x)} on the disk |x| <= R
 * (F_0(0) = F(0), F_k(0) = 0 otherwise, zero outside the disk). All of this runs in
 * float64 on the GPU; components are kept in float64 and float32.
 * Scale (Sec. 8): `filter` must be NULL and S, K are ignored (pass 0); the plan builds
 * the log-radial components of a Gaussian from `gp` (see ecc_group_params): F_k(x) =
 * c_k e^{i omega_k (ln|x| - u_lo)}, k = 0..n/2, on the disk of radius
 * R = ceil(4 sigma0 scale_max).
 * Rotation and scale (the Conclusion's product group): `filter` as for rotation; the plan
 * decomposes it into modes F_{k,l}(x) = c_{k,l} e^{i k phi(x)} e^{i omega_l (ln|x| - u_lo)},
 * k = -K..K, l = -(n-1)/2..(n-1)/2 with n = gp->scale_components (odd; default 9),
 * omega_l = 2 pi l / L: the filter is sampled bilinearly (zero outside the disk |x| <= R)
 * at M angles on the log-radii e^{u_lo + j L / n}, u_lo = -ln scale_max, the angular DFT
 * gives f_k, and the n-point DFT over j of f_k(e^u) gives c_{k,l}, where
 * L = scale_period_factor (u_hi - u_lo), u_hi = ln R - ln scale_min, and on (u_hi, u_lo + L)
 * f_k(e^u) is replaced by a raised-cosine blend from its value at u_hi back to that at
 * u_lo (defaults: scale range [1, 2], factor 1.5). F_{k,l}(0) = F(0) for (0, 0), else 0.
 * The plan keeps the real filter's half set, k = 0 with l = 0..(n-1)/2 and k = 1..K with
 * every l: (K+1) n - (n-1)/2 components; only ecc_joint_convolution takes such plans.
 * `gp` may be NULL (defaults). Waits for `stream`. Errors: INVALID_ARGUMENT, UNSUPPORTED
 * (complex filters are not accepted by this signature), OUT_OF_MEMORY, HIP. */
ecc_status ecc_filter_plan_create(ecc_context ctx, ecc_group group, const float* filter,
                                  int S, int K, const ecc_group_params* gp, void* stream,
                                  ecc_filter_plan* out);
/* Plan from explicit components: `comps` is device complex64 (interleaved), (K+1) x S x S,
 * k = 0..K, as described above. For ECC_GROUP_SCALE the field angle and weights come
 * from `gp` as for ecc_filter_plan_create; ECC_GROUP_ROTATION_SCALE is not accepted
 * (INVALID_ARGUMENT). Waits for `stream`. */
ecc_status ecc_filter_plan_from_components(ecc_context ctx, ecc_group group, const float* comps,
                                           int S, int K, const ecc_group_params* gp,
                                           void* stream, ecc_filter_plan* out);
/* Number of components U a plan stores: K + 1 for rotation plans, n/2 + 1 for scale plans,
 * (K+1) n - (n-1)/2 for rotation-and-scale plans. */
ecc_status ecc_filter_plan_component_count(ecc_filter_plan plan, int* U);
/* Copies the plan's complex64 components (U x S x S, interleaved; U as
 * ecc_filter_plan_component_count reports) to device `out`. */
ecc_status ecc_filter_plan_get_components(ecc_filter_plan plan, float* out, void* stream);
/* Window size S, band limit K (components k = 0..K) and angular samples M of a plan. */
ecc_status ecc_filter_plan_info(ecc_filter_plan plan, int* S, int* K, int* M);
ecc_status ecc_filter_plan_destroy(ecc_filter_plan plan);

/* ---------------------------------------------------------------- forward operators */

/* Extended correlation (Sec. 2.1) or convolution (Sec. 2.2) of `batch` images.
 * signal, field, out: device float32, batch x ny x nx with row strides ld_* and image
 * stride ny * ld_*. field = theta(p) in radians (rotation plans) or s(p) > 0 (scale
 * plans; the phase is e^{-i omega_k ln s}). out must not alias an input.
 * Rotation: correlation y = Re sum_k w_k e^{i k theta} (H star F_k), convolution
 * y = Re sum_k w_k (H e^{-i k theta}) * F_k, with w_0 = 1, w_k = 2 (k and -k together).
 * Only ECC_PREC_FP32 is implemented. Errors: INVALID_ARGUMENT (sizes, strides, NULL,
 * aliasing, filter larger than the image), UNSUPPORTED (precision; or the two-pass
 * strategy where its transform length, ecc_fft_size(n, R), exceeds 4096 along rows: the
 * block strategy covers the largest images for radii up to 56), HIP. */
ecc_status ecc_extended(ecc_context ctx, ecc_op op, ecc_filter_plan plan, int batch, int ny,
                        int nx, const float* signal, int ld_signal, const float* field,
                        int ld_field, float* out, int ld_out, ecc_precision prec, void* stream);

/* Scale-adaptive smoothing (Sec. 8, eq. normalization with the normalised signal):
 * out = {H / s^2, s} * F divided by {1 / s^2, s} * F, for a scale plan.
 * signal, scale, out: device float32 ny x nx with the given row strides. The same call as
 * ecc_normalized_convolution with batch = 1 (see there for the strategies and workspace). */
ecc_status ecc_scale_smooth(ecc_context ctx, ecc_filter_plan plan, int ny, int nx,
                            const float* signal, int ld_signal, const float* scale,
                            int ld_scale, float* out, int ld_out, ecc_precision prec,
                            void* stream);

/* Normalised adaptive filtering (Sec. 8, eq. normalization): the extended convolution of
 * the signal divided, pixel by pixel, by the extended convolution of the constant signal
 * 1 (1 inside the image, 0 outside) with the same field, so that every output is the
 * weighted average of the contributions it receives. Rotation plans: the signal is used
 * as it is (rotations keep the filter's integral); with a long, narrow anisotropic filter
 * and the angle of a vector field on a noise image this is line-integral convolution.
 * Scale plans: the signal is first divided by s(q)^2 and the constant signal is 1/s^2
 * (the normalised signal of Sec. 8), which is ecc_scale_smooth.
 * signal, field, out: device float32, batch x ny x nx with row strides ld_* and image
 * stride ny * ld_*; out must not alias an input. Where the denominator is zero the
 * output is not finite. Block strategy (TILED / AUTO with a block shape): where the block
 * convolution would use 128-point transforms (filter radii above about 16), for plans
 * whose components have parity (every plan made by ecc_filter_plan_create), one
 * overlap-add launch transforms the (at most) 64 x 64 sources of each block for both
 * signals at once and writes its 128 x 128 region of (numerator, denominator) to the
 * context workspace; a second kernel adds the overlapping regions in a fixed order and
 * divides. Otherwise two launches of the block convolution (numerator, then the
 * denominator divided into it). Two-pass: both signals' transforms in one set of
 * kernels. Workspace: ecc_workspace_size with ECC_WS_NORMALIZED_CONVOLUTION.
 * Precision: ECC_PREC_FP32 everywhere; ECC_PREC_MFMA_FP16_HILO / ECC_PREC_MFMA_BF16_HILO
 * in the overlap-add kernel only (else UNSUPPORTED): the radix-16 passes of its forward
 * transforms (16-point DFTs of 16 lines at a time) run on the matrix cores with float16
 * (scaled per tile) or bfloat16 operands split into hi + lo parts, float32 accumulation;
 * everything else stays float32. Errors as for ecc_extended. */
ecc_status ecc_normalized_convolution(ecc_context ctx, ecc_filter_plan plan, int batch, int ny,
                                      int nx, const float* signal, int ld_signal, const float* field,
                                      int ld_field, float* out, int ld_out, ecc_precision prec,
                                      void* stream);

/* Extended convolution with joint rotation and scale fields (a rotation-and-scale plan):
 *   y = Re sum_c w_c (Hn e^{-i (k_c theta + omega_{l_c} ln s)}) * F_c,
 * i.e. every pixel q scatters Hn(q) times the filter rotated by theta(q) and scaled by s(q)
 * (band-limited as the plan's modes), with w = 1 for (0, 0) and 2 otherwise; Hn = H when
 * `normalized` is 0. With `normalized` nonzero the output is the normalised smoothing of
 * Sec. 8 for this group: Hn = H / s^2, divided by the same convolution of 1 / s^2.
 * signal, angle (radians), scale (> 0), out: device float32, batch x ny x nx with row
 * strides ld_* and image stride ny * ld_*; out must not alias an input. Strategy as for
 * ecc_extended's convolution (ecc_set_strategy, ecc_describe): by blocks, the block
 * convolution with the components taken scale mode by scale mode (the phase of a pixel is
 * seeded once per mode and advanced by e^{-i theta} within it; no workspace); else the
 * two-pass form (one zero-padded transform per component and signal; context workspace as
 * ECC_WS_JOINT_CONVOLUTION reports). The normalised form runs the numerator and the
 * denominator as two launches. Errors: INVALID_ARGUMENT (sizes, strides, NULL, aliasing,
 * a plan of another group), UNSUPPORTED (TILED strategy without a block shape),
 * OUT_OF_MEMORY, HIP. */
ecc_status ecc_joint_convolution(ecc_context ctx, ecc_filter_plan plan, int batch, int ny, int nx,
                                 const float* signal, int ld_signal, const float* angle, int ld_angle,
                                 const float* scale, int ld_scale, float* out, int ld_out,
                                 int normalized, void* stream);

/* Rotation-independent matching (Sec. 5 in band-limited form): the correlation
 * response at n_angles equispaced angles 2 pi m / n_angles,
 * C(p, m) = sum_k w_k Re(e^{2 pi i k m / n_angles} (H star F_k)(p)); best_score = max_m C,
 * best_index = the smallest maximising m. 2K+1 <= n_angles <= 64.
 * signal: device float32 ny x nx (stride ld); best_score (float32) and best_index
 * (int32): device ny x nx with stride ld_out.
 * With a block shape (TILED / AUTO strategy) the components are computed block by block
 * into a stack in the context's workspace (K+1 planes of ny nx complex64 values, each
 * padded by less than 1.5 KiB) and the
 * angle search runs in the precision `prec`: ECC_PREC_FP32 (float32; for n_angles = 64
 * and K <= 31 a length-64 inverse DFT over k per pixel, else the dense product of the
 * angle table with the components), ECC_PREC_MFMA_FP16_HILO (the dense product on matrix
 * cores, float16 hi + lo operands, float32 accumulation; ~1e-6 relative),
 * ECC_PREC_MFMA_BF16_HILO (bfloat16 hi + lo; ~1e-5 relative). The two-pass strategy
 * supports ECC_PREC_FP32 only (else UNSUPPORTED). */
ecc_status ecc_match_rotations(ecc_context ctx, ecc_filter_plan plan, int ny, int nx,
                               const float* signal, int ld, int n_angles, float* best_score,
                               int* best_index, int ld_out, ecc_precision prec, void* stream);

/* Variant of ecc_match_rotations for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): same
 * arguments, same results, and it calls no hipMalloc, hipFree or allocating routine.
 * The component stack goes through a fixed 64 MiB device array of the library (one per
 * GPU, held until the process ends) instead of the context workspace, one band of block
 * rows at a time: for each band the stack kernel writes the band's K+1 planes and the
 * angle search reads them back. Every call on one GPU shares that array, whatever the
 * context: calls that overlap on one GPU (two host threads, or two streams without an
 * ordering between them) race and give wrong results. Nothing in the array needs to
 * start at zero (every band is fully written before it is read).
 * Preconditions (else ECC_ERR_UNSUPPORTED, nothing enqueued): a block shape exists for
 * the filter radius under the context's strategy; the plan's block spectra and angle
 * table for this image size and n_angles exist, i.e. ecc_match_rotations has run once
 * with the same plan, size and n_angles; if the autotuner is on, it has calibrated.
 * One block row of the stack, K+1 planes of T * nx complex64 values (T = the block side,
 * 64 for the 63 x 63 pattern) each padded by less than 1.5 KiB, must fit in 64 MiB, else
 * ECC_ERR_INVALID_ARGUMENT. */
ecc_status ecc_match_rotations_noalloc(ecc_context ctx, ecc_filter_plan plan, int ny, int nx,
                                       const float* signal, int ld, int n_angles, float* best_score,
                                       int* best_index, int ld_out, ecc_precision prec,
                                       void* stream);

/* ---------------------------------------------------------------- pattern detection */
/* The steps of pattern detection by extended convolution (Sec. 5): the target image gives
 * the signal and the field, the pattern gives the filter by voting, the extended
 * convolution (ecc_extended, ECC_CONVOLUTION, with a plan of that filter) makes every
 * pixel vote for the centres of rotated copies of the pattern, and the peaks of the
 * response are the detections. */

/* Signal and field of an image (eq. signal, eq. theta): magnitude = |grad I| and
 * angle = atan2(dI/dy, dI/dx) (radians, y = row, x = column), with central differences
 * inside and one-sided differences on the first and last row and column. image,
 * magnitude, angle: device float32, batch x ny x nx (row strides ld_image / ld_out, image
 * strides ny * ld). ny, nx >= 2. Outputs must not alias each other or the image.
 * Errors: INVALID_ARGUMENT, HIP. */
ecc_status ecc_gradient_field(ecc_context ctx, int batch, int ny, int nx, const float* image,
                              int ld_image, float* magnitude, float* angle, int ld_out,
                              void* stream);
/* Consensus filter of a pattern (eq. opt_filt; appendix "Defining Optimal Filters"): every
 * pixel x of the S x S pattern P (device float32, S odd, 3 <= S <= 255) within the disk
 * |x - c| <= R = (S-1)/2 around its centre c votes with weight |grad P(x)| (gradients as in
 * ecc_gradient_field) for the position of c seen from the frame at x whose first axis is
 * the gradient direction, R_{-theta_P(x)} (c - x); a vote is split bilinearly over the four
 * surrounding bins and dropped outside the window. `filter`: device float32 S x S, centre
 * at (R, R), ready for ecc_filter_plan_create. Computed in float64 (each bin sums its votes
 * in raster order: the same result on every run) and rounded once. Uses the context
 * workspace (24 S^2 bytes). Errors: INVALID_ARGUMENT, OUT_OF_MEMORY, HIP. */
ecc_status ecc_voting_filter(ecc_context ctx, int S, const float* pattern, float* filter,
                             void* stream);
/* Peaks of a response (device float32 ny x nx, stride ld): pixels whose value is >= the
 * threshold (`threshold` itself, or `threshold` times the largest value when `relative`
 * is nonzero; then 0 < threshold <= 1) and is not exceeded within the (2 radius + 1)^2
 * window around them, ties going to the first pixel in raster order. The strongest
 * min(max_peaks, number of peaks) are written to rows, cols (device int32) and values
 * (device float32) by decreasing value (ties by raster index); `count` (device int32)
 * receives their number. Deterministic. Uses the context workspace: 16 bytes per key
 * slot (one per (radius+1)^2 cell of each 64 x 16 pixel block for radius <= 32, one per
 * radius+1 pixels of each 256-pixel row segment above) plus the sort's temporary storage.
 * Errors: INVALID_ARGUMENT, OUT_OF_MEMORY, HIP. */
ecc_status ecc_find_peaks(ecc_context ctx, int ny, int nx, const float* response, int ld,
                          int radius, float threshold, int relative, int max_peaks, int* rows,
                          int* cols, float* values, int* count, void* stream);

/* ---------------------------------------------------------------- adjoint */

/* Gradients of the rotation-plan extended convolution y = Re sum_k w_k (H e^{-ik theta}) * F_k
 * with respect to H, theta and the components, given grad_out = dL/dy (all images
 * batch x ny x nx, contiguous rows, ld = nx):
 *   grad_signal(q) = Re sum_k w_k e^{-ik theta(q)} A_k(q), A_k(q) = sum_x gbar(q+x) F_k(x)
 *   grad_field(q)  = H(q) sum_k w_k k Im(e^{-ik theta(q)} A_k(q))
 *   grad_comps_k(x) = w_k sum_b sum_p gbar_b(p) conj(H_b(p-x) e^{-ik theta_b(p-x)})
 *                     (summed over the batch in a fixed order; complex64 (K+1) x S x S)
 * Any of grad_signal, grad_field, grad_comps may be NULL (not computed). `saved` is NULL
 * (recompute the modulated-signal stack) or device memory of
 * ecc_backward_saved_size() bytes filled by ecc_extended_save(). With the block strategy
 * (a block shape exists for the radius) grad_signal and grad_field come from one on-chip
 * correlation of grad_out with two outputs, and grad_comps from per-block lag sums
 * (context workspace) added in a fixed order; `saved` is then not read.
 * ECC_CORRELATION (y = Re sum_k w_k e^{ik theta} (H star F_k), G_k = H star F_k; `saved`
 * must be NULL):
 *   grad_signal = Re sum_k w_k (gbar e^{-ik theta}) * F_k (the forward convolution of gbar)
 *   grad_field  = -gbar sum_k w_k k Im(e^{ik theta} G_k)
 *   grad_comps_k(x) = w_k sum_b sum_p gbar_b(p) e^{ik theta_b(p)} H_b(p + x)
 * (the forward correlation's second output, and the convolution adjoint's filter part with
 * the signal and grad_out exchanged). */
ecc_status ecc_extended_backward(ecc_context ctx, ecc_op op, ecc_filter_plan plan, int batch,
                                 int ny, int nx, const float* signal, const float* field,
                                 const float* grad_out, float* grad_signal, float* grad_comps,
                                 float* grad_field, void* saved, void* stream);
/* Bytes of the stack saved by the forward pass for ecc_extended_backward: 0 when the
 * backward would not read one, i.e. when its filter gradient runs on chip (a block shape
 * exists for the radius under the context's strategy; then the backward recomputes what
 * it needs per block and a saving forward would only cost time and memory). Otherwise
 * batch * (K+1) * ny * P_x complex64 values (P_x = ecc_fft_size(nx, R)). */
ecc_status ecc_backward_saved_size(ecc_context ctx, ecc_filter_plan plan, int batch, int ny,
                                   int nx, size_t* bytes);
/* Forward extended convolution that also writes the per-component row spectra of the
 * modulated signal into `saved` (ecc_backward_saved_size bytes, device). Always runs the
 * two-pass form (whose intermediate the stack is); equal to ecc_extended up to rounding. */
ecc_status ecc_extended_save(ecc_context ctx, ecc_filter_plan plan, int batch, int ny, int nx,
                             const float* signal, const float* field, float* out, void* saved,
                             void* stream);

/* ---------------------------------------------------------------- batches */

/* One independent extended correlation of a batch (each instance one image with its own
 * filter plan, size and fields). Pointers are device float32 arrays owned by the caller,
 * rows of nx values with the given strides (in elements). */
typedef struct {
  ecc_op op;               /* ECC_CORRELATION (others run through the per-call path) */
  ecc_filter_plan plan;
  int ny, nx;
  const float* signal;
  int ld_signal;
  const float* field;
  int ld_field;
  float* out;
  int ld_out;
} ecc_instance;

/* Flags of ecc_batch_plan_create. */
#define ECC_BATCH_AUTOTUNE 1     /* time every block shape on this device first (once per
                                    context) and choose shapes from the measured costs */
#define ECC_BATCH_PERSISTENT 2   /* as many workgroups as fit on the device, each taking
                                    blocks from a device counter, instead of one workgroup
                                    per block; executions of one such plan must not
                                    overlap (they share the counter) */

/* Builds a batch plan: every instance that has a block shape (tiled path, the filter's
 * radius R <= 56; correlations and convolutions) is split into blocks; blocks of the same
 * op, shape and form go into one kernel launch, ordered longest first, and the launches
 * are captured once into a HIP graph as parallel branches. Instances without a block shape
 * are kept for the per-call path. Correlations take the direct sums (ECC_STRATEGY_DIRECT)
 * as a single call would: forced under DIRECT for every filter side that has a kernel
 * (larger filters then keep their block shapes), chosen by the time model under AUTO.
 * Convolution and direct launches always take the item table (one workgroup per block),
 * also under ECC_BATCH_PERSISTENT. Plans must outlive the batch
 * plan. Errors: INVALID_ARGUMENT (as ecc_extended for any instance), HIP. */
ecc_status ecc_batch_plan_create(ecc_context ctx, const ecc_instance* inst, int n, int flags,
                                 ecc_batch_plan* out);
/* Replaces the instances' pointers and strides (same count, ops, plans and sizes as at
 * creation; checked). Synchronous: waits for the last ecc_batch_execute of this plan to
 * finish (on whatever stream it was enqueued), then returns after the new descriptors
 * are on the device. */
ecc_status ecc_batch_update(ecc_batch_plan bp, const ecc_instance* inst, int n);
/* Runs the whole batch on `stream`: one graph launch for the tiled instances, then the
 * remaining instances one call each. */
ecc_status ecc_batch_execute(ecc_batch_plan bp, void* stream);
/* Number of instances in the graph, kernel launches in the graph, and blocks. Any output
 * may be NULL. */
ecc_status ecc_batch_info(ecc_batch_plan bp, int* graph_instances, int* launches, int* blocks);
ecc_status ecc_batch_plan_destroy(ecc_batch_plan bp);

/* ---------------------------------------------------------------- steering in 3D (Sec. 9)
 *
 * Volumes are device float32 arrays [nz][ny][nx], contiguous. A volume plan holds the
 * spherical-harmonic components of a real filter (Sec. 9, "Filter Decomposition"): the
 * filter F (S x S x S, centre (R, R, R), R = (S - 1) / 2, voxel offset q = (x, y, z) =
 * (column, row, slice)) restricted to the ball |q| <= R, with
 * f_l^m(r) = integral over the unit sphere of F(r w) conj(Y_l^m(w)) at every grid radius,
 * by Gauss-Legendre quadrature in cos(theta) (M / 2 nodes) times M azimuths, M the
 * smallest power of two >= max(8 (2K + 1), 4 ceil(2 pi R)), F(r w) trilinear (zero
 * outside the array); Y_l^m orthonormal with the Condon-Shortley phase, polar angle from
 * +z, azimuth atan2(y, x). The plan's components are C_{l,m',m}(q) = f_l^m(|q|)
 * Y_l^{m'}(q / |q|) on the ball (the centre keeps F(0) in l = 0) for the half set of a
 * real filter, in the order l = 0..K; m' = 0 with m = 0..l; m' = 1..l with m = -l..l,
 * weights w = 1 for (l, 0, 0) and 2 otherwise: U = sum_l (2 l^2 + 2 l + 1) components. */
typedef struct ecc_volume_plan_s* ecc_volume_plan;

/* Builds a volume plan from device `filter` (float32 S^3, S odd, 3..63) for band limit
 * K (0..8). Computed on the device in float64; waits for `stream`. The plan belongs to the
 * context (freed with it if still alive). Errors: INVALID_ARGUMENT, OUT_OF_MEMORY, HIP. */
ecc_status ecc_volume_plan_create(ecc_context ctx, const float* filter, int S, int K, void* stream,
                                  ecc_volume_plan* out);
ecc_status ecc_volume_plan_destroy(ecc_volume_plan plan);
/* U (components) and M (azimuth samples of the decomposition); either may be NULL. */
ecc_status ecc_volume_plan_info(ecc_volume_plan plan, int* U, int* M);
/* Copies the components (device complex64, U x S^3 interleaved) to `comps`, the host
 * table (l, m', m) of every component to `table` (3 U ints) and the host weights to
 * `weights` (U floats); NULL skips an output. Waits for `stream`. */
ecc_status ecc_volume_plan_components(ecc_volume_plan plan, float* comps, int* table, float* weights,
                                      void* stream);
/* Extended correlation / convolution of a volume with a rotation field (Sec. 9; the
 * definitions of Sec. 2 on Z^3). The rotation at voxel p is R_p = Rz(alpha) Ry(beta)
 * Rz(gamma) (ZYZ Euler angles in radians, active, acting on (x, y, z)); a rotated filter
 * is (R F)(q) = F(R^{-1} q), so that Y_l^m(R^{-1} x) = sum_m' D^l_{m'm}(R) Y_l^{m'}(x) with
 * D^l_{m'm} = e^{-i m' alpha} d^l_{m'm}(beta) e^{-i m gamma} (Wigner's explicit sum).
 *   correlation: y(p) = sum_q H(p + q) (R_p F)(q) = sum_c w_c Re(D_c(R_p) (H star C_c)(p));
 *   convolution: y(p) = sum_q H(q) (R_q F)(p - q) = sum_c w_c Re(((H D_c(R_.)) * C_c)(p));
 * zero outside the volume. Correlation: one forward 3D transform of H, U products and U
 * inverse transforms, then the per-voxel Wigner-D combination; convolution: U modulated
 * signals and forward transforms, one weighted sum of products, one inverse. Transform
 * sizes P = smallest 7-smooth >= max(n + R, 2R + 1, 8) per axis; float32 arithmetic with float64
 * spectra (rounded once) and float64 Wigner-D. Context workspace: (2 U + 1) Pz Py Lx
 * complex64, Lx = Px rounded up to a multiple of 16 (ecc_volume_workspace_size); the plan
 * caches its spectra per (op, P) (U Pz Py Lx complex64). signal, alpha, beta, gamma, out: device float32 nz x ny x nx; out must not
 * alias an input. Errors: INVALID_ARGUMENT, UNSUPPORTED (a transform too long), OUT_OF_MEMORY,
 * HIP. */
ecc_status ecc_extended_3d(ecc_context ctx, ecc_op op, ecc_volume_plan plan, int nz, int ny, int nx,
                           const float* signal, const float* alpha, const float* beta, const float* gamma,
                           float* out, void* stream);
/* Bytes of context workspace ecc_extended_3d takes for these sizes. */
ecc_status ecc_volume_workspace_size(ecc_context ctx, ecc_volume_plan plan, int nz, int ny, int nx,
                                     size_t* bytes);

#ifdef __cplusplus
}
#endif
#endif /* ECC_H */
