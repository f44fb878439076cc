/*
 * bsf.h -- C ABI of libbsf, constant-cost space-variant elliptical filtering with
 * four-direction box splines on AMD Instinct MI355X (gfx950).
 *
 * The filter (Chaudhury, Munoz-Barrutia, Unser, "Fast adaptive elliptical filtering
 * using box splines"): every output pixel m is the projection of the image onto the
 * four-direction box spline with that pixel's own scale vector a(m) = (a1,a2,a3,a4)
 * (Section 6, the projections s[m]; Section 7 fixes N = 4 directions at 0, 45, 90 and
 * 135 degrees and phi = delta).  a_d is the length of the generating segment along
 * direction d in pixel units (Section 4, eq. generator), so the diagonal lags in
 * lattice steps are a_d/sqrt2 (Section 7, a'_j = a_j/sqrt2).  Order n >= 1 is the
 * n-fold self-convolution of the box spline (Section 4, closing remark); n = 1 is the
 * paper's 16-tap mesh (Table 1, eq. final_eqn).
 *
 * It is computed as in Section 7: a global pre-integrator (n-fold running sums along
 * (1,0), (1,1), (0,1), (-1,1), eq. RS) followed by a per-pixel localisation mesh of
 * (n+1)^4 finite-difference taps at offsets set by a(m), each tap interpolated with
 * the lattice box spline (eq. final_eqn).  Pre-integration runs per output tile on a
 * restart window that holds the support of every pixel of the tile; this gives the
 * same result in exact arithmetic and bounds the magnitudes the mesh cancels.
 *
 * Conventions
 *   - Images are row-major: element (k1, k2) (k1 = column) lives at base[k2*pitch + k1].
 *   - Pitches are in elements of the array they describe; scales are float32 and their
 *     pitch counts pixels (4 floats each).
 *   - Every pointer in a bsf_job is a device pointer owned by the caller.  Calls are
 *     asynchronous on the given stream (a hipStream_t passed as void*, NULL = default
 *     stream) and the caller keeps the buffers alive until the stream reaches them.
 *   - Samples enter the pre-integrator as exact integers: each tile scales its window by the
 *     power of two that makes every sample an integer of at most 53 bits (float samples
 *     finer than 2^-53 of the window's largest magnitude are rounded to that grid).  When
 *     the running sums of those integers would leave int64, the tile runs stage 1 and the
 *     mesh on K base-2^B digits of the samples and adds the results (the filter is linear).
 *   - No call throws.  Argument errors are reported synchronously; errors found by the
 *     kernels (scale values out of range, a window larger than the chip's LDS, integer
 *     range) set sticky device flags returned by bsf_get_device_error, and the affected
 *     pixels are written as NaN.
 */
#ifndef BSF_H
#define BSF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bsf_ctx bsf_ctx;

typedef enum {
    BSF_OK = 0,
    BSF_ERR_INVALID_ARG = 1,   /* bad size, pitch, order, dtype/path pair or null pointer */
    BSF_ERR_OUT_OF_MEMORY = 2, /* the workspace would exceed the context's limit         */
    BSF_ERR_HIP = 3,           /* a HIP runtime call failed; bsf_last_error has the text  */
    BSF_ERR_UNSUPPORTED = 4,   /* a restart window does not fit the on-chip memory        */
    BSF_ERR_SCALE_RANGE = 5,   /* a scale is not finite or lies outside [0.5, 1e4]        */
    BSF_ERR_RANGE = 6          /* a pre-integrated value left the exact integer range     */
} bsf_status;

typedef enum { BSF_U8 = 0, BSF_F32 = 1, BSF_F64 = 2 } bsf_dtype;

/* BSF_PATH_F64: output float64; mesh interpolation and accumulation in double-double,
 *   so the result matches the exact filter to a few float64 ulps.
 * BSF_PATH_F32_TILED: output float32; the same restart windows with the running sums
 *   and the mesh in plain float64 (no integer grid, no digit passes).  Its error is the
 *   mesh's cancellation times a few float64 roundings: below 1e-5 of the output's
 *   magnitude for orders 1-3 at every scale in [0.5, 32] that was measured, and about
 *   1e-7 at scales >= 1 (float32 rounding then dominates). */
typedef enum { BSF_PATH_F64 = 0, BSF_PATH_F32_TILED = 1 } bsf_path;

/* Boundary rule for samples outside the image (the paper leaves it open): clamp to
 * the nearest edge pixel, or zero. */
typedef enum { BSF_BORDER_CLAMP = 0, BSF_BORDER_ZERO = 1 } bsf_border;

typedef struct {
    int width, height;              /* >= 1                                              */
    bsf_dtype in_dtype;             /* u8, f32 or f64                                     */
    const void* in;                 /* [height][in_pitch] samples                         */
    ptrdiff_t in_pitch;             /* >= width                                           */
    const float* scales;            /* [height][scale_pitch][4] = (a1,a2,a3,a4) per pixel */
    ptrdiff_t scale_pitch;          /* >= width, in pixels                                */
    int order;                      /* n in {1, 2, 3}                                     */
    bsf_path path;
    bsf_border border;
    float a_max;                    /* an upper bound on every a_d (sizes on-chip windows;
                                       0 = reserve the largest window the chip allows)   */
    void* out;                      /* [height][out_pitch] float64 (F64) / float32 (F32) */
    ptrdiff_t out_pitch;            /* >= width                                           */
} bsf_job;

/* Create a context on HIP device `hip_device`.  `workspace_limit_bytes` caps the device
 * memory the context may hold for its own workspace (0 = 16 GiB): a ring of eight work
 * areas, so that calls on different streams can be in flight together, whose total stays
 * within the limit.  A call whose own work area would exceed the limit returns
 * BSF_ERR_OUT_OF_MEMORY.  The context owns its workspace and a small sticky error word; it
 * is used by one host thread at a time. */
bsf_status bsf_create(bsf_ctx** ctx, int hip_device, size_t workspace_limit_bytes);

/* Release everything the context owns.  Waits for nothing: synchronise first. */
bsf_status bsf_destroy(bsf_ctx* ctx);

/* Device work area one bsf_filter call on `job` needs, in bytes (host only, no device
 * needed).  It is computed with the launch plan bsf_filter makes, taking the LDS of an
 * MI355X conservatively, so it is never below what the call asks of its context's
 * workspace on such a device (0 when every tile's window fits half of a workgroup's LDS).
 * A workspace limit of at least this size lets the call run. */
bsf_status bsf_workspace_size(const bsf_job* job, size_t* bytes);

/* out[m] = s[m] for every pixel (Section 6 projections computed by the two steps of
 * Section 7).  Asynchronous on `stream`. */
bsf_status bsf_filter(bsf_ctx* ctx, const bsf_job* job, void* stream);

/* The same for `njobs` independent jobs of any sizes, orders and paths in one
 * persistent launch (a device work queue of tiles).  Each output is bitwise equal to
 * what bsf_filter writes for that job alone.  `jobs` is a host array. */
bsf_status bsf_filter_batched(bsf_ctx* ctx, const bsf_job* jobs, int njobs, void* stream);

/* Captured batched launches for serving loops (the batched form of bsf_filter_batched as a
 * replayable plan).  bsf_batch_plan_create allocates a plan's own work area for batches of up
 * to `max_jobs` jobs and `max_tiles` 16x16 tiles in total, all of whose scales are bounded by
 * `a_max`, and captures the whole launch sequence once as a HIP graph: the upload of the
 * batch's descriptors from the plan's pinned staging, the persistent tile kernels of every
 * (order, path) variant and tier (they read the batch's counts from device memory, so the
 * same graph serves any batch within the capacity), and the download of one error word per
 * job.  bsf_batch_plan_run fills the staging for `jobs` (host array; each job's a_max must be
 * set and at most the plan's) and replays the graph on `stream`; every output is bitwise
 * equal to what bsf_filter writes for that job alone.  A run first waits (on the host) until
 * the plan's previous run has finished, so a caller that wants runs to overlap uses one plan
 * per stream.  bsf_batch_plan_job_status waits for the last run and writes, for its first
 * `njobs` jobs (the order of the `jobs` array), the status the kernels found for that job
 * alone: BSF_OK, BSF_ERR_SCALE_RANGE, BSF_ERR_UNSUPPORTED or BSF_ERR_RANGE (whose outputs
 * hold NaN where the error struck).  The plan belongs to the context it was created on and is
 * used by one host thread at a time. */
typedef struct bsf_batch_plan bsf_batch_plan;
bsf_status bsf_batch_plan_create(bsf_ctx* ctx, int max_jobs, long long max_tiles, float a_max, bsf_batch_plan** plan);
bsf_status bsf_batch_plan_run(bsf_batch_plan* plan, const bsf_job* jobs, int njobs, void* stream);
bsf_status bsf_batch_plan_job_status(bsf_batch_plan* plan, int* status, int njobs);
bsf_status bsf_batch_plan_destroy(bsf_batch_plan* plan);

/* Continuous image models (Section 6): the image is f(x) = sum_k c[k] phi(x - k) with
 * phi = beta^model x beta^model, the centred unit-scale B-spline of degree `model` along x and
 * y, and every pixel gets the projection of f onto the four-direction box spline at its own
 * scales:  out[m] = sum_k c_ext[k] (phi * B_a(m))(m - k).  model = -1 is phi = delta, Section
 * 7's choice and exactly bsf_filter; model = 0 (piecewise-constant) and 1 (bilinear) need no
 * prefilter (b^model is the unit impulse, c = the samples).  The two steps of Section 6 are
 * unchanged except the interpolant of eq. mask, phi * beta_b: the box spline of
 * {l1^(model+2), l2, l3^(model+2), l4}, tabulated exactly like beta_b; the restart windows
 * also hold phi's extra (model+1)/2 of support.  Models 0 and 1 are provided at order 1 (the
 * paper's 16-tap mesh, Table 1); other (order, model) pairs return BSF_ERR_UNSUPPORTED.  Same
 * paths, borders, workspace and errors as bsf_filter. */
bsf_status bsf_filter_model(bsf_ctx* ctx, const bsf_job* job, int model, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same result as bsf_filter, bitwise,
 * with the call's work area (tile lists, counters, tier-3 window slices) in a fixed 32 MiB
 * array in device memory that the library holds on each GPU until the process ends.  The
 * call allocates nothing and never waits on the host.  The caller still passes the job's
 * inputs and output; the context supplies the device and the error word.  A job whose work
 * area cannot fit the array (16 bytes per 16x16 tile, about 2 million tiles, plus at least
 * one restart window slice when a window exceeds the chip's LDS) returns
 * BSF_ERR_OUT_OF_MEMORY synchronously.  Every call on one GPU shares that GPU's array, from
 * any context: calls that overlap on the device (other streams, other threads) race and
 * must be serialised by the caller.  Asynchronous on `stream`. */
bsf_status bsf_filter_noalloc(bsf_ctx* ctx, const bsf_job* job, void* stream);

/* Stage 1 alone, as a global pre-integrator (eq. RS applied n times per direction):
 * the unit-weight n-fold running sums of the window  f_ext[y0 + r][x0 + c],
 * 0 <= r < hq, 0 <= c < wq  (f_ext = the job's image under its boundary rule; the job's
 * scales, path and out are ignored) are written to g[r*g_pitch + c] as int64.  The
 * recursions start from zero at the window's lower-left edges and run on the window
 * extended to the right by a triangle of zeros, which step (4) needs.  Float inputs are
 * taken on the 2^-24 grid (multiplied by 2^24).  Multiply by 2^n for the sqrt2 weights of
 * the two diagonal steps.  Values wrap modulo 2^64 if they exceed int64 (exact wherever
 * the true value fits).  Workspace: 8*hq*tp bytes, tp = wq+hq-1 rounded up to a
 * multiple of 4. */
bsf_status bsf_preintegrate(bsf_ctx* ctx, const bsf_job* job, int x0, int y0, int wq, int hq,
                            int64_t* g, ptrdiff_t g_pitch, void* stream);

/* Synchronise `stream`, return (and clear) the sticky device error of the context:
 * BSF_OK, BSF_ERR_SCALE_RANGE, BSF_ERR_UNSUPPORTED or BSF_ERR_RANGE (the first in this
 * order that occurred). */
bsf_status bsf_get_device_error(bsf_ctx* ctx, void* stream);

/* Scale field of elliptical windows (the step before the filter; the paper controls each
 * window through the box spline's covariance, Section 4, and leaves this map open).
 * For every pixel, ellipses[3*(y*ellipse_pitch + x) + {0,1,2}] = (s_major, s_minor, phi):
 * the standard deviations of the window along its two axes, in pixels, and the angle of
 * the first axis from the first lattice axis (x, columns) toward the second (y, rows), in
 * radians.  scales[4*(y*scale_pitch + x) + k] receives a_(k+1): the scales whose order-n
 * box spline has the covariance (n/12) sum_k a_k^2 r_k r_k^T closest in the Frobenius norm
 * to R(phi) diag(s_major^2, s_minor^2) R(phi)^T, with every a_k >= 0.5 (the filter's
 * smallest scale) and the least sum a_k^4 among equally close ones; an isotropic window
 * of deviation sigma gets a_k = sigma sqrt(6/n) (Theorem 4.3's scales).  Elongated windows
 * between the lattice directions are not reachable exactly and get the closest
 * covariance.  The output is the filter's scale format (bsf_job.scales).  Both buffers
 * are device memory owned by the caller; pitches count pixels; scales must be 16-byte
 * aligned.  Non-finite or non-positive deviations give NaN scales and the sticky
 * BSF_ERR_SCALE_RANGE flag.  Asynchronous on `stream`. */
bsf_status bsf_scales_from_ellipses(bsf_ctx* ctx, const float* ellipses, ptrdiff_t ellipse_pitch, int width,
                                    int height, int order, float* scales, ptrdiff_t scale_pitch, void* stream);

/* One-dimensional scale-adaptive filter (Section 3) on a batch of signals.  Sample m of
 * signal b gets the projection of the signal's continuous model onto the B-spline of degree
 * order-1 and scale a = scales[b*scale_pitch + m] centred at m (Section 3, the projections
 * s[m]; eq. definition for the scaled B-spline):
 *     s[m] = sum_k c_ext[k] (beta^model * beta_a^(order-1))(m - k),
 * where the model f(x) = sum_k c[k] beta^model(x - k) has degree model = -1 (impulses at the
 * samples, the model of the two-dimensional filter), 0 or 1 (for these the interpolation
 * filter is the unit impulse, so c = the samples), or 2 or 3 (c = the extended samples filtered
 * by the inverse of b^model[k] = beta^model(k), so that the model interpolates them: the
 * two-sided exponential rho z^|k| of the inverse, truncated where its tail falls below 2^-60),
 * and each signal is extended by its end values (clamp) or zeros.  Computed by Proposition
 * 3.1: order running sums (eq. RS, unit scale), then per sample the finite-difference mask
 * Delta_a^order (eq. FD) applied to the running sums interpolated with the B-spline of degree
 * model + order, on restart windows of 256 outputs.  BSF_PATH_F64: the running sums, the interpolation and the mask carry a
 * compensation term, so the float64 result matches the exact projection to a few ulps of its
 * largest terms.  BSF_PATH_F32_TILED: the running sums are compensated, the interpolation and
 * the mask plain float64, the result float32; its error is below 1e-5 of the output's
 * magnitude (tested at orders 1-3, all models, scales 0.5 to the largest window). */
typedef struct {
    int length, count;              /* samples per signal, number of signals (>= 1)       */
    bsf_dtype in_dtype;             /* u8, f32 or f64                                      */
    const void* in;                 /* [count][in_pitch] samples                           */
    ptrdiff_t in_pitch;             /* >= length, in elements                              */
    const float* scales;            /* [count][scale_pitch] scales a                        */
    ptrdiff_t scale_pitch;          /* >= length                                           */
    int order;                      /* number of running sums, 1..3 (B-spline degree + 1)  */
    int model;                      /* degree of the signal model: -1, 0, 1, 2 or 3        */
    bsf_path path;                  /* F64: float64 output; F32_TILED: float32 output       */
    bsf_border border;
    float a_max;                    /* upper bound on every scale (sizes the on-chip windows;
                                       0 = the largest bsf_filter1d_max_scale allows)      */
    void* out;                      /* [count][out_pitch] float64 (F64) / float32 (F32)    */
    ptrdiff_t out_pitch;            /* >= length                                           */
} bsf_job1d;

/* out[b][m] = s[m] of signal b for every sample.  All pointers are device memory owned by
 * the caller; asynchronous on `stream`; no workspace.  Scales must lie in [0.5, a_max]:
 * others (NaN included) give NaN outputs and the sticky BSF_ERR_SCALE_RANGE flag
 * (bsf_get_device_error).  BSF_ERR_UNSUPPORTED, synchronously, if a_max exceeds
 * bsf_filter1d_max_scale. */
bsf_status bsf_filter1d(bsf_ctx* ctx, const bsf_job1d* job, void* stream);

/* The largest a_max bsf_filter1d accepts for this order and model, on either path (the
 * restart window of 256 + about order * a_max samples, at (2 + model + order) * 16 bytes per
 * sample, must fit the on-chip memory of one workgroup).  Host only. */
bsf_status bsf_filter1d_max_scale(bsf_ctx* ctx, int order, int model, float* a_max);

/* Two-direction (rect) space-variant filter: Section 4, eq. def with directional order N = 2
 * (angles 0 and pi/2), whose box spline is the tensor product of a segment of length a1 along x
 * (columns) and one of length a2 along y (rows); rect is the one at (1, 1).  Order n is its
 * n-fold self-convolution beta_a1^(n-1)(x1) beta_a2^(n-1)(x2).  Every pixel m gets the
 * projection of the image's continuous model onto it at m's own scales (Section 6):
 *     out[m] = sum_k c_ext[k] K_a1(m1 - k1) K_a2(m2 - k2),   K_a = beta^model * beta_a^(order-1),
 * with the model f(x) = sum_k c[k] (beta^model x beta^model)(x - k) of degree model = -1
 * (impulses at the samples, the model of Section 7), 0 or 1 (c = the samples), or 2 or 3
 * (c = the extended samples filtered by the inverse of b^model x b^model, so that the model
 * interpolates them; the inverse is truncated where its tail falls below 2^-60), and the
 * image extended by clamp or zero.  Computed by the two steps of Section 6 with b = (1, 1):
 * order running sums along rows and columns (eq. RS_filter; the summed-area table for
 * order 1), then per pixel the (order+1)^2 finite-difference taps of eq. mask interpolated
 * with the tensor B-spline of degree model + order, on restart windows per tile.  Running
 * sums and mask carry a compensation term on both paths, which differ only in the output
 * (BSF_PATH_F64: float64; BSF_PATH_F32_TILED: float32).  scales is [height][scale_pitch][2]
 * float32 (a1, a2), 8-byte aligned; scales outside [0.5, a_max] (NaN included) give NaN and the
 * sticky BSF_ERR_SCALE_RANGE flag.  a_max (0 = the largest bsf_filter_rect_max_scale allows)
 * sizes the windows; beyond that limit the call returns BSF_ERR_UNSUPPORTED.  Models 2 and 3
 * use a work area of about 16 bytes per pixel of the image plus its halos (context
 * workspace).  Asynchronous on `stream`. */
typedef struct {
    int width, height;              /* >= 1                                                */
    bsf_dtype in_dtype;             /* u8, f32 or f64                                       */
    const void* in;                 /* [height][in_pitch] samples                           */
    ptrdiff_t in_pitch;             /* >= width                                             */
    const float* scales;            /* [height][scale_pitch][2] = (a1, a2) per pixel        */
    ptrdiff_t scale_pitch;          /* >= width, in pixels                                  */
    int order;                      /* n in {1, 2, 3}                                       */
    int model;                      /* degree of the image model: -1, 0, 1, 2 or 3          */
    bsf_path path;
    bsf_border border;
    float a_max;                    /* bound on every scale (0 = the largest allowed)       */
    void* out;                      /* [height][out_pitch] float64 (F64) / float32 (F32)   */
    ptrdiff_t out_pitch;            /* >= width                                             */
} bsf_job_rect;

bsf_status bsf_filter_rect(bsf_ctx* ctx, const bsf_job_rect* job, void* stream);

/* The largest a_max bsf_filter_rect accepts for this order and model (the restart window of
 * an 8x8 tile, 16 bytes per element, must fit one workgroup's LDS).  Host only. */
bsf_status bsf_filter_rect_max_scale(bsf_ctx* ctx, int order, int model, float* a_max);

/* Evaluation counters of the float64 path (Section 7 mesh, eq. final_eqn), kept per
 * context since its creation or the last reset.  A tile whose samples need a single
 * digit evaluates each tap's interpolant with the terms of total degree above 2 (order
 * 2) or 3 (order 3) in plain float64 and the rest compensated (in waves whose pixels all
 * have a1 a2 a3 a4 >= 625, resp. 410), and carries a rigorous bound on the plain
 * terms' rounding error; a pixel whose bound exceeds 2^-44 of its value is evaluated
 * again, compensated throughout.  Synchronises `stream` and writes the host array
 * out[2]: out[0] = pixels evaluated split, out[1] = pixels among them evaluated again.
 * reset != 0 clears both afterwards.  Order 1 is always compensated and not counted. */
bsf_status bsf_get_counters(bsf_ctx* ctx, void* stream, unsigned long long* out, int reset);

/* Test aid for the on-chip pre-integrator (stage 1 of Section 7, eq. RS): run only the
 * stage-1 part of the tile kernel for output tile `tile` (row-major tile index, 16x16
 * tiles) of `job` and write the box part of its restart window, int64 row-major
 * [hq][wq], to the device buffer `window` (capacity `cap` elements).  `geom` is a device
 * int[8]: the caller sets geom[4] = 1 to anchor every running sum at the tile centre
 * (what bsf_filter does) or 0 for the recursions' zero start at the window's lower-left
 * edges; the call writes geom[0..3] = x0, y0, wq, hq of the window and geom[5] = 1 if a
 * value left the int64 range and geom[6] = the power of two sh the samples were scaled by
 * (the window holds the digit-free running sums of f_ext * 2^sh).  For the float32-output
 * path the window holds float64 running sums of f_ext, as bit patterns, and geom[5..6]
 * are 0.  Asynchronous on `stream`. */
bsf_status bsf_debug_tile_window(bsf_ctx* ctx, const bsf_job* job, int tile, int64_t* window,
                                 long long cap, int* geom, void* stream);

const char* bsf_status_string(bsf_status s);

/* Detail text of the last failure on this context ("" if none). */
const char* bsf_last_error(const bsf_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* BSF_H */
