/*
 * bfgp -- Gauss-polynomial (GP) bilateral filter on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libbfgp.so.  Method: K. N. Chaudhury, "Fast and Accurate Bilateral
 * Filtering using Gauss-Polynomial Decomposition", arXiv 1505.00077.
 *
 * General conventions (every entry point):
 *  - Images are single-channel float32, row-major, H rows by W columns, with a
 *    row pitch given in ELEMENTS (pitch >= W).  Input and output share the pitch.
 *  - All image, workspace and gradient pointers are DEVICE pointers owned by the
 *    caller.  The library allocates no device memory in any entry point.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Every compute entry point only enqueues work on `stream` and returns; it
 *    never synchronises, except bf_gp_status which is documented as blocking.
 *  - Return value: BF_OK (0) or a negative bf_status.  Argument checks run on the
 *    host before any HIP call, so a rejected call enqueues nothing.  The text of
 *    the last failure on the calling thread is returned by bf_last_error().
 *  - Entry points are thread-safe as long as concurrent calls do not share a
 *    workspace.  Calls that share a workspace must be ordered on one stream.
 */
#ifndef BFGP_H
#define BFGP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define BF_OK 0
#define BF_EINVAL (-1)       /* a pointer, size or parameter is invalid            */
#define BF_ENOMEM (-2)       /* the workspace passed is smaller than required      */
#define BF_ERANGE (-3)       /* intensities too far from the centre for FP32
                                channels (reported by bf_gp_status)                */
#define BF_EHIP (-4)         /* a HIP runtime call failed                          */
#define BF_EUNSUPPORTED (-5) /* valid but not supported (e.g. FIR radius too large) */

/* ---- flags ---------------------------------------------------------------- */
/* Spatial filter used for the Gaussian filterings of eq. (8) (bits 0-1). */
#define BF_SPATIAL_AUTO 0u   /* FIR while ceil(3 sigma_s) is at most the crossover
                                radius, IIR above.  FIR and IIR are different
                                filters (truncated sampled Gaussian against
                                Deriche's untruncated kernel; they differ by
                                about 0.1 on 8-bit data), so AUTO's result, not
                                only its speed, depends on the crossover in
                                force: the process-wide radius (default 9) or
                                the size-dependent table a tuner installs
                                (bf_gp_set_fir_crossover_table)            */
#define BF_SPATIAL_FIR 1u    /* sampled Gaussian over |d| <= ceil(3 sigma_s), the
                                window of eq. (1)                                 */
#define BF_SPATIAL_IIR 2u    /* Deriche's 4th-order recursive Gaussian (causal +
                                anticausal, zero initial state), as in the
                                paper's experiments                                */
#define BF_SPATIAL_BOX 3u    /* box: uniform weights over the window of eq. (1),
                                |dy|, |dx| <= ceil(3 sigma_s), by running sums
                                (O(1) per pixel for any radius; Section 3, the
                                remark after eq. (11)).  Forward only; AUTO
                                never picks it                                     */
#define BF_SPATIAL_MASK 3u
/* Centre t_c of the intensity range (bits 2-3); Section 2, eq. (6). */
#define BF_CENTER_MEAN 0u     /* the mean, as in Algorithm 1 (default)           */
#define BF_CENTER_MIDRANGE 4u /* (min + max) / 2                                  */
#define BF_CENTER_NONE 8u     /* t_c = 0                                          */
#define BF_CENTER_MASK 12u

#define BF_MAX_DEGREE 64      /* largest N accepted                               */
#define BF_FIR_MAX_RADIUS 24  /* largest FIR radius ceil(3 sigma_s) (sigma_s <= 8) */

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int bf_version(void);

/* Message for the last non-zero status returned on the calling thread
 * (never NULL; empty when there was none). */
const char *bf_last_error(void);

/* ---- GP forward ------------------------------------------------------------
 * Algorithm 1 (GPF) with the channels rescaled as u_n(x) = exp(-x^2/2) x^n /
 * sqrt(n!), x = (f - t_c)/sigma_r, n = 0..N+1 (the images of eq. (7) divided by
 * sqrt(n!)), the spatial filtering of eq. (8) on every channel, and the
 * recombination of eqs. (9)-(11) in double precision:
 *     out = t_c + sigma_r * M / D,  D = sum_{n<=N} u_n(tau) Ubar_n,
 *                                   M = sum_{n<=N} u_n(tau) sqrt(n+1) Ubar_{n+1}.
 * Neighbours outside the image contribute nothing (zero extension).
 *
 *  img, out     device, H x W with row pitch `pitch` (elements); may not alias.
 *  sigma_s      spatial standard deviation (> 0, finite).
 *  sigma_r      range standard deviation (> 0, finite).
 *  N            degree of the Gauss-polynomial, 0..BF_MAX_DEGREE.  Even N keeps
 *               every approximate weight positive; with odd N the denominator
 *               can vanish and the output is whatever the division gives.
 *  flags        BF_SPATIAL_* | BF_CENTER_*.  Width limits: FIR none (radius up
 *               to BF_FIR_MAX_RADIUS), IIR and BOX W <= 16384, IIR with saved
 *               terms W <= 8192 (else BF_EUNSUPPORTED).  IIR rows past 8192
 *               samples are filtered as segments of 8192 whose end states
 *               are handed on through the workspace (8 floats per row,
 *               segment and channel).  BOX: the window radius is ceil(3 sigma_s)
 *               (capped at max(H, W), which covers the whole image); its two
 *               passes keep running and prefix sums in double, and the
 *               workspace holds the column-filtered stack (4 (N + 2) H P bytes,
 *               P = W rounded up to a multiple of 256 (W <= 4096) or 1024).
 *  saved        NULL, or a device buffer of 16*H*W bytes that receives what
 *               bf_gp_backward needs (per pixel: M/D and its tau-derivative as
 *               float, the rescaled denominator as double), planar.  FIR or
 *               IIR mode (BOX returns BF_EUNSUPPORTED); the backward must use
 *               the same mode.
 *  ws, ws_bytes device workspace of at least bf_gp_workspace_bytes(...) bytes.
 * Intensities whose |x| is so large that the channels leave the FP32 range make
 * the output NaN and set BF_ERANGE in the workspace status (bf_gp_status). */
size_t bf_gp_workspace_bytes(int H, int W, int N, double sigma_s, unsigned flags);

int bf_gp_forward(const float *img, float *out, int H, int W, int pitch,
                  double sigma_s, double sigma_r, int N, unsigned flags,
                  void *saved, void *ws, size_t ws_bytes, void *stream);

/* ---- GP forward without allocation --------------------------------------------
 * For callers that cannot allocate device memory at call time (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation and kernels as bf_gp_forward, with the workspace taken from
 * a static device array of BF_NOALLOC_SCRATCH_BYTES bytes inside the library
 * instead of a caller buffer.  Every GPU the library runs this on holds its own
 * copy of that array until the process ends.  The call allocates nothing (no
 * hipMalloc, no library routine that allocates); the caller still provides
 * img, out and, when wanted, saved.  Arguments as for bf_gp_forward.
 *  - Returns BF_ENOMEM when bf_gp_workspace_bytes(H, W, N, sigma_s, flags)
 *    exceeds BF_NOALLOC_SCRATCH_BYTES (at N 20: the FIR mode at any image
 *    size, the IIR mode up to about 1.2 MP).
 *  - Calls on one GPU share its array: calls that overlap on one GPU (on
 *    streams with no ordering between them) race and give undefined results.
 *    Calls ordered on one stream are safe; each rewrites every word it reads.
 *  - The device status word (BF_ERANGE) lives in that array and is not
 *    readable: out-of-range intensities show as NaN outputs. */
#define BF_NOALLOC_SCRATCH_BYTES (128u << 20)
int bf_gp_forward_noalloc(const float *img, float *out, int H, int W, int pitch,
                          double sigma_s, double sigma_r, int N, unsigned flags,
                          void *saved, void *stream);

/* ---- joint (cross) GP forward ------------------------------------------------
 * The variant the Conclusion names as a direct extension: the range kernel is
 * evaluated on a guide image g and the weighted average is taken of a data
 * image f,
 *     out(i) = sum_j k(j) g_r(g(i-j) - g(i)) f(i-j) / sum_j k(j) g_r(g(i-j) - g(i)),
 * approximated as in Algorithm 1 with the guide in every range term: with
 * x = (g - t_c)/sigma_r (t_c the guide's centre) and the channels u_n(x) and
 * u_n(x) f, n = 0..N, each filtered spatially,
 *     out = sum_n u_n(tau) Kbar[u_n f] / sum_n u_n(tau) Kbar[u_n],  tau = x(i).
 * With g = f it equals bf_gp_forward.  2 (N + 1) channels.
 *  guide, data, out  device, H x W with one row pitch `pitch`; out may alias
 *                    neither input.
 *  flags             BF_SPATIAL_AUTO or BF_SPATIAL_IIR (the recursive Gaussian,
 *                    as in the paper's experiments; BF_SPATIAL_FIR and
 *                    BF_SPATIAL_BOX return BF_EUNSUPPORTED), | BF_CENTER_*.
 *                    W up to 8192.
 *  ws, ws_bytes      device workspace of bf_gp_joint_workspace_bytes(...) bytes
 *                    (0 for unsupported arguments).
 * A guide too far from its centre for the FP32 channels makes the output NaN
 * and sets BF_ERANGE in the workspace status, as bf_gp_forward does. */
size_t bf_gp_joint_workspace_bytes(int H, int W, int N, double sigma_s, unsigned flags);

int bf_gp_joint_forward(const float *guide, const float *data, float *out, int H, int W, int pitch,
                        double sigma_s, double sigma_r, int N, unsigned flags,
                        void *ws, size_t ws_bytes, void *stream);

/* ---- volumes and video ------------------------------------------------------
 * The extension to higher-dimensional signals that the introduction and the
 * Conclusion name: Algorithm 1 on a T x H x W volume (frames t, rows y,
 * columns x), with eq. (8) the separable spatial filter over all three axes,
 * scale sigma_s along y and x and sigma_t along t (time in a video; equal to
 * sigma_s for an isotropic volume), zero extension, the centre taken over the
 * whole volume.  Recursive spatial mode (BF_SPATIAL_AUTO or BF_SPATIAL_IIR;
 * BF_SPATIAL_FIR and BF_SPATIAL_BOX return BF_EUNSUPPORTED): a time pass on
 * the volume seen as T rows of H W samples, a column pass in every frame, and
 * the row pass with the FP64 recombination.  With T = 1 the result is bf_gp_forward's (IIR).
 *  vol, out     device, contiguous T x H x W float (frame after frame, rows of
 *               W); may not alias.  W up to 8192, H W below 2^31.
 *  ws, ws_bytes device workspace of bf_gp_volume_workspace_bytes(...) bytes:
 *               two channel stacks of the volume (about 8 (N + 2) bytes per
 *               voxel) and the band carries.
 * Intensities too far from the centre make the output NaN and set BF_ERANGE
 * in the workspace status. */
size_t bf_gp_volume_workspace_bytes(int T, int H, int W, int N, double sigma_s, double sigma_t, unsigned flags);

int bf_gp_volume_forward(const float *vol, float *out, int T, int H, int W, double sigma_s, double sigma_t,
                         double sigma_r, int N, unsigned flags, void *ws, size_t ws_bytes, void *stream);

/* Blocking: waits for `stream`, then stores the status of the last forward or
 * backward that used `ws` in *status (BF_OK or BF_ERANGE). */
int bf_gp_status(const void *ws, void *stream, int *status);

/* Degree rule (the paper fixes N = 20 and leaves the choice of N open; this
 * rule is the library's own).  For centred intensities with |x| <= xmax
 * (x = (f - t_c)/sigma_r), the Gauss-polynomial weight of eqs. (4)-(5) differs
 * from the exact range weight by at most P(Poisson(xmax^2) > N) for every
 * pair of intensities once N >= xmax^2 - 1 (pairs of one sign: e^-y (e^y -
 * T_N(y)), y = t tau <= xmax^2, is that tail; opposite signs: the alternating
 * remainder times e^-|y| is a Poisson probability the tail dominates there).
 * Returns the smallest even N >= xmax^2 - 1 with tail <= eps (even N keeps
 * every weight positive), BF_EINVAL for xmax < 0 or eps outside (0, 1), and
 * BF_ERANGE when no N up to BF_MAX_DEGREE suffices.  Host only.  The bound is
 * on each weight; the output error also scales with the intensity spread and
 * the spatial kernel's mass. */
int bf_gp_degree_for(double xmax, double eps);

/* The spatial mode BF_SPATIAL_AUTO resolves to for this sigma_s (FIR or IIR)
 * under the process-wide crossover radius. */
unsigned bf_gp_resolve_spatial(double sigma_s, unsigned flags);
/* The same for an H x W image: the size-dependent crossover table, when set,
 * takes precedence (bf_gp_forward, the workspace size and the batched plan
 * resolve AUTO this way). */
unsigned bf_gp_resolve_spatial_for(int H, int W, double sigma_s, unsigned flags);

/* Sets the AUTO crossover: FIR is used while ceil(3 sigma_s) <= radius.
 * radius in 0..BF_FIR_MAX_RADIUS (0 = always IIR).  Process-wide. */
int bf_gp_set_fir_crossover(int radius);
int bf_gp_get_fir_crossover(void);

/* Size-dependent AUTO crossover, as a tuner measures it on a device: an image
 * of H * W pixels takes radius[k] of the first k with H * W <= max_pixels[k];
 * larger images take the process-wide radius.  max_pixels strictly increasing
 * and positive, radius in 0..BF_FIR_MAX_RADIUS, count in 0..8 (0 clears the
 * table).  Host arrays, copied.  Process-wide.  Returns BF_EINVAL on bad
 * input, leaving the table unchanged. */
int bf_gp_set_fir_crossover_table(const long long *max_pixels, const int *radius, int count);
/* Copies up to `max` entries of the table; returns the number of entries. */
int bf_gp_get_fir_crossover_table(long long *max_pixels, int *radius, int max);

/* Launch-shape overrides of the IIR mode, process-wide, for tuning (0 restores
 * the automatic choice):
 *   band_rows   0, 32 or 64: rows per band of the column passes (automatic:
 *               64 where the image gives at least 1024 column waves of 64
 *               rows, else 32; 32 for batched plans, the joint filter and
 *               the volume filter, which runs 32 whatever the override);
 *   col_groups  0..8: channel groups of the column passes;
 *   row_groups  0..8: channel groups of the row pass (capped by the row width
 *               and by the channel count).
 * They change how the passes split the work, hence the rounding of the
 * result (never its mathematics), and the workspace size of the IIR mode:
 * size the workspace after setting them.  The batched plan reads them when it
 * is built.  The IIR backward takes col_groups and row_groups (capped at 4)
 * as its channel groups.  Returns BF_EINVAL for values outside the ranges. */
int bf_gp_set_iir_tuning(int band_rows, int col_groups, int row_groups);
/* The IIR launch shape an H x W image of degree N gets under the current
 * settings: shape[0] band rows, [1] column channel groups, [2] samples per row
 * thread, [3] row threads per channel group, [4] row channel groups.
 * W up to 16384; past 8192 the row pass runs ceil(W / 8192) segments of 512
 * threads x 16 samples per row. */
int bf_gp_iir_shape(int H, int W, int N, int *shape /* 5 ints, host */);

/* ---- GP backward -------------------------------------------------------------
 * Adjoint of bf_gp_forward for a scalar loss L with upstream gradient
 * grad_out = dL/dout.  Derived by the chain rule through eqs. (7)-(11) and the
 * mean that Algorithm 1 takes as the centre.  The spatial filter is symmetric with
 * zero extension, so its adjoint is itself: the adjoint channels are filtered
 * by the forward's own kernel.  FIR mode: the radius ceil(3 sigma_s) is held
 * fixed when differentiating in sigma_s.  IIR mode: the recursion is
 * differentiated exactly in log sigma_s (a tangent recursion beside each
 * section); the workspace then holds two transposed channel stacks
 * (2 * (N+2) * W * ceil64(H) floats) and the band carries.
 *  saved              the buffer filled by bf_gp_forward with the same
 *                     image, parameters and spatial mode.
 *  grad_img           NULL or device H x W (pitch) float: dL/dimg.
 *  grad_log_sigma_s   NULL or device double: dL/d(log sigma_s) (overwritten).
 *  grad_log_sigma_r   NULL or device double: dL/d(log sigma_r) (overwritten).
 * Supported for the FIR and IIR modes (AUTO resolves as in bf_gp_forward;
 * BF_SPATIAL_BOX returns BF_EUNSUPPORTED and a workspace size of 0) with
 * centre mean or none; the midrange centre returns BF_EUNSUPPORTED. */
size_t bf_gp_backward_workspace_bytes(int H, int W, int N, double sigma_s, unsigned flags);

int bf_gp_backward(const float *img, const float *grad_out, const void *saved,
                   int H, int W, int pitch, double sigma_s, double sigma_r, int N,
                   unsigned flags, float *grad_img, double *grad_log_sigma_s,
                   double *grad_log_sigma_r, void *ws, size_t ws_bytes, void *stream);

/* ---- stacked batch: forward with saved terms and backward --------------------
 * B images of one size H x W filtered with one (sigma_s, sigma_r, N) and one
 * spatial mode (a training batch): Algorithm 1 per image, its backward as
 * bf_gp_backward, every stage one launch over all B images.  Image b is at
 * img + b * img_stride (elements); out, grad_out and grad_img use the same
 * stride and pitch; saved holds B blocks of 16 H W bytes (image b's block at
 * saved + b * 16 H W).  Every image's outputs and gradients equal those of a
 * single bf_gp_forward / bf_gp_backward call on it bit for bit.
 *  img_stride   >= H * pitch; the image, output and gradient batches must not
 *               overlap (BF_EINVAL).
 *  ws           device workspace of at least the *_stacked_workspace_bytes.
 *  grad_log_sigma_s, grad_log_sigma_r
 *               device arrays of B doubles (nullable): the scalar gradients of
 *               each image, as bf_gp_backward gives them (sum them for a
 *               shared parameter).
 * FIR and IIR modes (BOX returns BF_EUNSUPPORTED); the same width limits and
 * error behaviour as the single-image calls. */
size_t bf_gp_forward_stacked_workspace_bytes(int B, int H, int W, int N, double sigma_s, unsigned flags);
int bf_gp_forward_stacked(const float *img, float *out, int B, int H, int W, int pitch, size_t img_stride,
                          double sigma_s, double sigma_r, int N, unsigned flags, void *saved,
                          void *ws, size_t ws_bytes, void *stream);
size_t bf_gp_backward_stacked_workspace_bytes(int B, int H, int W, int N, double sigma_s, unsigned flags);
int bf_gp_backward_stacked(const float *img, const float *grad_out, const void *saved, int B, int H, int W,
                           int pitch, size_t img_stride, double sigma_s, double sigma_r, int N,
                           unsigned flags, float *grad_img, double *grad_log_sigma_s,
                           double *grad_log_sigma_r, void *ws, size_t ws_bytes, void *stream);

/* ---- batched GP forward ---------------------------------------------------
 * Many images of uneven size, each with its own sigma_s and sigma_r (Algorithm 1
 * applied per image), filtered by one short sequence of grouped launches: one
 * launch per stage (statistics, FIR tiles, column-band states, carry
 * resolution, column pass, row pass), each covering every image of the batch,
 * so no workgroup ever waits on another.  Plans are host objects;
 * bf_gp_plan_upload copies the plan's descriptors into the workspace (once,
 * outside any graph capture, synchronising `stream`); bf_gp_forward_batched
 * then only launches kernels and may be captured into a hipGraph and replayed.
 * Each image gets the spatial mode a single bf_gp_forward call would give it
 * (the AUTO crossover table is read when the plan is built).  The batch fills
 * the device by itself, so its IIR images are not split into channel groups:
 * each image's output is bit-identical to a single call made under
 * bf_gp_set_iir_tuning(0, 1, 1) (with other tuning overrides, under the same
 * overrides), and differs from a default single call only in rounding.
 * Images are limited to 8192 columns (the IIR limit).  FIR, IIR or AUTO:
 * BF_SPATIAL_BOX returns BF_EUNSUPPORTED. */
typedef struct bf_gp_item {
    const float *img; /* device, H x W, row pitch `pitch` elements */
    float *out;       /* device, same shape and pitch */
    int H, W, pitch;
    float sigma_s, sigma_r;
    int N;
} bf_gp_item;

int bf_gp_plan_batched(const bf_gp_item *items, int count, unsigned flags, void **plan_out);
size_t bf_gp_plan_workspace_bytes(const void *plan);
int bf_gp_plan_upload(void *plan, void *ws, size_t ws_bytes, void *stream);
int bf_gp_forward_batched(void *plan, void *ws, size_t ws_bytes, void *stream);
void bf_gp_plan_free(void *plan);

/* ---- direct filter ---------------------------------------------------------
 * Eq. (1) evaluated directly: O((2W+1)^2) range-kernel evaluations per pixel,
 * spatial Gaussian of eq. (2) over the square window |dy|,|dx| <= window,
 * in-image neighbours only.  window < 0 selects ceil(3 sigma_s).  Used as the
 * O(sigma_s^2) comparator.  window <= 64. */
int bf_direct_forward(const float *img, float *out, int H, int W, int pitch,
                      double sigma_s, double sigma_r, int window, void *stream);

/* ---- stage timing ----------------------------------------------------------
 * Profiling aid.  While enabled, every entry point records a pair of HIP events
 * on its stream around each kernel it launches.  bf_profile_enable(1) (re)starts
 * the record, bf_profile_enable(0) stops recording.  bf_profile_collect waits for
 * the recorded events and fills, for up to `max` distinct kernel names, the
 * number of launches, the summed duration in milliseconds and the grid size
 * (in threads) of the last launch; it returns the number of names filled (or a
 * negative status).  Name strings are static. */
int bf_profile_enable(int on);
int bf_profile_collect(int max, const char **names, int *counts, double *total_ms, long long *threads);

#ifdef __cplusplus
}
#endif

#endif /* BFGP_H */
