/*
 * rgbid.h - C ABI of the MI355X (gfx950) dense RGB-D alignment library.
 *
 * The library estimates the rigid motion between two RGB-D frames by dense
 * frame-to-keyframe alignment in inverse-depth parametrisation and fuses
 * inverse-depth maps into a keyframe, following Gutierrez-Gomez & Guerrero,
 * "RGBiD-SLAM for Accurate Real-time Localisation and 3D Mapping":
 *   - problem statement and frames A (reference) / B (current): sec. 6.1;
 *   - coarse-to-fine Gauss-Newton / IRLS with the photometric and
 *     inverse-depth residuals and the pose update: sec. 6.2;
 *   - robust location / scale / degrees of freedom on a systematic sample:
 *     sec. 6.3;
 *   - inverse geometric warping: sec. 5.3;
 *   - keyframe fusion with the covisibility test: sec. 7.2 and sec. 6.4.
 *
 * Conventions (all calls)
 *   Images are row-major; element (u, v) is at index v * pitch + u, with u the
 *   column and v the row, pixel centres at integer coordinates.  Intensity is
 *   in grey levels (finite values, below 65504 with FP16 storage); inverse
 *   depth W = 1/Z in 1/m, and W <= 0 or non-finite marks a hole.  Device pointers are HIP device memory on the context's
 *   device (a torch tensor's data_ptr() is fine).
 *   A pose is T = (R, t), R row-major, the pose of B in A: X_A = R X_B + t
 *   (the paper's T_A^B).  Twists are xi = (v, theta), translation first.
 *
 * Errors
 *   Every call returns an rgbid_status; nothing throws or aborts across the
 *   ABI.  rgbid_last_error() returns a text description of the last failure
 *   on that context.  Calls on one context are not thread-safe; use one
 *   context per host thread (each with its own stream).
 *
 * Synchrony
 *   Calls enqueue work on the context's stream.  Calls that return host
 *   results (poses, statistics, counts) synchronise that stream before
 *   returning; calls that only produce device data do not.
 */
#ifndef RGBID_H
#define RGBID_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RGBID_OK = 0,
    RGBID_E_ARG = -1,         /* invalid argument (NULL, range, mismatched parameters) */
    RGBID_E_SHAPE = -2,       /* image sizes / formats of the operands do not match */
    RGBID_E_DEVICE = -3,      /* a HIP runtime call failed */
    RGBID_E_NOMEM = -4,       /* device or pinned-host allocation failed */
    RGBID_E_DEGENERATE = -5   /* normal equations not positive definite, or fewer
                                 than 6 valid residuals: the pose keeps its last value */
} rgbid_status;

/* Level-0 pinhole camera of undistorted images (sec. 4.1 without the
   distortion term).  Level l uses f/2^l and (c + 0.5)/2^l - 0.5. */
typedef struct {
    int width, height;
    double fx, fy, cx, cy;
} rgbid_camera;

/* T_A^B: X_A = R X_B + t, R row-major. */
typedef struct {
    double R[9];
    double t[3];
} rgbid_pose;

/* Storage format of pyramid images: FP32, or FP16 (per-pixel arithmetic is
   FP32 either way). */
typedef enum { RGBID_F32 = 0, RGBID_F16 = 1 } rgbid_format;

/* Robust weight: Student-t with estimated degrees of freedom (sec. 6.3), or
   Huber with threshold huber_k on the normalised residual. */
typedef enum { RGBID_W_STUDENT_T = 0, RGBID_W_HUBER = 1 } rgbid_weight;

/* FULLRES: every iteration warps B at full resolution and downsamples the
   warped images to the current level (sec. 6.2).  PER_LEVEL: warps the
   level-l images of B directly (a cheaper variant). */
typedef enum { RGBID_WARP_FULLRES = 0, RGBID_WARP_PER_LEVEL = 1 } rgbid_warp_mode;

typedef struct {
    int levels;              /* pyramid levels used, 1..8 (<= the pyramids' levels) */
    int iters[8];            /* Gauss-Newton iterations at each level (index = level) */
    int weight;              /* rgbid_weight */
    double huber_k;          /* Huber threshold, default 1.345 */
    int estimate_nu;         /* Student-t: estimate nu by bisection on [2, 10] (default 1) */
    int sample_max;          /* N, maximum size of the systematic sample (default 19200,
                                at most 24576) */
    int scale_iters;         /* fixed-point iterations for location and scale (default 20) */
    int warp;                /* rgbid_warp_mode */
    double stop_eps_t;       /* early stop of a level when |v| < eps_t and |theta| < eps_r; */
    double stop_eps_r;       /*   both 0 = fixed schedule (default) */
    int scale_warm;          /* 1 (default): the location / scale fixed point of every
                                iteration after the first at a level starts from the
                                previous iteration's mu, sigma, and the step that moves
                                both by at most 2^-16 sigma is its last (at most
                                scale_iters steps); 0: every iteration starts from mu = 0,
                                sigma^2 = mean r^2 and takes scale_iters steps (sec. 6.3) */
} rgbid_align_params;

/* Statistics of the last linearisation of an alignment.  H is the upper
   triangle of the 6x6 normal matrix, row-major (H00 H01 .. H05 H11 .. H55);
   g = sum w J^T r, so that the step is xi = -H^-1 g.  H is the inverse of the
   pose covariance (sec. 6.2). */
typedef struct {
    double H[21], g[6];
    double mu_I, sigma_I, nu_I, mu_W, sigma_W, nu_W;
    double cost;                   /* sum of w r^2 over both channels */
    long long n_valid_I, n_valid_W;
    int iters_done[8];
    int status;                    /* rgbid_status of this pair */
} rgbid_align_stats;

typedef struct rgbid_ctx rgbid_ctx;
typedef struct rgbid_pyr rgbid_pyr;
typedef struct rgbid_kf rgbid_kf;

/* Fills p with the defaults: 4 levels, 10 iterations per level, Huber
   k = 1.345, nu estimated (Student-t only), N = 19200, 20 scale iterations,
   FULLRES warp, fixed schedule. */
void rgbid_default_params(rgbid_align_params* p);

/* ------------------------------------------------------------ lifecycle */

/* Creates a context on HIP device `device`, enqueuing on `hip_stream` (a
   hipStream_t; NULL = the legacy default stream).  The context owns its
   scratch memory.  *ctx is NULL on failure.  A batch is split into up to 4
   launch chains that run on streams of their own, forked from and joined back
   into `hip_stream`; the environment variable RGBID_CHAINS (1-8), read here,
   sets another number. */
rgbid_status rgbid_create(rgbid_ctx** ctx, int device, void* hip_stream);

/* Releases the context and its scratch memory (synchronises its stream).
   Pyramids and keyframes must be freed separately.  NULL is ignored. */
void rgbid_destroy(rgbid_ctx* ctx);

/* Text of the last error on this context ("" if none).  Owned by the context. */
const char* rgbid_last_error(const rgbid_ctx* ctx);

/* ------------------------------------------------------------ pyramid */

/* Builds a `levels`-level image pyramid (sec. 6.2: images are downsampled at
   every level) from caller-owned FP32 device images I_dev, W_dev of size
   cam->width x cam->height with row pitch `pitch_elems` (elements, >= width).
   Level l+1 is the 2x2 mean of level l (size floor(w/2) x floor(h/2)); the
   inverse depth mean skips holes and is a hole when all four are holes.
   Images are stored in `storage` format (FP16 rounds to nearest even).
   The input is copied (not aliased) and may be released when the call
   returns; the call does not synchronise.  *out is library-owned; free it
   with rgbid_pyramid_free.  Errors: E_ARG (NULL, levels outside 1..8, a
   level smaller than 1x1, 2^22 = 4194304 pixels or more), E_NOMEM,
   E_DEVICE. */
rgbid_status rgbid_pyramid(rgbid_ctx* ctx, const rgbid_camera* cam, int levels,
                           rgbid_format storage, const float* I_dev, const float* W_dev,
                           size_t pitch_elems, rgbid_pyr** out);

/* Rebuilds an existing pyramid in place from new images of the same size
   (no allocation).  Same arguments and errors as rgbid_pyramid. */
rgbid_status rgbid_pyramid_update(rgbid_ctx* ctx, rgbid_pyr* pyr, const float* I_dev,
                                  const float* W_dev, size_t pitch_elems);

/* Rebuilds n existing pyramids in place in one batched launch per level.
   I_dev[i], W_dev[i], pitch_elems[i] describe frame i as in rgbid_pyramid and
   must match pyrs[i]'s size.  All pyramids share one storage format.  Does
   not synchronise.  Errors: E_ARG, E_SHAPE, E_NOMEM, E_DEVICE. */
rgbid_status rgbid_pyramid_update_batch(rgbid_ctx* ctx, int n, rgbid_pyr* const* pyrs,
                                        const float* const* I_dev, const float* const* W_dev,
                                        const size_t* pitch_elems);

/* Copies level `level` of a pyramid into caller-owned FP32 device buffers of
   size w_l x h_l (dense rows), converting from the storage format.  Holes
   read as 0.  Does not synchronise.  Errors: E_ARG. */
rgbid_status rgbid_pyramid_read(rgbid_ctx* ctx, const rgbid_pyr* pyr, int level,
                                float* I_out_dev, float* W_out_dev);

/* Level size of a pyramid (host-side, no device work). */
rgbid_status rgbid_pyramid_level_size(const rgbid_pyr* pyr, int level, int* w, int* h);

void rgbid_pyramid_free(rgbid_pyr* pyr);

/* ------------------------------------------------------------ alignment */

/* Estimates T_A^B between reference A and current frame B (sec. 6.2):
   coarse-to-fine from level params->levels-1 to 0, params->iters[l]
   iterations at level l; each iteration warps B towards A at the current
   estimate (sec. 5.3), forms the photometric and inverse-depth residuals
   with their Jacobians, estimates location / scale (and nu) on the systematic
   sample (sec. 6.3), reduces the weighted 6x6 normal equations, solves them
   by Cholesky in FP64 on the device and applies T <- exp(xi)^-1 T.
   `init` NULL = identity (sec. 6.2).  Writes the pose to *out and, if
   stats != NULL, the statistics of the last linearisation.  Synchronises.
   A degenerate system stops the iteration and returns E_DEGENERATE with the
   last good pose in *out.  Errors: E_ARG, E_SHAPE (A and B differ in size,
   format or levels), E_NOMEM, E_DEVICE. */
rgbid_status rgbid_align(rgbid_ctx* ctx, const rgbid_pyr* A, const rgbid_pyr* B,
                         const rgbid_pose* init, const rgbid_align_params* params,
                         rgbid_pose* out, rgbid_align_stats* stats);

/* rgbid_align for callers that cannot allocate memory: code under HIP graph
   capture of the surrounding work, tight serving loops, harnesses that
   forbid hipMalloc.  Same arguments, results and errors as rgbid_align for
   one pair with the library's default launch shapes (the ones rgbid_align
   uses for a pair shape it has not tuned), and the same poses bit for bit
   in that case.  It calls no device or host allocation routine and no graph:
   every device buffer (pair descriptor, state, chunk tables, partial sums,
   sample residuals, stored warped level images) lies in one static device
   array of 8 MiB per device, which the library reaches through the address
   rgbid_create looks up for its device and holds until the process ends;
   tables are written by a set-up kernel from its arguments, and the results
   are read back into the call's own stack memory.  A pair whose buffers
   need more than 8 MiB is refused with E_ARG (a 1280x960 pair needs under
   3 MiB with FULLRES, its largest stored warped level being 640x480).
   Every call on a device shares that device's array and leaves its contents
   behind: calls that overlap on one device (two host threads, or two
   contexts on different streams) race and must be serialised by the caller.
   Synchronises the context's stream. */
rgbid_status rgbid_align_noalloc(rgbid_ctx* ctx, const rgbid_pyr* A, const rgbid_pyr* B,
                                 const rgbid_pose* init, const rgbid_align_params* params,
                                 rgbid_pose* out, rgbid_align_stats* stats);

/* Aligns n independent pairs (A[i], B[i]) of possibly different sizes in one
   schedule: every iteration of every level is a fixed sequence of launches
   that covers all pairs, replayed from a cached HIP graph when the batch
   shape repeats.  All pyramids must share one storage format and have at
   least params->levels levels.  init: n poses or NULL (identity); out: n
   poses; stats: n entries or NULL.  Per-pair failure is reported in
   stats[i].status (the call itself returns OK unless an argument or the
   device failed).  Synchronises. */
rgbid_status rgbid_align_batch(rgbid_ctx* ctx, int n, const rgbid_pyr* const* A,
                               const rgbid_pyr* const* B, const rgbid_pose* init,
                               const rgbid_align_params* params, rgbid_pose* out,
                               rgbid_align_stats* stats);

/* Asynchronous form of rgbid_align_batch for callers that keep results on
   the device (serving loops, pipelines that enqueue the next batch while
   this one runs): the same computation, but the n poses and (if stats_dev
   != NULL) the n statistics are written to caller-owned device memory in
   the layouts above, and the call returns as soon as the work is enqueued
   on the context's stream.  init is host memory (n poses or NULL), read
   before the call returns.  Pyramids and output buffers must stay alive
   until the stream reaches this work.  Errors (argument checks only):
   E_ARG, E_SHAPE, E_NOMEM, E_DEVICE. */
rgbid_status rgbid_align_batch_async(rgbid_ctx* ctx, int n, const rgbid_pyr* const* A,
                                     const rgbid_pyr* const* B, const rgbid_pose* init,
                                     const rgbid_align_params* params, rgbid_pose* out_dev,
                                     rgbid_align_stats* stats_dev);

/* One linearisation without an update: the normal equations of the pair at
   pyramid level `level` and pose T, with the same sampling and weights as an
   alignment iteration (diagnostic; also the Hessian for a covariance).
   Synchronises.  Errors as rgbid_align; E_DEGENERATE is not raised (the
   counts in *out tell). */
rgbid_status rgbid_normal_equations(rgbid_ctx* ctx, const rgbid_pyr* A, const rgbid_pyr* B,
                                    int level, const rgbid_pose* T,
                                    const rgbid_align_params* params,
                                    rgbid_align_stats* out);

/* ------------------------------------------------------------ autotuner */

/* Times, for every level of `params`, candidate launch shapes of the pixel
   kernels on this batch -- warp fused into the reduction or stored, 2 / 4 / 8
   waves per workgroup, 1 / 2 / 4 / 8 / 16 tiles of 64 pixels per wave, and
   XCD-aware chunk order on or off; then, for the best of those, 1 / 2 / 4 /
   8 / 16 passes per wave of the warp kernel -- over `reps` replayed
   iterations (normal equations only, the poses stay at the identity), and
   keeps the fastest for later calls with a batch of the same shape (pair
   sizes in order, levels, warp mode, storage) on this context.  Every
   candidate is timed twice; the four fastest four more times, and the lowest
   median wins.  best_ms (params->levels entries or NULL) receives the best
   time per iteration.  Synchronises. */
rgbid_status rgbid_autotune(rgbid_ctx* ctx, int n, const rgbid_pyr* const* A,
                            const rgbid_pyr* const* B, const rgbid_align_params* params, int reps,
                            double* best_ms);

/* Writes / reads the context's tuned launch shapes as text (one
   "key fused waves tiles_per_wave xcd_remap warp_passes" line per entry). */
rgbid_status rgbid_tune_save(const rgbid_ctx* ctx, const char* path);
rgbid_status rgbid_tune_load(rgbid_ctx* ctx, const char* path);

/* ------------------------------------------------------------ covariance */

/* Bilateral filter of the covariance iteration (the paper gives no
   parameters): window (2 radius + 1)^2 (radius <= 7), spatial weight
   exp(-d^2 / (2 sigma_s^2)), intensity range weight exp(-dI^2 / (2 sigma_I^2)),
   inverse-depth range weight exp(-(dW / (rel_W W(p)))^2 / 2); holes skipped.
   Defaults: 2, 1.5 px, 10 grey levels, 0.05. */
typedef struct {
    int radius;
    double sigma_s, sigma_I, rel_W;
} rgbid_bilateral;

/* Pose covariance of sec. 6.2: one extra linearisation at level 0 and pose T
   (the final estimate) without an update, with {I_A, W_A} bilateral-filtered
   before the pyramid and gradients are formed; Sigma (6 x 6, row-major) =
   H_filt^-1, inverted by FP64 Cholesky.  bf NULL = defaults; stats (NULL ok)
   receives the filtered linearisation.  Synchronises.  Errors: E_ARG,
   E_SHAPE, E_DEGENERATE (H_filt not positive definite). */
rgbid_status rgbid_covariance(rgbid_ctx* ctx, const rgbid_pyr* A, const rgbid_pyr* B,
                              const rgbid_pose* T, const rgbid_align_params* params,
                              const rgbid_bilateral* bf, double Sigma[36],
                              rgbid_align_stats* stats);

/* ------------------------------------------------------------ covisibility */

/* Dense covisibility ratio of sec. 6.4 at pyramid `level`: the pixels of A
   with a valid inverse depth (S_H) are transferred into B with T (the pose of
   B in A); a pixel is visible (S_V) when it lands in the image with four valid
   W_B taps and |W_B(p_B) - w_B| < tol (tol = 3 sigma_W), w_B the transferred
   inverse depth.  The same is done from B to A with T^-1, and
   *ratio = min(|S_V|/|S_H| over both directions).  counts (4 entries or NULL)
   receives |S_H(A)|, |S_V(A->B)|, |S_H(B)|, |S_V(B->A)|.  Synchronises.
   Errors: E_ARG, E_SHAPE. */
rgbid_status rgbid_covisibility(rgbid_ctx* ctx, const rgbid_pyr* A, const rgbid_pyr* B, int level,
                                const rgbid_pose* T, double tol, double* ratio, long long* counts);

/* ------------------------------------------------------------ keyframe fusion */

/* Creates a keyframe from a caller-owned FP32 inverse-depth map (copied) with
   weight C = 1 everywhere (sec. 7.2).  Does not synchronise. */
rgbid_status rgbid_keyframe_init(rgbid_ctx* ctx, const rgbid_camera* cam, const float* W_dev,
                                 size_t pitch_elems, rgbid_kf** out);

/* Fuses frame k's FP32 inverse-depth map into the keyframe (sec. 7.2): every
   keyframe pixel with valid W_kf is transferred into frame k with T_kf_k
   (the pose of frame k in the keyframe: X_kf = R X_k + t), W_k is sampled
   bilinearly (four valid taps), and if |W_k(p_w) - 1/Y_z| < tol (the
   covisibility test of sec. 6.4, tol = 3 sigma_W) the warped inverse depth W*
   is merged: W_kf <- (W_kf C_kf + C_k W*)/(C_kf + C_k), C_kf <- C_kf + C_k,
   with C_k the inverse-variance weight of the warp.  Keyframe holes stay
   holes.  If n_fused != NULL the number of fused pixels is written there
   (synchronises); otherwise the call does not synchronise.  Errors: E_ARG. */
rgbid_status rgbid_fuse(rgbid_ctx* ctx, rgbid_kf* kf, const float* Wk_dev, size_t pitch_elems,
                        const rgbid_pose* T_kf_k, double tol, long long* n_fused);

/* Fuses n frames (1 <= n <= 256) into the keyframe in order, as n calls of
   rgbid_fuse would (the same per-pixel arithmetic, so the same result bit for
   bit), in one launch: each keyframe pixel is read and written once instead
   of n times.  Wk_dev[i] is frame i's caller-owned FP32 inverse-depth map
   (device, all with row pitch `pitch_elems`), T_kf_k[i] its pose in the
   keyframe.  If n_fused != NULL (n entries) it receives the number of
   pixels fused by each frame (synchronises); otherwise the call does not
   synchronise.  Errors: E_ARG. */
rgbid_status rgbid_fuse_batch(rgbid_ctx* ctx, rgbid_kf* kf, int n, const float* const* Wk_dev,
                              size_t pitch_elems, const rgbid_pose* T_kf_k, double tol,
                              long long* n_fused);

/* Re-initialises an existing keyframe from a new FP32 inverse-depth map of
   the same size, with C = 1 (no allocation, does not synchronise). */
rgbid_status rgbid_keyframe_reset(rgbid_ctx* ctx, rgbid_kf* kf, const float* W_dev,
                                  size_t pitch_elems);

/* Copies the keyframe's W and C maps into caller-owned FP32 device buffers
   (dense rows).  Either pointer may be NULL.  Does not synchronise. */
rgbid_status rgbid_keyframe_read(rgbid_ctx* ctx, const rgbid_kf* kf, float* W_out_dev,
                                 float* C_out_dev);

void rgbid_keyframe_free(rgbid_kf* kf);

/* ------------------------------------------------------------ sensor input path */

/* A camera with Brown distortion (sec. 4.1, eq. proj_dist): k = (k1, k2, k3,
   k4, k5), radial k1, k2, k5 and tangential k3, k4; cam is the pinhole part. */
typedef struct {
    rgbid_camera cam;
    double k[5];
} rgbid_lens;

/* Calibration of an RGB-D sensor (sec. 4.1, 4.2).  Raw depth Z_m (m) is
   corrected as W_d(p) = beta1 / Z_m(p - p0) + beta0 (p0 = (p0x, p0y),
   (4, 4) for the sensor of the paper), then, if spatial != 0,
   W_u(p) = D1(p) W_d(p) + D0(p) with D_i(p) = q_i0 + q_i1 r^2 + q_i2 r^4 +
   q_i3 r^6 + q_i4 m_x + q_i5 m_y + q_i6 m_x m_y + q_i7 m_x^2 m_y +
   q_i8 m_x m_y^2, m = K_depth^-1 p (all nine listed terms are used).  T_dc is
   the pose of the colour camera in the depth camera (T_D^C). */
typedef struct {
    rgbid_lens color, depth;
    double beta0, beta1;
    int p0x, p0y;
    int spatial;
    double q0[9], q1[9];
    rgbid_pose T_dc;
} rgbid_sensor;

/* Undistortion by inverse warping (sec. 5.1): dst(p) = src(K h(K^-1 p)),
   bilinear, on the lens's own grid (dst dense, width x height, caller-owned
   device memory).  is_depth: src is an inverse-depth map, a sample needs
   four valid taps and holes are 0.  Unmapped pixels are 0.  Does not
   synchronise.  Errors: E_ARG. */
rgbid_status rgbid_undistort(rgbid_ctx* ctx, const rgbid_lens* lens, const float* src,
                             size_t pitch_elems, int is_depth, float* dst);

/* Forward registration (sec. 5.2) of the undistorted inverse-depth map W_A
   of camera A into camera B with T = T_A^B (X_A = R X_B + t): first the
   translation alone, each pixel's footprint square (side 1/(1 - W t_z),
   centred on the translated position) written to the intermediate frame
   with an atomic maximum of the inverse depth (pixels whose centres lie in
   the half-open square); then the rotation as an inverse warp with nearest
   neighbour, W_B(p) = W_Bt(p_t) (R K_B^-1 p)_z.  WB: dense B-sized
   caller-owned device buffer, holes 0.  Does not synchronise.  Errors:
   E_ARG, E_NOMEM. */
rgbid_status rgbid_register(rgbid_ctx* ctx, const rgbid_camera* camA, const float* WA,
                            size_t pitch_elems, const rgbid_camera* camB, const rgbid_pose* T,
                            float* WB);

/* Input path of one RGB-D frame: depth correction of Z_raw on the depth
   grid, undistortion through the depth lens, registration into the colour
   camera with T_dc, and undistortion of the colour image I_raw (grey
   levels, colour grid).  I_out, W_out: dense colour-sized caller-owned
   device buffers, ready for rgbid_pyramid.  The corrected and undistorted
   depth maps are formed inside the registration kernel and never stored.
   Does not synchronise.  Errors: E_ARG, E_NOMEM. */
rgbid_status rgbid_preprocess(rgbid_ctx* ctx, const rgbid_sensor* sensor, const float* I_raw,
                              size_t pitch_I, const float* Z_raw, size_t pitch_Z, float* I_out,
                              float* W_out);

/* ------------------------------------------------------------ tracking front-end */

/* Frame-to-reference tracking of an RGB-D sequence with keyframe fusion
   (sec. 7.1, sec. 7.2).  Every frame k is aligned to the current reference
   frame from the constant-velocity guess T_rf^{k-1} T_{k-2}^{k-1}; the
   odometry constraint T_{k-1}^k and, if requested, its covariance (pose
   covariance of sec. 6.2 propagated as in the appendix on covariance
   composition) are formed; the dense covisibility ratio (sec. 6.4, at
   pyramid level covis_level, tol = tol_sigmas * sigma_W of that alignment)
   against the keyframe decides whether frame k starts a new keyframe
   (ratio < kf_threshold) or is fused into it; after a keyframe switch the
   frames recorded with the previous keyframe (at most `buffer`, most recent
   first) are fused into the new one, one per incoming frame; the ratio
   against the reference frame decides whether frame k becomes the next
   reference frame (ratio < rf_threshold).  Covariances are over the left
   perturbation (dt, dtheta): t -> t + dt, R -> exp(dtheta) R. */
typedef struct {
    rgbid_align_params align;  /* alignment of each frame to the reference */
    double rf_threshold;       /* reference-frame switch (default 0.8; above kf_threshold) */
    double kf_threshold;       /* keyframe switch (default 0.7) */
    int covis_level;           /* pyramid level of the covisibility ratios (default 2) */
    double tol_sigmas;         /* occlusion tolerance in sigma_W (default 3) */
    int buffer;                /* pre-keyframe frame buffer, 0..64 (default 8) */
    int covariance;            /* 1: pose and odometry covariances (default 1) */
} rgbid_tracker_params;

typedef struct {
    long long frame;           /* k, counted from 0 */
    rgbid_pose T_w_k;          /* pose of frame k in frame 0 */
    rgbid_pose T_rf_k;         /* pose of frame k in its reference frame */
    rgbid_pose T_prev_k;       /* odometry constraint: pose of frame k in frame k-1 */
    double Sigma_rf_k[36];     /* covariance of T_rf_k, row-major (0 if not requested) */
    double Sigma_odo[36];      /* covariance of T_prev_k (0 if not requested) */
    double covis_rf, covis_kf; /* covisibility ratios with the reference frame and keyframe */
    int rf_switched;           /* frame k is the reference frame of frame k+1 */
    int kf_switched;           /* frame k started a new keyframe */
    int cov_status;            /* rgbid_status of the covariance iteration */
    long long n_fused;         /* keyframe pixels fused from frame k */
    long long n_fused_buffer;  /* keyframe pixels fused from a buffered frame */
    rgbid_align_stats stats;   /* alignment of frame k (zeros for frame 0) */
} rgbid_track_result;

typedef struct rgbid_tracker rgbid_tracker;

/* Fills p with the defaults listed above (align = rgbid_default_params). */
void rgbid_tracker_default_params(rgbid_tracker_params* p);

/* Creates a tracker for frames of camera `cam`, with pyramids of `levels`
   levels in `storage` format (levels >= align.levels, > covis_level).  The
   tracker owns its pyramids (three), the keyframe and `2 buffer + 1` FP32
   inverse-depth maps.  Errors: E_ARG, E_NOMEM. */
rgbid_status rgbid_tracker_create(rgbid_ctx* ctx, const rgbid_camera* cam, int levels,
                                  rgbid_format storage, const rgbid_tracker_params* params,
                                  rgbid_tracker** out);

/* Tracks the next frame (caller-owned FP32 device images, copied): frame 0
   initialises the reference frame and the keyframe.  A degenerate alignment
   keeps the guess and is reported in out->stats.status; a degenerate
   covariance iteration sets cov_status and zero covariances.  Synchronises.
   Errors: E_ARG, E_DEVICE. */
rgbid_status rgbid_track(rgbid_ctx* ctx, rgbid_tracker* trk, const float* I_dev,
                         const float* W_dev, size_t pitch_elems, rgbid_track_result* out);

/* The tracker's active keyframe (owned by the tracker; read it with
   rgbid_keyframe_read). */
const rgbid_kf* rgbid_tracker_keyframe(const rgbid_tracker* trk);

/* Releases the tracker (synchronises the device).  NULL is ignored. */
void rgbid_tracker_free(rgbid_tracker* trk);

/* ------------------------------------------------------------ pose maps */

/* Decoupled exponential and logarithm of sec. 3: exp(xi) = (Rot(theta), v) for
   xi = (v, theta); log(T) = (t, log R) with |theta| < pi.  Host only. */
void rgbid_pose_exp(const double xi[6], rgbid_pose* T);
void rgbid_pose_log(const rgbid_pose* T, double xi[6]);

/* ------------------------------------------------------------ learned warm start */

/* A convolutional network that predicts the initial twist of an alignment
   from the 80 x 60 pyramid level of both frames (an addition to the method:
   the paper starts from the identity or a constant-velocity guess, sec. 6.2,
   sec. 7.1).  Gauss-Newton always runs after it.  Input per pair: 4 x 60 x 80
   FP32 (I_A/255, W_A/2, I_B/255, W_B/2, holes as 0).  Layers: 4 x [3x3
   convolution, stride 2, zero padding 1, bias, ReLU] with channels 4 -> 32 ->
   64 -> 128 -> 128, global average pool, fully connected 128 -> 6.  The output
   o is normalised: xi0 = o * (0.15, 0.15, 0.15, 0.1745, 0.1745, 0.1745) (m, rad).
   Parameters (rgbid_warmstart_param_count() floats, FP32 master copy) are laid
   out w1 b1 w2 b2 w3 b3 w4 b4 wfc bfc, conv weights as Co x Ci x 3 x 3, FC as
   6 x 128.  Weights are used in bfloat16 (nearest even), biases, activations,
   gradients and AdamW state in FP32. */
typedef struct rgbid_net rgbid_net;

size_t rgbid_warmstart_param_count(void);

/* Creates a network from host FP32 parameters (copied) with zeroed AdamW
   state.  Does not synchronise.  Errors: E_ARG, E_NOMEM, E_DEVICE. */
rgbid_status rgbid_warmstart_create(rgbid_ctx* ctx, const float* params_host, rgbid_net** out);
void rgbid_warmstart_free(rgbid_net* net);

/* Copies the FP32 master parameters to host memory (synchronises). */
rgbid_status rgbid_warmstart_get_params(rgbid_ctx* ctx, const rgbid_net* net, float* params_host);

/* Builds the n x 4 x 60 x 80 input in caller-owned device memory x_dev from
   the level of each pair's pyramids whose size is 80 x 60.  Does not
   synchronise.  Errors: E_ARG, E_SHAPE (no 80 x 60 level). */
rgbid_status rgbid_warmstart_input(rgbid_ctx* ctx, int n, const rgbid_pyr* const* A,
                                   const rgbid_pyr* const* B, float* x_dev);

/* Forward pass on n inputs; writes the predicted twists xi0 (n x 6, metres and
   radians) to host memory (synchronises). */
rgbid_status rgbid_warmstart_forward(rgbid_ctx* ctx, rgbid_net* net, int n, const float* x_dev,
                                     double* xi_out);

/* The same forward pass on the matrix cores, reading the input from the
   80 x 60 level of each pair's pyramids: the convolutions are implicit GEMMs
   of the bf16 weights and the FP32 activations carried as three exact bf16
   limbs (v_mfma_f32_32x32x16_bf16, FP32 accumulation), so the result is that
   of rgbid_warmstart_forward up to the order of FP32 additions.  Writes xi0
   (n x 6, metres and radians) to host memory (synchronises).  Errors: E_ARG,
   E_SHAPE (no 80 x 60 level, mixed formats), E_NOMEM, E_DEVICE. */
rgbid_status rgbid_warmstart_forward_pyr(rgbid_ctx* ctx, rgbid_net* net, int n,
                                         const rgbid_pyr* const* A, const rgbid_pyr* const* B,
                                         double* xi_out);

/* Matrix-core forward + exponential: initial poses for rgbid_align_batch.
   x_scratch_dev is not used (kept for callers of the FP32 input path). */
rgbid_status rgbid_warmstart_predict(rgbid_ctx* ctx, rgbid_net* net, int n,
                                     const rgbid_pyr* const* A, const rgbid_pyr* const* B,
                                     float* x_scratch_dev, rgbid_pose* init_out);

/* The warm-started batch alignment without a host round trip: the matrix-core
   forward of rgbid_warmstart_forward_pyr, the initial poses T0 = (exp(theta),
   v) formed on the device from its output, then rgbid_align_batch from T0.
   Same outputs and errors as rgbid_align_batch; the poses equal those of
   rgbid_warmstart_predict followed by rgbid_align_batch up to the last bits
   of the initial poses (device versus host FP64 sin / cos).  Synchronises. */
rgbid_status rgbid_align_batch_warm(rgbid_ctx* ctx, rgbid_net* net, int n,
                                    const rgbid_pyr* const* A, const rgbid_pyr* const* B,
                                    const rgbid_align_params* params, rgbid_pose* out,
                                    rgbid_align_stats* stats);

/* Loss (mean over the batch of the squared normalised twist error) and its
   gradient w.r.t. every parameter for labels xi (n x 6, host), without an
   update.  grad_host: rgbid_warmstart_param_count() floats or NULL.
   Synchronises. */
rgbid_status rgbid_warmstart_gradient(rgbid_ctx* ctx, rgbid_net* net, int n, const float* x_dev,
                                      const double* xi, double* loss, float* grad_host);

/* One AdamW training step (beta 0.9 / 0.999, eps 1e-8, decoupled weight decay
   wd on the weights only) on a batch; writes the batch loss before the update
   if loss != NULL (synchronises only then). */
rgbid_status rgbid_warmstart_train_step(rgbid_ctx* ctx, rgbid_net* net, int n, const float* x_dev,
                                        const double* xi, double lr, double wd, double* loss);

/* ------------------------------------------------------------ diagnostics */

/* Kernel families of one iteration, in launch order. */
typedef enum {
    RGBID_K_WARP = 0,     /* warp (+ downsample) and sample residuals */
    RGBID_K_SCALE = 1,    /* location / scale / nu */
    RGBID_K_REDUCE = 2,   /* residuals, Jacobians, weights, normal-equation partials */
    RGBID_K_SOLVE = 3     /* FP64 sum, Cholesky, pose update */
} rgbid_kernel;

/* Turns per-kernel timing on (1) or off (0).  While on, the alignment
   driver launches directly (not from a cached graph), records HIP events
   between the kernel launches of every iteration on the context's stream, and
   accumulates, per level and kernel family, the elapsed time and the number of
   launches when each call completes.  Turning it on clears the accumulators. */
rgbid_status rgbid_set_profiling(rgbid_ctx* ctx, int on);

/* Reads the accumulators: ms_total[l * 4 + k] and launches[l * 4 + k] for
   level l < 8 and kernel family k (rgbid_kernel); arrays of 32 entries. */
rgbid_status rgbid_kernel_times(const rgbid_ctx* ctx, double* ms_total, long long* launches);

#ifdef __cplusplus
}
#endif

#endif /* RGBID_H */
