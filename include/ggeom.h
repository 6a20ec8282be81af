/*
 * ggeom.h -- C ABI of the MI355X geometry stage of "Geometry-guided Online 3D
 * Video Synthesis with Multi-View Temporal Consistency" (arXiv 2505.18932):
 * forward splatting of K RGB-D views into a target camera, fusion of their
 * depths into a truncated signed distance field held as an H x W x D frustum
 * volume in the target's image space, carried across frames with a running
 * weight, and zero-crossing extraction of one depth per pixel; plus adjoints
 * and a batched path.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Cameras: world -> camera x_c = R x_w + t (R row-major), intrinsics
 *   K = [[fx, 0, cx], [0, fy, cy], [0, 0, 1]]; the projection of a world point
 *   p into camera k is (x_k, y_k, z_k) = K_k (R_k p + t_k) and its pixel
 *   coordinates are (x_k / z_k, y_k / z_k) (paper, Suppl. A.1).  Pixel (i, j)
 *   is column i, row j, with its centre at (i + 0.5, j + 0.5); it samples the
 *   area [i, i+1) x [j, j+1).  Depth is camera-frame z in metres; a depth
 *   sample is usable iff it is > 0 and finite (holes are 0).
 * Memory: every array pointer is a DEVICE pointer on the current HIP device,
 *   owned by the caller, unless marked [host].  Images are row-major, one view
 *   after the other (view-major).  Volumes are H x W x D with D innermost.
 * Streams: `stream` is a hipStream_t (NULL: the default stream).  All work is
 *   enqueued on it; a return value of GG_OK means "enqueued".  Kernel faults
 *   surface at the caller's next synchronisation.
 * Workspace: scratch comes from the caller's `ws` buffer of `ws_bytes` bytes
 *   (device memory, 256-byte aligned); gg_workspace_size() gives the size.
 *   These calls never allocate device memory.  Workspace contents need not be
 *   initialised and are clobbered.
 * Errors: 0 on success; a negative GG_ERR_* code otherwise, with a message
 *   readable through gg_last_error() (thread-local).  Invalid arguments are
 *   detected before anything is enqueued.  Nothing throws across the ABI.
 * Aliasing: outputs never alias inputs, except F / W, which may alias
 *   F_prev / W_prev (in-place temporal update), and depth_filtered, which
 *   may alias depth_filtered_prev.
 * Determinism: every output is bitwise reproducible run to run; integer
 *   outputs (winner indices, bins) and the volume F / W are bitwise equal to
 *   the plain FP32 definition (no contraction, correctly rounded divide and
 *   square root, floor for pixel indices, ties broken by the smaller index).
 */
#ifndef GGEOM_H
#define GGEOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GG_OK 0
#define GG_ERR_INVALID (-1)     /* an argument is out of range or NULL          */
#define GG_ERR_WORKSPACE (-2)   /* ws is NULL or ws_bytes too small             */
#define GG_ERR_HIP (-3)         /* a HIP runtime call or launch failed          */
#define GG_ERR_UNSUPPORTED (-4) /* valid but beyond the library's limits        */

#define GG_MAX_VIEWS 16     /* K per call                                    */
#define GG_MAX_BINS 4096    /* D per volume                                  */
#define GG_MAX_WINDOW 15    /* confidence window side                        */

/* Pinhole camera (Suppl. A.1 projection).  width/height in pixels. */
typedef struct gg_camera {
  float fx, fy, cx, cy;
  float R[9]; /* world -> camera rotation, row-major */
  float t[3]; /* world -> camera translation          */
  int32_t width, height;
} gg_camera;

/* Pixel-Gaussian splat (§3.1, Suppl. A.3).  Each input pixel is an isotropic
 * opaque Gaussian whose source-image footprint is one pixel. */
typedef struct gg_splat_params {
  float sigma_px; /* std of the Gaussian in source pixels (0.5: one-pixel footprint) */
  float band_rel; /* blend band: splats with z <= z_winner * (1 + band_rel), >= 0  */
  float z_min;    /* splats with target depth <= z_min are dropped, >= 0            */
  float r_max_px; /* cap on the coverage radius in target pixels, in (0, 64]        */
} gg_splat_params;

/* Frustum-volume TSDF (Suppl. A.1, A.2). */
typedef struct gg_tsdf_params {
  float z_near, z_far;   /* depth range; bins uniform in 1/z, z_0 = z_near, 0 < near < far */
  int32_t num_bins;      /* D, 2 .. GG_MAX_BINS                                          */
  float trunc;           /* truncation: metres, or bins if trunc_in_bins                 */
  int32_t trunc_in_bins; /* 1: tau_d = trunc * du * z_d^2 (local metric width of bins)   */
  float conf_tau;        /* tau of the window statistic nu (Suppl. A.1: 0.02 m)          */
  float conf_scale;      /* scale of the fusion weight (Suppl. A.1: 0.001)               */
  int32_t conf_window;   /* w, odd, 1 .. GG_MAX_WINDOW (Suppl. A.1: 7)                   */
  float decay;           /* beta of Suppl. A.2, weight carried per frame, in [0, 1]      */
  float weight_cap;      /* eta of Suppl. A.2, cap on the carried weight, >= 0           */
} gg_tsdf_params;

/* Colour-difference masks between consecutive frames (Eq. 1, §3.2). */
typedef struct gg_mask_params {
  float beta;     /* offset of the mask (Eq. 1: 0.6), in [0, 1]                       */
  float lambda_t; /* colour-change scale (Eq. 1: 0.7), > 0                            */
  int32_t factor; /* the mask is formed at 1/factor resolution (§3.2: 4), 1 .. 16     */
} gg_mask_params;

/* Launch shape of the volume kernels (tsdf_integrate and its variants,
 * tsdf_extract_depth, gg_fusion_stream_probe), passed with each call; NULL or
 * a zero field takes the default.  Results never depend on it (it exists for
 * the autotuner).
 *   pixels_per_block  whole target pixels per workgroup, 0..1024 (0: 512
 *                     threads' worth)
 *   pixels_per_row    neighbouring pixels interleaved in a wavefront row of
 *                     the fusion, 0..64 (the largest power of two <= it
 *                     dividing pixels_per_block is used; 0: 16)
 *   bins_per_thread   1, 2, 4 or 8 (0: 4 where it divides num_bins); used
 *                     where it divides num_bins and, for 8, where every
 *                     volume argument is 32-byte aligned, else the largest of
 *                     4, 2, 1 dividing num_bins.
 *   band_width        order in which the fusion visits its workgroup tiles:
 *                     vertical bands of about this many target pixels
 *                     across, each walked row by row from the top, so that
 *                     the view-table lines which neighbouring target rows
 *                     share are still cached when the next row needs them;
 *                     0..65536 (0: 256); a band as wide as the target is
 *                     plain row-major order, which is also taken where the
 *                     target width is not a multiple of pixels_per_block.
 * Invalid values: GG_ERR_INVALID. */
typedef struct gg_volume_tuning {
  int32_t pixels_per_block;
  int32_t pixels_per_row;
  int32_t bins_per_thread;
  int32_t band_width;
} gg_volume_tuning;

/* Operations for gg_workspace_size(). */
enum {
  GG_OP_SPLAT = 1,
  GG_OP_SPLAT_BACKWARD = 2,
  GG_OP_TSDF_INTEGRATE = 3,
  GG_OP_TSDF_INTEGRATE_BACKWARD = 4,
  GG_OP_DIFFERENCE_MASKS = 5, /* src_w x src_h frames, num_bins = the mask factor */
  GG_OP_SPLAT_EWA = 6
};

/* Bytes of workspace `op` needs for K source views of src_w x src_h pixels, a
 * tgt_w x tgt_h target and D bins (sp: splat parameters, [host], needed by the
 * splat ops, may be NULL otherwise).  Returns 0 on invalid arguments. */
size_t gg_workspace_size(int op, int32_t K, int32_t src_w, int32_t src_h, int32_t tgt_w,
                         int32_t tgt_h, int32_t num_bins, const gg_splat_params *sp);

/* ---------------------------------------------------------------------------
 * splat_views -- forward rendering of per-pixel Gaussians (§3.1; Suppl. A.3),
 * each view into its own target images, z-buffered.
 *
 * Source pixel q = (i, j) of view k with usable depth D is moved to the target
 * (x_T, y_T, z_T) = K_T (R_T p + t_T), p its world point; it is dropped unless
 * z_T > z_min.  Centre (x, y) = (x_T, y_T) / z_T, target std
 * sigma = sigma_px * (fx_T / fx_k) * (D / z_T), coverage radius^2
 * R2 = min(2 sigma^2, r_max^2).  Target pixel p is covered iff its centre lies
 * within R2 of (x, y).  The winner of p is the covering splat with the
 * smallest (z_T, q); its band is every covering splat with
 * z_T <= z_win * (1 + band_rel).  With G = exp(-d^2 / (2 sigma^2)) and
 * colour c = rgb / 255: out_rgb = sum G c / sum G over the band,
 * out_alpha = 1 - prod (1 - G) (accumulated opacity), out_depth = z_win,
 * win_idx = q_win = j * src_w + i.  Uncovered pixels: -1, 0, 0, 0.
 *
 * src [host] K cameras, all of one size src_w x src_h; K in 1..GG_MAX_VIEWS.
 * depth  float  K x src_h x src_w            rgb uint8 K x src_h x src_w x 3
 * tgt [host] target camera (tgt_w x tgt_h).  prm [host].
 * win_idx int32 K x tgt_h x tgt_w             out_depth float K x tgt_h x tgt_w
 * out_rgb float K x 3 x tgt_h x tgt_w (planar) out_alpha float K x tgt_h x tgt_w
 * out_tape float K x 3 x tgt_h x tgt_w or NULL: per pixel sum G, the sum of
 *   log(1 - G) over band members with G < 1, and the count of G == 1 (what
 *   splat_views_backward needs).
 * Colour and opacity are accumulated in 64-bit fixed point, so they are
 * independent of the order splats arrive in; the means and the opacity are
 * then formed in FP32 and equal the sequential FP32 results to a few 1e-7
 * relative.
 * ------------------------------------------------------------------------- */
int splat_views(const gg_camera *src, int32_t K, const float *depth, const uint8_t *rgb,
                const gg_camera *tgt, const gg_splat_params *prm, int32_t *win_idx,
                float *out_depth, float *out_rgb, float *out_alpha, float *out_tape, void *ws,
                size_t ws_bytes, void *stream);

/* splat_views plus one per-pixel scalar of the source views (the
 * difference masks of Eq. 1) carried to the target like a colour channel
 * (Suppl. A.2): out_mask = sum G m / sum G over the band of each target
 * pixel, 0 where no splat covers it, and out_mask_max its maximum over the
 * K views (the channel-wise maximum that weights the temporal carry of
 * tsdf_integrate).  mask float K x src_h x src_w; out_mask float
 * K x tgt_h x tgt_w or NULL; out_mask_max float tgt_h x tgt_w or NULL (at
 * least one of the two).  The other outputs are exactly those of
 * splat_views; the workspace is splat_views'.  The mask sums use the same
 * 64-bit fixed point as the colours. */
int splat_views_masked(const gg_camera *src, int32_t K, const float *depth, const uint8_t *rgb,
                       const gg_camera *tgt, const gg_splat_params *prm, const float *mask,
                       int32_t *win_idx, float *out_depth, float *out_rgb, float *out_alpha,
                       float *out_tape, float *out_mask, float *out_mask_max, void *ws,
                       size_t ws_bytes, void *stream);

/* Adjoint of splat_views with respect to source depth and colour, for the
 * loss L = <g_rgb, out_rgb> + <g_depth, out_depth> + <g_alpha, out_alpha>.
 * Coverage, band and winner are held fixed (piecewise differentiation).
 * Inputs as splat_views plus its outputs win_idx, out_depth, out_rgb and
 * out_tape (required here).  g_rgb / g_depth / g_alpha: same shapes as
 * out_rgb / out_depth / out_alpha (any may be NULL = zero).
 * g_depth_in float K x src_h x src_w, g_rgb_in float K x src_h x src_w x 3
 * (gradient with respect to c = rgb / 255): overwritten.  Gather formulation
 * (one thread per source pixel), so it needs no atomics; ws may be NULL. */
int splat_views_backward(const gg_camera *src, int32_t K, const float *depth,
                         const uint8_t *rgb, const gg_camera *tgt, const gg_splat_params *prm,
                         const int32_t *win_idx, const float *out_depth, const float *out_rgb,
                         const float *out_tape, const float *g_rgb, const float *g_depth,
                         const float *g_alpha, float *g_depth_in, float *g_rgb_in, void *ws,
                         size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * splat_views_ewa -- the per-pixel Gaussians of splat_views rendered as the
 * 3D Gaussian splatting rasteriser renders them (§3.1): projected with the
 * local affine (EWA) approximation of the perspective map and alpha-
 * composited front to back, each view into its own target images.
 *
 * Source pixel q of view k with usable depth D and target point (x_T, y_T,
 * z_T) (dropped unless z_T > z_min) is a Gaussian with mean (u, v) =
 * (x_T, y_T) / z_T and image covariance
 *   S = sig^2 [[1 + a^2, r a b], [r a b, r^2 (1 + b^2)]] + lowpass I,
 * a = (u - cx) / fx, b = (v - cy) / fy, r = fy / fx (target intrinsics),
 * sig = sigma_px (fx_T / fx_k) (D / z_T): the perspective Jacobian applied to
 * an isotropic 3D Gaussian of std sigma_px D / fx_k (one source pixel), plus
 * the rasteriser's screen-space low-pass (0.3 px^2 there).  At target pixel
 * centre p, d = p - (u, v): alpha = min(0.99, exp(-d^T S^-1 d / 2)); the term
 * is skipped when alpha < 1/255 or when |d_x| or |d_y| exceeds r_max_px (the
 * clip that bounds the footprint).  Per pixel the terms are taken in
 * ascending (z_T in FP32, q) order, colour += c alpha T, depth += z_T alpha
 * T, T *= (1 - alpha), stopping before the first term that would bring T
 * below 1e-4.  out_rgb = the colour sum (c = rgb / 255), out_alpha = 1 - T,
 * out_depth = depth sum / (1 - T) (0 where no term was taken).  band_rel is
 * not used.
 * Every step is FP32 in a fixed order with no contraction, including the
 * exponential (Cody-Waite reduction, degree-6 Taylor polynomial, within 3
 * ulp): the outputs are bitwise reproducible, independent of the launch.
 *
 * src, K, depth, rgb, tgt, prm: as splat_views.  lowpass >= 0 (px^2).
 * sort_limit: the longest per-tile key list sorted in LDS in one piece
 * (64..512; 0: 512); longer lists are sorted as runs of the largest power of
 * two not above it, merged in global memory.  Results do not depend on it.
 * out_rgb float K x 3 x tgt_h x tgt_w; out_alpha, out_depth float
 * K x tgt_h x tgt_w: overwritten.  ws: gg_workspace_size(GG_OP_SPLAT_EWA,
 * ...), 256-byte aligned; it holds the Gaussians' records and per-tile key
 * lists (about 16 K src_w src_h 16-byte words for r_max_px = 8).
 * ------------------------------------------------------------------------- */
int splat_views_ewa(const gg_camera *src, int32_t K, const float *depth, const uint8_t *rgb,
                    const gg_camera *tgt, const gg_splat_params *prm, float lowpass,
                    int32_t sort_limit, float *out_rgb, float *out_alpha, float *out_depth,
                    void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * tsdf_raymarch -- the volume-free form of the fusion (Suppl. A.1): per
 * target pixel, the fused signed distance is evaluated on the fly along the
 * ray and the first sign change is located by marching and bisection; the
 * previous output depth enters as one more input (Suppl. A.2).  No volume.
 *
 * Fused value at target depth z (the sampling, sign, occlusion and clamp of
 * tsdf_integrate, with tau(z) = trunc du z^2 if trunc_in_bins else trunc):
 *   S = sum_k omega_k min(s_k, tau), Wo = sum_k omega_k over kept samples,
 *   views in order; then, where depth_prev(p) > 0 and omega_tmp > 0, one more
 *   sample s = depth_prev(p) - z with weight omega_tmp (same rules);
 *   omega_tmp = min((decay * acc_prev(p)) * max(1 - M(p), 0), weight_cap).
 *   Wt = Wo (+ omega_tmp if kept); s(z) = S / Wt, unobserved where Wt = 0.
 * March from z = z_near while z <= z_far (at most 4 D + 16 samples), with
 *   step_min(z) = (du z) z (one inverse-depth bin): observed s > 0: z +=
 *   max(0.8 s, step_min); observed s <= 0 after an observed s > 0: surface
 *   bracketed; observed s <= 0 otherwise: z += step_min; unobserved: z +=
 *   0.8 tau(z).  Three bisections of the bracket [a, b] (a = mid where s(mid)
 *   is observed and > 0, else b = mid); depth = a + (b - a) * 0.5.
 *   No surface: depth 0, acc 0.  out_acc = omega_tmp + Wo at the depth (the
 *   accumulated weight of Suppl. A.2 for the next frame's acc_prev).
 * All FP32 in this order (no contraction): bitwise reproducible.
 *
 * src, K, depth, tgt, prm: as tsdf_integrate (num_bins sets du and the
 * sample cap).  depth_prev, acc_prev: float tgt_h x tgt_w, both or neither
 * (no temporal term).  temporal_mask: float tgt_h x tgt_w or NULL (M = 0);
 * needs depth_prev.  out_depth float tgt_h x tgt_w; out_acc float
 * tgt_h x tgt_w or NULL; out_steps int32 tgt_h x tgt_w or NULL (samples
 * before the bisection).  ws: gg_workspace_size(GG_OP_TSDF_INTEGRATE, ...).
 * ------------------------------------------------------------------------- */
int tsdf_raymarch(const gg_camera *src, int32_t K, const float *depth, const gg_camera *tgt,
                  const gg_tsdf_params *prm, const float *depth_prev, const float *acc_prev,
                  const float *temporal_mask, float *out_depth, float *out_acc,
                  int32_t *out_steps, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * network_inputs -- the input stack of the blending network (§3.3 and the
 * supplement's list of network inputs), (9K + 1) planes of tgt_h x tgt_w:
 *   [0, 3K) rgb (the splat's out_rgb), [3K, 4K) depth (its out_depth),
 *   [4K, 5K) alpha (its out_alpha), 5K the TSDF depth, then per view k
 *   5K+1+k  dot(input-view ray direction, TSDF normal),
 *   6K+1+k  dot(input-view ray direction, target ray direction),
 *   7K+1+k  |C_k - C_t| (camera centres), 8K+1+k dot of the optical axes.
 * Surface point X = C_t + D a, a = R_t^T K_t^-1 (px, py, 1) (FP64-formed,
 * rounded once; X = fma(D, a, C_t)).  Normal: the normalised cross product
 * of the horizontal and vertical differences of neighbouring surface points
 * (central where both neighbours have a depth > 0, else one-sided, else
 * none), oriented towards the target.  Input-view ray: (X - C_k) / |X - C_k|;
 * target ray: a / |a|.  Dot planes are 0 without a TSDF depth (or normal).
 * FP32, sums of three products left to right, no contraction: bitwise
 * reproducible.
 * src [host] K in 1..GG_MAX_VIEWS; tgt [host]; tsdf_depth float tgt_h x
 * tgt_w; rgb float K x 3 x tgt_h x tgt_w; depth, alpha float K x tgt_h x
 * tgt_w; out float (9K + 1) x tgt_h x tgt_w.
 * ------------------------------------------------------------------------- */
int network_inputs(const gg_camera *src, int32_t K, const gg_camera *tgt,
                   const float *tsdf_depth, const float *rgb, const float *depth,
                   const float *alpha, float *out, void *stream);

/* blend_views -- Eq. 4-5 for given weights: I_FG = sum_k I_k alpha_k w_k /
 * sum_k alpha_k w_k (0 where the sum is 0), I = (1 - w_BG) I_FG + w_BG I_BG;
 * the depths blend with the same weights (Eq. 6's blended depth).  Order:
 * aw = alpha_k w_k; num = fma(x_k, aw, num), den = den + aw, k in order;
 * I = fma(w_BG, I_BG, (1 - w_BG) I_FG).
 * rgb float K x 3 x height x width; depth, alpha, weights float
 * K x height x width; w_bg float height x width; rgb_bg float
 * 3 x height x width; out_rgb float 3 x height x width; out_depth float
 * height x width. */
int blend_views(int32_t K, int32_t width, int32_t height, const float *rgb, const float *depth,
                const float *alpha, const float *weights, const float *w_bg,
                const float *rgb_bg, float *out_rgb, float *out_depth, void *stream);

/* ---------------------------------------------------------------------------
 * difference_masks -- soft colour-difference masks between consecutive frames
 * of K views (Eq. 1, §3.2) and, optionally, the temporally filtered depth of
 * Eq. 2.
 *
 * Per view, at 1/factor resolution: each low-resolution pixel is the
 * factor x factor box of full-resolution pixels (clipped at the border,
 * n pixels); with S the box's integer sums of each u8 channel,
 *   dI = (|S_r - S_r'| + |S_g - S_g'| + |S_b - S_b'|) / (765 n)
 * (the channel mean of |I - I'|, colours u8 / 255), M = min(dI / lambda_t +
 * beta, 1); then the maximum over the 3 x 3 neighbourhood (clipped); then
 * bilinear upsampling at the full-resolution pixel centres,
 * x = (i + 0.5) / factor - 0.5 clamped to [0, W / factor rounded up - 1]
 * (likewise y), top = m00 + fx (m10 - m00), bottom likewise, mask = top +
 * fy (bottom - top).  Every step is FP32 in this order (no contraction).
 * Filter (Eq. 2), where depth is given: filtered = fma(M, D, (1 - M) * prev);
 * a hole in D gives 0; where prev is NULL (first frame) or a hole, D.
 *
 * rgb, rgb_prev  uint8 K x height x width x 3 (frames t and t - 1)
 * prm [host].  mask float K x height x width (output).
 * depth float K x height x width or NULL (no filtering); depth_filtered_prev
 * float K x height x width or NULL; depth_filtered float K x height x width
 * (required with depth; may alias depth_filtered_prev).
 * ws: gg_workspace_size(GG_OP_DIFFERENCE_MASKS, K, width, height, width, height,
 *   prm->factor, NULL).
 * ------------------------------------------------------------------------- */
int difference_masks(int32_t K, int32_t width, int32_t height, const uint8_t *rgb,
                     const uint8_t *rgb_prev, const gg_mask_params *prm, float *mask,
                     const float *depth, const float *depth_filtered_prev,
                     float *depth_filtered, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * tsdf_integrate -- fuse K depth maps into the target's frustum volume
 * (Suppl. A.1) with the temporal weight of Suppl. A.2 carried per voxel.
 *
 * Bins: un = 1/z_near, uf = 1/z_far, du = (un - uf)/(D - 1),
 *   z_d = 1 / (un - d du); tau_d = trunc * du * z_d^2 if trunc_in_bins else
 *   trunc.
 * Fusion weight per source pixel (Suppl. A.1): nu = sum over the w x w window
 *   (row-major) of min((D_q - D_n)^2, conf_tau^2); out-of-image neighbours are
 *   skipped, hole neighbours add conf_tau^2; omega = 1 if nu == 0 else
 *   min(conf_scale / sqrt(nu / w^2), 1); holes have omega = 0.
 * Voxel (x, y, d): for k = 0 .. K-1, project the point at depth z_d on the
 *   ray of pixel (x, y) into view k; skip unless z_k > 0; sample the pixel
 *   (floor(x_k / z_k), floor(y_k / z_k)) (skip if outside or a hole);
 *   s = D_k - z_k (positive in front of the surface); skip if s < -tau_d;
 *   S += omega * min(s, tau_d); Wo += omega.
 * Temporal: m = max(1 - mask, 0) (1 without a mask); with a previous volume,
 *   w_tmp = min(decay * W_prev * m, weight_cap), else 0;
 *   W = w_tmp + Wo; F = (w_tmp F_prev + S) / W, or 0 where W == 0.
 * Extraction (when out_depth is not NULL): as tsdf_extract_depth, fused.
 *
 * depth float K x src_h x src_w.  temporal_mask float tgt_h x tgt_w or NULL.
 * F_prev, W_prev float tgt_h x tgt_w x D or both NULL (no carry); they may
 * alias F, W.  F, W float tgt_h x tgt_w x D: overwritten.
 * out_depth float tgt_h x tgt_w, out_bin int32 tgt_h x tgt_w: both or neither.
 * tuning [host]: the launch shape, or NULL (gg_volume_tuning).
 * ------------------------------------------------------------------------- */
int tsdf_integrate(const gg_camera *src, int32_t K, const float *depth, const gg_camera *tgt,
                   const gg_tsdf_params *prm, const float *temporal_mask, const float *F_prev,
                   const float *W_prev, float *F, float *W, float *out_depth, int32_t *out_bin,
                   const gg_volume_tuning *tuning, void *ws, size_t ws_bytes, void *stream);

/* The fusion in two calls, for a caller that builds a frame's view table on
 * another stream ahead of the fusion (it depends on the depth maps only):
 * tsdf_view_table computes into ws what tsdf_integrate computes first -- per
 * source pixel the usable depth and the fusion weight of Eq. 3 (the
 * confidence of the supplement), and the bin depths; tsdf_integrate_tabled
 * then fuses from that ws exactly as tsdf_integrate does (bitwise the same
 * outputs).  Arguments as tsdf_integrate; both calls take the same src, K,
 * prm and ws (gg_workspace_size(GG_OP_TSDF_INTEGRATE, ...)); the caller
 * orders them (one stream, or an event) and keeps ws untouched between. */
int tsdf_view_table(const gg_camera *src, int32_t K, const float *depth,
                    const gg_tsdf_params *prm, void *ws, size_t ws_bytes, void *stream);
int tsdf_integrate_tabled(const gg_camera *src, int32_t K, const gg_camera *tgt,
                          const gg_tsdf_params *prm, const float *temporal_mask,
                          const float *F_prev, const float *W_prev, float *F, float *W,
                          float *out_depth, int32_t *out_bin, const gg_volume_tuning *tuning,
                          void *ws, size_t ws_bytes, void *stream);

/* tsdf_integrate without a workspace argument and without allocating: for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Arguments, results
 * and errors are those of tsdf_integrate (bitwise the same outputs); the
 * scratch (the view table and the bin table) is a static device array of the
 * library, GG_NOALLOC_SCRATCH_BYTES (64 MiB) per device, held from the first
 * call on a device until the process ends.  A call whose workspace would
 * exceed it (gg_workspace_size(GG_OP_TSDF_INTEGRATE, ...) > 64 MiB, e.g.
 * more than about 8.3 M source pixels over all views) returns
 * GG_ERR_UNSUPPORTED before anything is enqueued.  Every call on one device
 * shares that device's scratch, which keeps the last call's contents and is
 * fully rewritten before it is read: calls that overlap on one device (other
 * streams, other threads) race and must be ordered by the caller. */
#define GG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int tsdf_integrate_noalloc(const gg_camera *src, int32_t K, const float *depth,
                           const gg_camera *tgt, const gg_tsdf_params *prm,
                           const float *temporal_mask, const float *F_prev, const float *W_prev,
                           float *F, float *W, float *out_depth, int32_t *out_bin,
                           const gg_volume_tuning *tuning, void *stream);

/* tsdf_extract_depth -- the surface is where the fused signed distance
 * changes sign along the ray (Suppl. A.1).  On the bins: d* = the smallest
 * d in [0, D-2] with W_d > 0, W_{d+1} > 0, F_d > 0 and F_{d+1} <= 0;
 * out_depth = z_d + (z_{d+1} - z_d) F_d / (F_d - F_{d+1}), out_bin = d*;
 * no crossing: 0 and -1.  F, W float tgt_h x tgt_w x D.  tuning [host]: the
 * launch shape or NULL (results do not depend on it). */
int tsdf_extract_depth(const gg_camera *tgt, const gg_tsdf_params *prm, const float *F,
                       const float *W, float *out_depth, int32_t *out_bin,
                       const gg_volume_tuning *tuning, void *stream);

/* Adjoint of tsdf_extract_depth: for L = <g_depth, out_depth>,
 * g_F2[p] = (dL/dF_{d*}, dL/dF_{d*+1}) at the pixel's crossing (0, 0 where
 * bin < 0).  bin: the out_bin of the forward.  g_F2 float tgt_h x tgt_w x 2. */
int tsdf_extract_depth_backward(const gg_camera *tgt, const gg_tsdf_params *prm,
                                const float *F, const float *W, const int32_t *bin,
                                const float *g_depth, float *g_F2, void *stream);

/* Adjoint of tsdf_integrate with respect to the input depths, given the
 * gradient g_F2 on the two voxels per pixel that extraction read (d*, d*+1;
 * pixels with bin < 0 carry none).  The per-view terms of those voxels are
 * recomputed from the inputs and the post-update F, W (nothing per voxel is
 * stored between forward and backward).  No gradient reaches F_prev, W_prev,
 * the mask or the cameras.  Discrete choices (sampled pixel, occlusion,
 * clamp, the min of the fusion weight) are held fixed.
 * Arguments as tsdf_integrate, with F, W the forward's outputs (call before
 * the next frame overwrites them), bin its out_bin; g_depth_in float
 * K x src_h x src_w is overwritten.  Scatter uses 64-bit fixed-point atomics
 * with a data-derived scale, so the result is deterministic: with m the
 * largest bound |g_F| max(1, tau + |F|) / W over the pixels' two voxels (FP32)
 * and 2^(e-1) <= 2 m tgt_w tgt_h < 2^e, every term is rounded to the quantum
 * 2^-(61-e), which keeps every sum below 2^61 in magnitude. */
int tsdf_integrate_backward(const gg_camera *src, int32_t K, const float *depth,
                            const gg_camera *tgt, const gg_tsdf_params *prm, const float *F,
                            const float *W, const int32_t *bin, const float *g_F2,
                            float *g_depth_in, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Batched path: many target views of uneven resolution, view count and bin
 * count (each with its own inputs, cameras, parameters, volume and outputs)
 * fused by kernels over per-phase work lists (persistent ones for the splat
 * binning, one workgroup per tile for the others) in one hipGraph launch.
 * Every output is
 * bitwise identical to the plain calls (splat_views + tsdf_integrate with
 * fused extraction) on the same item, for any tuning.
 * ------------------------------------------------------------------------- */
typedef struct gg_batch_item {
  const gg_camera *src;         /* [host] K source cameras, one size per item        */
  int32_t K;
  const float *depth;           /* K x src_h x src_w                                 */
  const uint8_t *rgb;           /* K x src_h x src_w x 3, or NULL: no splat          */
  gg_camera tgt;
  gg_splat_params splat;
  gg_tsdf_params tsdf;
  const float *temporal_mask;   /* tgt_h x tgt_w or NULL                             */
  const float *F_prev, *W_prev; /* both or neither; may alias F, W                   */
  float *F, *W;                 /* tgt_h x tgt_w x D                                 */
  float *out_depth;             /* tgt_h x tgt_w or NULL (with out_bin)              */
  int32_t *out_bin;
  int32_t *win_idx;             /* splat outputs, as splat_views (required with rgb) */
  float *sp_depth, *sp_rgb, *sp_alpha;
  float *sp_tape;               /* or NULL                                           */
  gg_volume_tuning volume;      /* this item's fusion launch shape, as tsdf_integrate
                                   takes it (all 0: the plan's pixels_per_block and
                                   bins_per_thread, bands of 256 pixels); invalid
                                   values fail the plan with GG_ERR_INVALID         */
} gg_batch_item;

/* Launch shape chosen by the autotuner (0 = default). */
typedef struct gg_batch_tuning {
  int32_t pixels_per_block; /* target pixels per fusion workgroup, 0..1024 (0: 16; fewer
                               where the workgroup would exceed 1024 threads)             */
  int32_t blocks_per_cu;   /* resident workgroups per compute unit of the persistent splat
                              binning phases, 0..64 (0: as many as fit)                    */
  int32_t bins_per_thread; /* of the fusion, as in gg_volume_tuning (0: default)            */
  int32_t branches;        /* 0 or 2: the splat phases form a branch of the graph that runs
                              beside the fusion; 1: every phase in one sequence          */
} gg_batch_tuning;

typedef struct gg_batch gg_batch;

/* Validates every item (as the plain calls do), allocates the plan's device
 * memory (descriptors, work lists, workspaces: gg_batch_device_bytes),
 * uploads descriptors and captures the phases into a graph.  The plan binds
 * the items' device pointers: refill those buffers between launches.  This
 * call allocates and synchronises; gg_batch_launch does neither. */
int gg_batch_plan(const gg_batch_item *items, int32_t n, const gg_batch_tuning *tuning,
                  gg_batch **plan);
/* One graph launch running the whole batch on `stream`. */
int gg_batch_launch(gg_batch *plan, void *stream);
size_t gg_batch_device_bytes(const gg_batch *plan);
/* Frees the plan (call after its last launch has completed). */
int gg_batch_free(gg_batch *plan);

/* ---------------------------------------------------------------------------
 * Utilities.
 * ------------------------------------------------------------------------- */

/* Message of the last failing call on this thread ("" if none). */
const char *gg_last_error(void);

/* The relative projection a -> b [host, no GPU work]: a pixel centre
 * (px, py) of camera a at camera-a depth z maps to
 * (x_b, y_b, z_b) = z * H (px, py, 1)^T + c  (exact in real arithmetic),
 * H = K_b R_b R_a^T K_a^{-1}, c = K_b (t_b - R_b R_a^T t_a): the FP32
 * rounding (to nearest, ties to even) of the exact products, formed in
 * binary128; an entry below 2^-50 of its terms' summed magnitudes is 0.
 * H [host] 9 floats row-major, c [host] 3. */
int gg_relative_projection(const gg_camera *a, const gg_camera *b, float *H, float *c);

/* Measurement utility: the fusion kernel of tsdf_integrate launched in the
 * launch shape of `tuning` with no views, so that it
 * moves exactly its volume stream -- F_prev and W_prev read, F and W
 * written (16 bytes per voxel, may alias), the fused extraction -- and none
 * of the view-table gathers: the ceiling of the fusion's memory access
 * pattern on this device.  Each voxel only decays its carried weight:
 * W = min(decay W_prev, weight_cap), F = (W F_prev) / W (0 where W is 0).
 * Arguments as tsdf_integrate; out_depth and out_bin are required; ws:
 * gg_workspace_size(GG_OP_TSDF_INTEGRATE, 1, 1, 1, tgt_w, tgt_h, D, NULL). */
int gg_fusion_stream_probe(const gg_camera *tgt, const gg_tsdf_params *prm,
                           const float *F_prev, const float *W_prev, float *F, float *W,
                           float *out_depth, int32_t *out_bin, const gg_volume_tuning *tuning,
                           void *ws, size_t ws_bytes, void *stream);

/* Self-check of the correctly rounded reciprocal the fusion kernels use for
 * 1/z: for every FP32 value with biased exponent in [e_lo, e_hi] (all 2^23
 * significands of each), compares it bitwise with IEEE division on the
 * device and adds the number of mismatches to *mismatches (a device
 * counter the caller zeroes).  For the test suite. */
int gg_selftest_reciprocal(int32_t e_lo, int32_t e_hi, unsigned long long *mismatches,
                           void *stream);

/* The kernels' reciprocal 1/z (z > 0) of n device floats, for comparison
 * with a host reference.  For the test suite. */
int gg_fast_reciprocal(const float *in, float *out, int64_t n, void *stream);

/* Kernel timing for profiling: when enabled, every kernel the library
 * launches is bracketed by HIP events on its stream.  gg_timing_read
 * synchronises on the recorded events and returns the summed milliseconds
 * and the number of launches of kernels whose name contains `name` (all if
 * NULL) since the last gg_timing_reset. */
int gg_timing_enable(int on);
/* Restrict the timing to kernels whose name contains `name` (NULL or "":
 * all), so that a timed region brackets only the launches it reports. */
int gg_timing_filter(const char *name);
int gg_timing_reset(void);
int gg_timing_read(const char *name, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* GGEOM_H */
