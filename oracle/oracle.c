/*
 * oracle.c -- plain CPU reference of the geometry stage of "Geometry-guided
 * Online 3D Video Synthesis with Multi-View Temporal Consistency"
 * (arXiv 2505.18932).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP library: it is written from the paper and the written readings of
 * the paper only.
 *
 * What it computes (one function per step, each citing its passage):
 *   orc_relproj      -- the projection (x_k, y_k, z_k) = K_k (R_k p + t_k) of
 *                       Suppl. A.1, written for a point at depth z on a pixel
 *                       ray of another camera (exact in real arithmetic).
 *   orc_confidence   -- the noise-aware weight omega_k and the window
 *                       statistic nu_k of Suppl. A.1.
 *   orc_bins         -- the depth samples along each target ray.
 *   orc_integrate    -- the fused truncated signed distance of Suppl. A.1
 *                       (sum of omega_k * clamp(s_k, -tau, tau), occlusion
 *                       cut s_k < -tau => omega_k = 0) plus the temporal
 *                       weight of Suppl. A.2 carried per voxel.
 *   orc_extract      -- the sign change along the ray of Suppl. A.1.
 *   orc_network_inputs, orc_blend -- the geometry maps the blending network
 *                       takes (§3.3 and the supplement's network inputs) and
 *                       the blend of Eq. 4-5 for given weights.
 *   orc_raymarch     -- the volume-free form of the same fusion: the march
 *                       along each target ray with step 0.8 s and three
 *                       bisections of Suppl. A.1, with the previous output
 *                       depth as one more input (Suppl. A.2).
 *   orc_splat        -- forward rendering of per-pixel Gaussians of §3.1 and
 *                       Suppl. A.3 as a z-buffered splat; orc_splat_masked
 *                       also carries a per-pixel scalar (the difference
 *                       mask) and its maximum over the views (Suppl. A.2).
 *   orc_splat_ewa    -- the same pixel Gaussians projected with EWA
 *                       (anisotropic image-space covariance) and composited
 *                       front to back in depth order, as the 3D Gaussian
 *                       renderer the paper uses does (§3.1).
 *   orc_difference_mask -- the soft colour-difference mask of Eq. 1 at
 *                       quarter resolution, max-pooled and upsampled (§3.2).
 *   orc_temporal_filter -- the temporally filtered depth of Eq. 2 (§3.2).
 *   *_backward       -- the adjoints of the above with respect to input depth
 *                       and colour.
 *
 * Arithmetic: this file is compiled twice.  The default build computes in
 * FP32 (the precision of the workload's depth maps and volumes, and the
 * precision in which the GPU takes its integer decisions: pixel floors,
 * z-test winners and the zero-crossing bin) in the operation order written
 * below, with no contraction (-ffp-contract=off): every fused multiply-add is
 * an explicit fmaf.  Built with -DORC_DOUBLE every computed quantity is FP64;
 * that build serves the finite-difference gradient checks and bounds the FP32
 * rounding.  Inputs (cameras, depth, colour) are FP32 / uint8 in both builds.
 *
 * Readings of the paper that this file implements where the paper is silent
 * or garbled (sign convention, sampling, pixel centres, border handling of the
 * window statistic, per-voxel temporal carry, extraction on dense bins,
 * coverage and band of the z-buffered splat) are listed in the repository's
 * design notes; each is marked "reading" at the line that takes it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef ORC_DOUBLE
typedef double real;
#define RFMA fma
#define RSQRT sqrt
#define REXP exp
#define RLOG log
#define RMIN fmin
#define RMAX fmax
#define RABS fabs
#define ORC_PREC 64
#else
typedef float real;
#define RFMA fmaf
#define RSQRT sqrtf
#define REXP expf
#define RLOG logf
#define RMIN fminf
#define RMAX fmaxf
#define RABS fabsf
#define ORC_PREC 32
#endif

typedef struct {
  float fx, fy, cx, cy;
  float R[9]; /* world -> camera rotation, row-major */
  float t[3];
  int32_t width, height;
} orc_camera;

typedef struct {
  float sigma_px;  /* source-image std of a pixel Gaussian, in source pixels */
  float band_rel;  /* band of the blend: z <= z_winner * (1 + band_rel)     */
  float z_min;     /* splats with target z <= z_min are dropped             */
  float r_max_px;  /* cap on the coverage radius, target pixels             */
} orc_splat_params;

typedef struct {
  float z_near, z_far;
  int32_t num_bins;
  float trunc;
  int32_t trunc_in_bins;
  float conf_tau, conf_scale;
  int32_t conf_window;
  float decay, weight_cap;
} orc_tsdf_params;

int orc_precision(void) { return ORC_PREC; }

/* A depth sample is usable iff it is positive and finite (holes are 0). */
static int depth_ok(float d) { return d > 0.0f && d < INFINITY; }

/* ------------------------------------------------------------------------
 * Relative projection (Suppl. A.1 projection equation).
 *
 * A pixel centre (px, py) of camera a at camera-a depth z is the world point
 *   p = R_a^T (z K_a^{-1} (px, py, 1)^T - t_a).
 * Its image in camera b, K_b (R_b p + t_b), is exactly
 *   z * H (px, py, 1)^T + c,   H = K_b R_b R_a^T K_a^{-1},
 *                              c = K_b (t_b - R_b R_a^T t_a),
 * i.e. affine in z along the ray.  H and c are these plain matrix products,
 * each 3 x 3 factor written out from the camera (K_a^{-1} = [[1/fx, 0,
 * -cx/fx], [0, 1/fy, -cy/fy], [0, 0, 1]]), evaluated right to left in
 * binary128 (113-bit significand) and rounded once to the working
 * precision.  Reading: the constants are the rounding of the exact products;
 * binary128 carries them to far below an FP32 (or FP64) rounding step, also
 * where an entry is the small difference of large terms, so the rounded
 * value does not depend on the order of evaluation.  An entry whose value
 * is below 2^-50 of the sum of the magnitudes of the monomials forming it
 * (the same products over the entries' magnitudes) is pure cancellation
 * residue (an identity pair's off-diagonal terms, say) and is taken as 0:
 * binary128 leaves such residues order-dependent, the threshold does not.
 * ---------------------------------------------------------------------- */
typedef __float128 quad;

static void q3_mul(const quad A[9], const quad B[9], quad C[9]) {
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      quad acc = 0;
      for (int m = 0; m < 3; ++m) acc += A[3 * r + m] * B[3 * m + k];
      C[3 * r + k] = acc;
    }
}

static void q3_vec(const quad A[9], const quad x[3], quad y[3]) {
  for (int r = 0; r < 3; ++r) {
    quad acc = 0;
    for (int m = 0; m < 3; ++m) acc += A[3 * r + m] * x[m];
    y[r] = acc;
  }
}

static quad qabs(quad x) { return x < 0 ? -x : x; }

/* H = K_b R_b R_a^T K_a^{-1} and c = K_b (t_b - R_b R_a^T t_a) from the
 * factors M1 .. M4 (row-major), and with every factor replaced by its
 * entrywise magnitude, the sums of the monomials' magnitudes (Hm, cm). */
static void relproj_q(const orc_camera *a, const orc_camera *b, quad H[9], quad c[3], quad Hm[9],
                      quad cm[3]) {
  const quad fxa = a->fx, fya = a->fy;
  const quad Kb[9] = {b->fx, 0, b->cx, 0, b->fy, b->cy, 0, 0, 1};
  const quad Kai[9] = {1 / fxa, 0, -(quad)a->cx / fxa, 0, 1 / fya, -(quad)a->cy / fya, 0, 0, 1};
  quad Rb[9], RaT[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      Rb[3 * r + k] = b->R[3 * r + k];
      RaT[3 * r + k] = a->R[3 * k + r];
    }
  const quad ta[3] = {a->t[0], a->t[1], a->t[2]};
  const quad tb[3] = {b->t[0], b->t[1], b->t[2]};
  for (int pass = 0; pass < 2; ++pass) {
    /* pass 0: the values; pass 1: the same products over magnitudes */
    quad kb[9], kai[9], rb[9], rat[9], xa[3], xb[3];
    for (int i = 0; i < 9; ++i) {
      kb[i] = pass ? qabs(Kb[i]) : Kb[i];
      kai[i] = pass ? qabs(Kai[i]) : Kai[i];
      rb[i] = pass ? qabs(Rb[i]) : Rb[i];
      rat[i] = pass ? qabs(RaT[i]) : RaT[i];
    }
    for (int i = 0; i < 3; ++i) {
      xa[i] = pass ? qabs(ta[i]) : ta[i];
      xb[i] = pass ? qabs(tb[i]) : tb[i];
    }
    quad T1[9], T2[9], u[3], v[3], e[3];
    quad *Ho = pass ? Hm : H, *co = pass ? cm : c;
    q3_mul(rat, kai, T1); /* R_a^T K_a^{-1}            */
    q3_mul(rb, T1, T2);   /* R_b R_a^T K_a^{-1}        */
    q3_mul(kb, T2, Ho);   /* K_b R_b R_a^T K_a^{-1}    */
    q3_vec(rat, xa, u);   /* R_a^T t_a                 */
    q3_vec(rb, u, v);     /* R_b R_a^T t_a             */
    for (int r = 0; r < 3; ++r) e[r] = pass ? xb[r] + v[r] : xb[r] - v[r];
    q3_vec(kb, e, co);    /* K_b (t_b - R_b R_a^T t_a) */
  }
  const quad tiny = 0x1p-50Q;
  for (int i = 0; i < 9; ++i)
    if (qabs(H[i]) < tiny * Hm[i]) H[i] = 0;
  for (int i = 0; i < 3; ++i)
    if (qabs(c[i]) < tiny * cm[i]) c[i] = 0;
}

/* FP64 rounding (the FP64 oracle and the tests' world-space check). */
void orc_relproj_d(const orc_camera *a, const orc_camera *b, double H[9], double c[3]) {
  quad Hq[9], cq[3], Hm[9], cm[3];
  relproj_q(a, b, Hq, cq, Hm, cm);
  for (int i = 0; i < 9; ++i) H[i] = (double)Hq[i];
  for (int i = 0; i < 3; ++i) c[i] = (double)cq[i];
}

/* Round to FP32 a binary128 value x that stands for an exact product whose
 * monomials' magnitudes sum to m.  The binary128 evaluation is off by far
 * less than 2^-100 m, so x rounds as the exact value does -- except at an
 * exact tie (the exact value halfway between two floats, which rigs aligned
 * with the axes produce), where that error alone would pick the side.  So a
 * point within 2^-100 m of the halfway point between the floats below and
 * above x counts as the tie, which goes to the float whose last significand
 * bit is 0. */
static float to_f32(quad x, quad m) {
  float f = (float)x, below, above;
  uint32_t u;
  memcpy(&u, &f, 4);
  /* the float on the other side of x: one step of the bit pattern (the
   * pattern grows with |f|) */
  const int up = ((quad)f <= x) == (f >= 0);
  uint32_t w = up ? u + 1u : u - 1u;
  if (f == 0) w = ((quad)f <= x) ? 1u : 0x80000001u;
  float g;
  memcpy(&g, &w, 4);
  below = f < g ? f : g;
  above = f < g ? g : f;
  const quad half = ((quad)below + (quad)above) / 2;
  if (qabs(x - half) <= 0x1p-100Q * m) {
    uint32_t lb;
    memcpy(&lb, &below, 4);
    return (lb & 1u) == 0 ? below : above;
  }
  return f;
}

/* The relative projection in the oracle's working precision. */
static void relproj(const orc_camera *a, const orc_camera *b, real H[9], real c[3]) {
  quad Hq[9], cq[3], Hm[9], cm[3];
  relproj_q(a, b, Hq, cq, Hm, cm);
  for (int i = 0; i < 9; ++i) H[i] = sizeof(real) == 4 ? (real)to_f32(Hq[i], Hm[i]) : (real)Hq[i];
  for (int i = 0; i < 3; ++i) c[i] = sizeof(real) == 4 ? (real)to_f32(cq[i], cm[i]) : (real)cq[i];
}

/* Exported FP32 rounding of the relative projection (for tests). */
void orc_relproj(const orc_camera *a, const orc_camera *b, float H[9], float c[3]) {
  quad Hq[9], cq[3], Hm[9], cm[3];
  relproj_q(a, b, Hq, cq, Hm, cm);
  for (int i = 0; i < 9; ++i) H[i] = to_f32(Hq[i], Hm[i]);
  for (int i = 0; i < 3; ++i) c[i] = to_f32(cq[i], cm[i]);
}

/* The ray of pixel centre (px, py): h = H (px, py, 1)^T, fused per row. */
static void ray_of(const real H[9], real px, real py, real h[3]) {
  for (int r = 0; r < 3; ++r) h[r] = RFMA(H[3 * r + 0], px, RFMA(H[3 * r + 1], py, H[3 * r + 2]));
}

/* The point at depth z on that ray, in the other camera's homogeneous
 * pixel coordinates: X = z h + c (x_k, y_k, z_k of Suppl. A.1). */
static void point_at(const real h[3], const real c[3], real z, real X[3]) {
  for (int r = 0; r < 3; ++r) X[r] = RFMA(z, h[r], c[r]);
}

/* ------------------------------------------------------------------------
 * Noise-aware fusion weight (Suppl. A.1):
 *   nu_k = sum over the w x w window N of min((D_k[u,v] - D_k[p,q])^2, tau^2)
 *   omega_k = min(0.001 * (nu_k / (w w))^(-1/2), 1)
 * evaluated around the pixel that nearest sampling picks, so it is a map over
 * the input pixels.  Readings: window offsets visited row-major; neighbours
 * outside the image are skipped; hole neighbours contribute tau^2; the
 * divisor stays w*w; nu = 0 gives omega = 1 (the limit of the min); a hole
 * pixel has omega = 0.
 * ---------------------------------------------------------------------- */
void orc_confidence(const float *depth, int W, int H, const orc_tsdf_params *p, real *conf) {
  const int r = (p->conf_window - 1) / 2;
  const real tw2 = (real)p->conf_tau * (real)p->conf_tau;
  const real n2 = (real)(p->conf_window * p->conf_window);
#pragma omp parallel for schedule(static)
  for (int j = 0; j < H; ++j)
    for (int i = 0; i < W; ++i) {
      const float dq = depth[(size_t)j * W + i];
      if (!depth_ok(dq)) {
        conf[(size_t)j * W + i] = 0;
        continue;
      }
      real nu = 0;
      for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
          const int ii = i + dx, jj = j + dy;
          if (ii < 0 || ii >= W || jj < 0 || jj >= H) continue;
          const float dn = depth[(size_t)jj * W + ii];
          real term;
          if (depth_ok(dn)) {
            const real dd = (real)dq - (real)dn;
            term = RMIN(dd * dd, tw2);
          } else {
            term = tw2;
          }
          nu = nu + term;
        }
      conf[(size_t)j * W + i] = (nu == 0) ? (real)1 : RMIN((real)p->conf_scale / RSQRT(nu / n2), (real)1);
    }
}

/* ------------------------------------------------------------------------
 * Depth samples along a target ray.  Reading: the paper marches the ray with
 * steps of 0.8 s; the volume form samples it at num_bins depths uniform in
 * inverse depth from z_near to z_far, and expresses a truncation given "in
 * bins" as the local metric width of that many bins, tau_d = N du z_d^2.
 * ---------------------------------------------------------------------- */
void orc_bins(const orc_tsdf_params *p, real *z, real *tau) {
  const int D = p->num_bins;
  const real un = (real)1 / (real)p->z_near;
  const real uf = (real)1 / (real)p->z_far;
  const real du = (un - uf) / (real)(D - 1);
  for (int d = 0; d < D; ++d) {
    const real u = un - (real)d * du;
    z[d] = (real)1 / u;
    tau[d] = p->trunc_in_bins ? ((real)p->trunc * du) * (z[d] * z[d]) : (real)p->trunc;
  }
}

/* ------------------------------------------------------------------------
 * Fusion of K depth maps into the target's frustum volume (Suppl. A.1) with
 * the temporal weight of Suppl. A.2 carried per voxel.
 *
 * For voxel (x, y, d) at depth z_d on the ray of target pixel (x, y):
 *   for each view k (in order): project, X = (x_k, y_k, z_k); skip unless
 *   z_k > 0; (u, v) = (x_k / z_k, y_k / z_k) evaluated as x_k * (1 / z_k);
 *   nearest sample (reading): pixel (floor u, floor v), skip if outside or a
 *   hole; s_k = D_k - z_k (reading: positive in front of the surface, so that
 *   "omega_k = 0 if s_k < -tau" drops samples occluded in view k);
 *   skip if s_k < -tau_d; S += omega_k * min(s_k, tau_d); Wo += omega_k.
 * Temporal carry (reading of Suppl. A.2, per voxel): with m = max(1 - M, 0)
 * (1 without a mask), omega_tmp = min(decay * W_prev * m, cap),
 * W = omega_tmp + Wo, F = (omega_tmp F_prev + S) / W (0 where W = 0).
 * Reading: F is the weighted mean rather than the paper's unnormalised sum;
 * the sign, and hence the surface, is the same.
 *
 * pixels/npix select target pixels (NULL: all, in row-major order); volumes
 * F/W (and F_prev/W_prev) then hold npix x D values in that order.
 * conf may be NULL, in which case it is computed here.
 * ---------------------------------------------------------------------- */
int orc_integrate(const orc_camera *src, int K, const float *depth, const real *conf_in,
                  const orc_camera *tgt, const orc_tsdf_params *p, const float *mask,
                  const real *F_prev, const real *W_prev, real *F, real *W,
                  const int32_t *pixels, int npix) {
  const int D = p->num_bins;
  const int Ws = src[0].width, Hs = src[0].height;
  const size_t ns = (size_t)Ws * Hs;
  if (K < 1 || D < 2) return -1;
  real *conf = (real *)conf_in;
  if (!conf) {
    conf = (real *)malloc(sizeof(real) * ns * K);
    if (!conf) return -2;
    for (int k = 0; k < K; ++k) orc_confidence(depth + ns * k, Ws, Hs, p, conf + ns * k);
  }
  real *zb = (real *)malloc(sizeof(real) * D), *tb = (real *)malloc(sizeof(real) * D);
  real (*Hk)[9] = malloc(sizeof(real[9]) * K);
  real (*ck)[3] = malloc(sizeof(real[3]) * K);
  orc_bins(p, zb, tb);
  for (int k = 0; k < K; ++k) relproj(tgt, &src[k], Hk[k], ck[k]);
  const int total = pixels ? npix : tgt->width * tgt->height;
  const real cap = (real)p->weight_cap, decay = (real)p->decay;
#pragma omp parallel for schedule(dynamic, 64)
  for (int n = 0; n < total; ++n) {
    const int pix = pixels ? pixels[n] : n;
    const int x = pix % tgt->width, y = pix / tgt->width;
    real h[16][3];
    for (int k = 0; k < K; ++k) ray_of(Hk[k], (real)x + (real)0.5, (real)y + (real)0.5, h[k]);
    const real m = mask ? RMAX((real)1 - (real)mask[pix], (real)0) : (real)1;
    for (int d = 0; d < D; ++d) {
      const real z = zb[d], tau = tb[d];
      real S = 0, Wo = 0;
      for (int k = 0; k < K; ++k) {
        real X[3];
        point_at(h[k], ck[k], z, X);
        if (!(X[2] > 0)) continue;
        const real inv = (real)1 / X[2];
        const real u = X[0] * inv, v = X[1] * inv;
        if (!(u >= 0 && u < (real)Ws && v >= 0 && v < (real)Hs)) continue;
        const size_t q = (size_t)(int)v * Ws + (size_t)(int)u; /* floor: u, v >= 0 */
        const float Dk = depth[ns * k + q];
        if (!depth_ok(Dk)) continue;
        const real s = (real)Dk - X[2];
        if (s < -tau) continue; /* occluded in view k */
        const real cval = RMIN(s, tau);
        const real w = conf[ns * k + q];
        S = RFMA(w, cval, S);
        Wo = Wo + w;
      }
      const size_t o = (size_t)n * D + d;
      const real wp = (W_prev) ? RMIN((decay * W_prev[o]) * m, cap) : (real)0;
      const real Wn = wp + Wo;
      const real Fp = (W_prev) ? F_prev[o] : (real)0;
      F[o] = (Wn > 0) ? RFMA(wp, Fp, S) / Wn : (real)0;
      W[o] = Wn;
    }
  }
  if (!conf_in) free(conf);
  free(zb);
  free(tb);
  free(Hk);
  free(ck);
  return 0;
}

/* ------------------------------------------------------------------------
 * Volume-free TSDF raymarch (Suppl. A.1: advance along the ray by 0.8 s until
 * s changes sign, then three bisection steps; Suppl. A.2: the previous
 * output depth as one more input with the temporal weight).
 *
 * Fused value at target depth z on the ray of target pixel (x, y): the views
 * in order with the projection, sampling, sign, occlusion and clamp rules of
 * orc_integrate, tau(z) = trunc du z^2 (trunc in bins) or trunc:
 * S = sum omega_k min(s_k, tau), Wo = sum omega_k over kept samples; then,
 * where the pixel has a previous depth Dp > 0 and omega_tmp > 0, one more
 * sample s = Dp - z with weight omega_tmp (same occlusion cut and clamp).
 * Wt = Wo (+ omega_tmp when kept); s(z) = S / Wt, no value (unobserved)
 * where Wt = 0.  Temporal weight (Suppl. A.2): omega_tmp =
 * min((decay acc) m, cap), m = max(1 - M, 0) (1 without a mask), acc the
 * pixel's accumulated weight from the previous frame.
 *
 * March (readings; the paper gives the step rule only): with
 * step_min(z) = (du z) z, the width of one inverse-depth bin at z,
 *   observed, s > 0 : z <- z + max(0.8 s, step_min(z))
 *   observed, s <= 0: a surface if the previous sample was observed with
 *                     s > 0, else z <- z + step_min(z)
 *   unobserved      : z <- z + 0.8 tau(z)
 * from z = z_near while z <= z_far (at most 4 D + 16 samples); no surface:
 * depth 0, acc_next 0.  Bracket [a, b], s(a) > 0 >= s(b); three bisections
 * m = a + (b - a) * 0.5, a = m if s(m) is observed and > 0, else b = m;
 * depth = a + (b - a) * 0.5.  acc_next = omega_tmp + Wo at that depth (the
 * accumulated weight of Suppl. A.2 for the next frame).
 * dprev, acc, mask: Ht x Wt or NULL (no temporal term without dprev and
 * acc).  out_depth, out_acc (nullable), out_steps (nullable: samples taken
 * before the bisection): Ht x Wt.
 * ---------------------------------------------------------------------- */
typedef struct {
  real S, Wo, Wt;
} orc_fused;

static orc_fused fused_at(real z, real tau, int K, real (*h)[3], real (*ck)[3], const float *depth,
                          const real *conf, int Ws, int Hs, real wtmp, real Dp) {
  const size_t ns = (size_t)Ws * Hs;
  orc_fused f = {0, 0, 0};
  for (int k = 0; k < K; ++k) {
    real X[3];
    point_at(h[k], ck[k], z, X);
    if (!(X[2] > 0)) continue;
    const real inv = (real)1 / X[2];
    const real u = X[0] * inv, v = X[1] * inv;
    if (!(u >= 0 && u < (real)Ws && v >= 0 && v < (real)Hs)) continue;
    const size_t q = (size_t)(int)v * Ws + (size_t)(int)u;
    const float Dk = depth[ns * k + q];
    if (!depth_ok(Dk)) continue;
    const real s = (real)Dk - X[2];
    if (s < -tau) continue;
    const real w = conf[ns * k + q];
    f.S = RFMA(w, RMIN(s, tau), f.S);
    f.Wo = f.Wo + w;
  }
  f.Wt = f.Wo;
  if (wtmp > 0 && Dp > 0) {
    const real s = Dp - z;
    if (!(s < -tau)) {
      f.S = RFMA(wtmp, RMIN(s, tau), f.S);
      f.Wt = f.Wt + wtmp;
    }
  }
  return f;
}

int orc_raymarch(const orc_camera *src, int K, const float *depth, const orc_camera *tgt,
                 const orc_tsdf_params *p, const real *dprev, const real *acc, const float *mask,
                 real *out_depth, real *out_acc, int32_t *out_steps) {
  const int D = p->num_bins;
  const int Ws = src[0].width, Hs = src[0].height;
  const size_t ns = (size_t)Ws * Hs;
  if (K < 1 || K > 16 || D < 2) return -1;
  real *conf = (real *)malloc(sizeof(real) * ns * K);
  if (!conf) return -2;
  for (int k = 0; k < K; ++k) orc_confidence(depth + ns * k, Ws, Hs, p, conf + ns * k);
  real Hk[16][9], ck[16][3];
  for (int k = 0; k < K; ++k) relproj(tgt, &src[k], Hk[k], ck[k]);
  const real un = (real)1 / (real)p->z_near, uf = (real)1 / (real)p->z_far;
  const real du = (un - uf) / (real)(D - 1);
  const real zn = (real)p->z_near, zf = (real)p->z_far;
  const real cap = (real)p->weight_cap, decay = (real)p->decay;
  const int max_samples = 4 * D + 16;
  const int npix = tgt->width * tgt->height;
#pragma omp parallel for schedule(dynamic, 64)
  for (int n = 0; n < npix; ++n) {
    const int x = n % tgt->width, y = n / tgt->width;
    real h[16][3];
    for (int k = 0; k < K; ++k) ray_of(Hk[k], (real)x + (real)0.5, (real)y + (real)0.5, h[k]);
    real wtmp = 0, Dp = 0;
    if (dprev && acc) {
      const real m = mask ? RMAX((real)1 - (real)mask[n], (real)0) : (real)1;
      wtmp = RMIN((decay * acc[n]) * m, cap);
      Dp = dprev[n];
    }
#define TAU_AT(zz) (p->trunc_in_bins ? ((real)p->trunc * du) * ((zz) * (zz)) : (real)p->trunc)
    real z = zn, zprev = 0;
    int prev_pos = 0, found = 0, steps = 0;
    while (z <= zf && steps < max_samples) {
      const real tau = TAU_AT(z);
      const orc_fused f = fused_at(z, tau, K, h, ck, depth, conf, Ws, Hs, wtmp, Dp);
      ++steps;
      const real smin = (du * z) * z;
      if (f.Wt > 0) {
        const real s = f.S / f.Wt;
        if (s > 0) {
          zprev = z;
          prev_pos = 1;
          z = z + RMAX((real)0.8 * s, smin);
        } else if (prev_pos) {
          found = 1;
          break;
        } else {
          prev_pos = 0;
          z = z + smin;
        }
      } else {
        prev_pos = 0;
        z = z + (real)0.8 * tau;
      }
    }
    real dep = 0, an = 0;
    if (found) {
      real a = zprev, b = z;
      for (int it = 0; it < 3; ++it) {
        const real mid = a + (b - a) * (real)0.5;
        const orc_fused f = fused_at(mid, TAU_AT(mid), K, h, ck, depth, conf, Ws, Hs, wtmp, Dp);
        if (f.Wt > 0 && f.S / f.Wt > 0)
          a = mid;
        else
          b = mid;
      }
      dep = a + (b - a) * (real)0.5;
      const orc_fused f = fused_at(dep, TAU_AT(dep), K, h, ck, depth, conf, Ws, Hs, wtmp, Dp);
      an = wtmp + f.Wo;
    }
#undef TAU_AT
    out_depth[n] = dep;
    if (out_acc) out_acc[n] = an;
    if (out_steps) out_steps[n] = steps;
  }
  free(conf);
  return 0;
}

/* ------------------------------------------------------------------------
 * Inputs of the blending network (§3.3; the supplement's list of network
 * inputs): a (9K + 1) x H x W stack of planes,
 *   [0, 3K)      forward-rendered images I_k (3 planes per view, view-major),
 *   [3K, 4K)     forward-rendered depths D_k (the splat's winner depths),
 *   [4K, 5K)     alphas alpha_k,
 *   5K           the TSDF depth D^t,
 *   [5K+1, 6K+1) dot(input-view ray direction, TSDF normal),
 *   [6K+1, 7K+1) dot(input-view ray direction, target ray direction),
 *   [7K+1, 8K+1) distance between input and target camera centres,
 *   [8K+1, 9K+1) dot(input and target optical axes).
 * Readings: the surface point X(p) is target pixel p back-projected at D^t(p)
 * (X = C_t + D a with a = R_t^T K_t^-1 (px, py, 1), evaluated affine in D as
 * fma(D, a_r, C_r)); the normal is the normalised cross product of the
 * horizontal and vertical differences of neighbouring surface points
 * (central where both neighbours have a depth, else one-sided, else none),
 * oriented towards the target camera; the input-view ray direction is
 * (X - C_k) / |X - C_k|; the target ray direction a / |a|.  Pixels without a
 * TSDF depth (or a normal) get 0 in the dot-product planes.  Centres, axes,
 * distances and the matrix R_t^T K_t^-1 are formed in FP64 from the FP32
 * cameras and rounded once.  Sums of three products are evaluated left to
 * right without fused multiply-adds; cross products as a b - c d.
 * ---------------------------------------------------------------------- */
static void cam_centre_d(const orc_camera *c, double C[3]) {
  for (int r = 0; r < 3; ++r) {
    double v = 0;
    for (int k = 0; k < 3; ++k) v -= (double)c->R[3 * k + r] * (double)c->t[k];
    C[r] = v;
  }
}

static real dot3(const real a[3], const real b[3]) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

int orc_network_inputs(const orc_camera *src, int K, const orc_camera *tgt, const float *tsdf_depth,
                       const float *rgb, const float *depth, const float *alpha, real *out) {
  const int W = tgt->width, H = tgt->height;
  const size_t n = (size_t)W * H;
  if (K < 1 || K > 16) return -1;
  double Ct[3], Ck[16][3];
  cam_centre_d(tgt, Ct);
  for (int k = 0; k < K; ++k) cam_centre_d(&src[k], Ck[k]);
  /* M = R_t^T K_t^-1 (FP64, then FP32 once) */
  double Ki[9] = {1.0 / (double)tgt->fx, 0, -(double)tgt->cx / (double)tgt->fx,
                  0, 1.0 / (double)tgt->fy, -(double)tgt->cy / (double)tgt->fy, 0, 0, 1};
  real M[9], C[3], Cs[16][3], dist[16], axd[16];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) {
      double v = 0;
      for (int k = 0; k < 3; ++k) v += (double)tgt->R[3 * k + r] * Ki[3 * k + c];
      M[3 * r + c] = (real)v;
    }
    C[r] = (real)Ct[r];
  }
  for (int k = 0; k < K; ++k) {
    double d2 = 0, ax = 0;
    for (int r = 0; r < 3; ++r) {
      Cs[k][r] = (real)Ck[k][r];
      d2 += (Ck[k][r] - Ct[r]) * (Ck[k][r] - Ct[r]);
      ax += (double)src[k].R[6 + r] * (double)tgt->R[6 + r];
    }
    dist[k] = (real)sqrt(d2);
    axd[k] = (real)ax;
  }
  /* copies of the rendered planes and the TSDF depth */
  for (size_t i = 0; i < 3 * (size_t)K * n; ++i) out[i] = (real)rgb[i];
  for (size_t i = 0; i < (size_t)K * n; ++i) {
    out[3 * K * n + i] = (real)depth[i];
    out[4 * K * n + i] = (real)alpha[i];
  }
  for (size_t i = 0; i < n; ++i) out[5 * K * n + i] = (real)tsdf_depth[i];
#pragma omp parallel for schedule(static)
  for (int j = 0; j < H; ++j)
    for (int i = 0; i < W; ++i) {
      const size_t p = (size_t)j * W + i;
      real a[3], X[3], nrm[3] = {0, 0, 0};
      ray_of(M, (real)i + (real)0.5, (real)j + (real)0.5, a);
      const real D = (real)tsdf_depth[p];
      const int ok = D > 0;
      int has_n = 0;
      if (ok) {
        point_at(a, C, D, X);
        real P[4][3];
        int v[4];
        const int ni[4] = {i - 1, i + 1, i, i}, nj[4] = {j, j, j - 1, j + 1};
        for (int e = 0; e < 4; ++e) {
          v[e] = ni[e] >= 0 && ni[e] < W && nj[e] >= 0 && nj[e] < H &&
                 tsdf_depth[(size_t)nj[e] * W + ni[e]] > 0;
          if (v[e]) {
            real b[3];
            ray_of(M, (real)ni[e] + (real)0.5, (real)nj[e] + (real)0.5, b);
            point_at(b, C, (real)tsdf_depth[(size_t)nj[e] * W + ni[e]], P[e]);
          }
        }
        real tx[3], ty[3];
        int hx = 1, hy = 1;
        for (int r = 0; r < 3; ++r) {
          tx[r] = v[0] && v[1] ? P[1][r] - P[0][r] : v[1] ? P[1][r] - X[r] : v[0] ? X[r] - P[0][r] : 0;
          ty[r] = v[2] && v[3] ? P[3][r] - P[2][r] : v[3] ? P[3][r] - X[r] : v[2] ? X[r] - P[2][r] : 0;
        }
        if (!(v[0] || v[1])) hx = 0;
        if (!(v[2] || v[3])) hy = 0;
        if (hx && hy) {
          real c3[3] = {tx[1] * ty[2] - tx[2] * ty[1], tx[2] * ty[0] - tx[0] * ty[2],
                        tx[0] * ty[1] - tx[1] * ty[0]};
          const real len = RSQRT(dot3(c3, c3));
          if (len > 0) {
            for (int r = 0; r < 3; ++r) nrm[r] = c3[r] / len;
            const real tc[3] = {C[0] - X[0], C[1] - X[1], C[2] - X[2]};
            if (dot3(nrm, tc) < 0)
              for (int r = 0; r < 3; ++r) nrm[r] = -nrm[r];
            has_n = 1;
          }
        }
      }
      const real alen = RSQRT(dot3(a, a));
      const real dt[3] = {a[0] / alen, a[1] / alen, a[2] / alen};
      for (int k = 0; k < K; ++k) {
        real dn = 0, dd = 0;
        if (ok) {
          real r3[3] = {X[0] - Cs[k][0], X[1] - Cs[k][1], X[2] - Cs[k][2]};
          const real rl = RSQRT(dot3(r3, r3));
          if (rl > 0) {
            for (int r = 0; r < 3; ++r) r3[r] = r3[r] / rl;
            if (has_n) dn = dot3(r3, nrm);
            dd = dot3(r3, dt);
          }
        }
        out[(5 * (size_t)K + 1 + k) * n + p] = dn;
        out[(6 * (size_t)K + 1 + k) * n + p] = dd;
        out[(7 * (size_t)K + 1 + k) * n + p] = dist[k];
        out[(8 * (size_t)K + 1 + k) * n + p] = axd[k];
      }
    }
  return 0;
}

/* ------------------------------------------------------------------------
 * The blend of Eq. 4-5 for given weights: I_FG = sum_k I_k alpha_k w_k /
 * sum_k alpha_k w_k (reading of the printed fraction: the denominator sums
 * over the views; I_FG = 0 where it is 0), I = (1 - w_BG) I_FG + w_BG I_BG;
 * the depths D_k blend with the same weights (the blended depth of Eq. 6).
 * Order: aw = alpha_k w_k; num = fma(I_k, aw, num), den = den + aw over k
 * in order; I = fma(w_BG, I_BG, (1 - w_BG) I_FG).
 * rgb K x 3 x H x W, depth / alpha / w K x H x W, w_bg H x W, rgb_bg
 * 3 x H x W; out_rgb 3 x H x W, out_depth H x W.
 * ---------------------------------------------------------------------- */
void orc_blend(int K, int W, int H, const float *rgb, const float *depth, const float *alpha,
               const float *w, const float *w_bg, const float *rgb_bg, real *out_rgb,
               real *out_depth) {
  const size_t n = (size_t)W * H;
  for (size_t p = 0; p < n; ++p) {
    real num[4] = {0, 0, 0, 0}, den = 0;
    for (int k = 0; k < K; ++k) {
      const real aw = (real)alpha[k * n + p] * (real)w[k * n + p];
      for (int c = 0; c < 3; ++c) num[c] = RFMA((real)rgb[(3 * k + c) * n + p], aw, num[c]);
      num[3] = RFMA((real)depth[k * n + p], aw, num[3]);
      den = den + aw;
    }
    const real wb = (real)w_bg[p];
    for (int c = 0; c < 3; ++c) {
      const real fg = den > 0 ? num[c] / den : (real)0;
      out_rgb[c * n + p] = RFMA(wb, (real)rgb_bg[c * n + p], ((real)1 - wb) * fg);
    }
    out_depth[p] = den > 0 ? num[3] / den : (real)0;
  }
}

/* ------------------------------------------------------------------------
 * Surface extraction (Suppl. A.1: the surface is where s changes sign along
 * the ray).  Reading: on the dense bins, the first d in [0, D-2] with
 * W_d > 0, W_{d+1} > 0, F_d > 0 and F_{d+1} <= 0; the depth is the linear
 * interpolation z_d + (z_{d+1} - z_d) F_d / (F_d - F_{d+1}).  No crossing:
 * depth 0, bin -1.
 * ---------------------------------------------------------------------- */
void orc_extract(const orc_tsdf_params *p, const real *F, const real *W, int npix, real *depth,
                 int32_t *bin) {
  const int D = p->num_bins;
  real *zb = (real *)malloc(sizeof(real) * D), *tb = (real *)malloc(sizeof(real) * D);
  orc_bins(p, zb, tb);
#pragma omp parallel for schedule(static)
  for (int n = 0; n < npix; ++n) {
    const real *f = F + (size_t)n * D, *w = W + (size_t)n * D;
    depth[n] = 0;
    bin[n] = -1;
    for (int d = 0; d + 1 < D; ++d)
      if (w[d] > 0 && w[d + 1] > 0 && f[d] > 0 && f[d + 1] <= 0) {
        const real frac = f[d] / (f[d] - f[d + 1]);
        depth[n] = zb[d] + (zb[d + 1] - zb[d]) * frac;
        bin[n] = d;
        break;
      }
  }
  free(zb);
  free(tb);
}

/* ------------------------------------------------------------------------
 * Forward rendering of one view's per-pixel Gaussians into the target
 * (§3.1, Suppl. A.3), as a z-buffered splat.
 *
 * Each valid source pixel q = (i, j) of view k carries an isotropic, opaque
 * Gaussian at its back-projected point with the pixel's colour, scaled so its
 * source-image footprint is one pixel (reading: std sigma_px = 0.5 source
 * px).  Moved to the target: X = D h + c, dropped unless z_T > z_min;
 * (x, y) = (x_T, y_T) / z_T; target std sigma = s_k (D / z_T) with
 * s_k = sigma_px f_T / f_k; coverage radius^2 R2 = min(2 sigma^2, r_max^2)
 * (reading: the G >= e^-1 disc, so an identity warp covers only its own
 * pixel).  Target pixel p is covered iff d2 = |centre(p) - (x, y)|^2 <= R2.
 * Winner(p) = the covering splat with the smallest (z_T, q) (z-buffer, ties to
 * the smaller source index).  Band S(p) = covering splats with
 * z_T <= z_win (1 + band_rel); with G = exp(-d2 / (2 sigma^2)) and
 * c = u8 / 255: colour = sum G c / sum G, accumulated opacity
 * alpha = 1 - prod (1 - G) (reading: an order-free stand-in for front-to-back
 * compositing of the front surface), depth = z_win, index = q_win.
 * Sums and products run over ascending q.  Empty pixels: -1, 0, 0, 0.
 * tape (nullable, 3 planes per view): sum G, sum over G < 1 of log(1 - G),
 * and the count of G == 1.
 * ---------------------------------------------------------------------- */
typedef struct {
  int ok;
  real x, y, z, s2, R2;
  int a0, a1, b0, b1;
} orc_splat_geom;

static void splat_geom(const real H[9], const real c[3], real sscale, real rmax2,
                       const orc_splat_params *sp, int i, int j, float D, int Wt, int Ht,
                       orc_splat_geom *g) {
  g->ok = 0;
  if (!depth_ok(D)) return;
  real h[3], X[3];
  ray_of(H, (real)i + (real)0.5, (real)j + (real)0.5, h);
  point_at(h, c, (real)D, X);
  if (!(X[2] > (real)sp->z_min)) return;
  const real inv = (real)1 / X[2];
  g->x = X[0] * inv;
  g->y = X[1] * inv;
  g->z = X[2];
  const real sig = sscale * ((real)D * inv);
  g->s2 = sig * sig;
  g->R2 = RMIN((real)2 * g->s2, rmax2);
  /* candidate window: a superset of the covered pixel centres */
  const double r = sqrt((double)g->R2);
  double a0 = floor((double)g->x - 0.5 - r) - 1, a1 = floor((double)g->x - 0.5 + r) + 1;
  double b0 = floor((double)g->y - 0.5 - r) - 1, b1 = floor((double)g->y - 0.5 + r) + 1;
  if (a0 < 0) a0 = 0;
  if (b0 < 0) b0 = 0;
  if (a1 > Wt - 1) a1 = Wt - 1;
  if (b1 > Ht - 1) b1 = Ht - 1;
  if (a0 > a1 || b0 > b1) return;
  g->a0 = (int)a0;
  g->a1 = (int)a1;
  g->b0 = (int)b0;
  g->b1 = (int)b1;
  g->ok = 1;
}

static real cover_d2(const orc_splat_geom *g, int a, int b) {
  const real dx = ((real)a + (real)0.5) - g->x;
  const real dy = ((real)b + (real)0.5) - g->y;
  return RFMA(dx, dx, dy * dy);
}

static uint32_t f32_bits(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  return u;
}

/* mask (nullable, K x Hs x Ws): a per-source-pixel scalar blended over the
 * band like one colour channel, sum G m / sum G, into out_mask (nullable,
 * K x Ht x Wt; 0 where no splat covers); out_mask_max (nullable, Ht x Wt)
 * is its maximum over the K views (Suppl. A.2: the channel-wise maximum of
 * the splatted difference masks; reading: 0 where no view covers). */
int orc_splat_masked(const orc_camera *src, int K, const float *depth, const uint8_t *rgb,
                     const orc_camera *tgt, const orc_splat_params *sp, int32_t *win_idx,
                     real *out_depth, real *out_rgb, real *out_alpha, real *tape,
                     const float *mask, real *out_mask, real *out_mask_max) {
  const int Ws = src[0].width, Hs = src[0].height, Wt = tgt->width, Ht = tgt->height;
  const size_t ns = (size_t)Ws * Hs, nt = (size_t)Wt * Ht;
  const real rmax2 = (real)sp->r_max_px * (real)sp->r_max_px;
  const real band = (real)1 + (real)sp->band_rel;
  uint64_t *zbuf = (uint64_t *)malloc(sizeof(uint64_t) * nt);
  real *nrm = (real *)malloc(sizeof(real) * nt), *prod = (real *)malloc(sizeof(real) * nt);
  real *lsum = (real *)malloc(sizeof(real) * nt), *ones = (real *)malloc(sizeof(real) * nt);
  real *zwin = (real *)malloc(sizeof(real) * nt);
  real *msum = (real *)malloc(sizeof(real) * nt);
  if (!zbuf || !nrm || !prod || !lsum || !ones || !zwin || !msum) return -2;
  if (out_mask_max)
    for (size_t p = 0; p < nt; ++p) out_mask_max[p] = 0;
  for (int k = 0; k < K; ++k) {
    real H[9], c[3];
    relproj(&src[k], tgt, H, c);
    const real sscale = (real)((double)sp->sigma_px * (double)tgt->fx / (double)src[k].fx);
    const float *dk = depth + ns * k;
    const uint8_t *ck = rgb + ns * 3 * k;
    real *prgb = out_rgb + nt * 3 * k;
    for (size_t p = 0; p < nt; ++p) {
      zbuf[p] = UINT64_MAX;
      nrm[p] = 0;
      prod[p] = 1;
      lsum[p] = 0;
      ones[p] = 0;
      msum[p] = 0;
      prgb[p] = prgb[nt + p] = prgb[2 * nt + p] = 0;
    }
    /* pass 1: z-test */
    for (int j = 0; j < Hs; ++j)
      for (int i = 0; i < Ws; ++i) {
        orc_splat_geom g;
        splat_geom(H, c, sscale, rmax2, sp, i, j, dk[(size_t)j * Ws + i], Wt, Ht, &g);
        if (!g.ok) continue;
        const uint64_t key = ((uint64_t)f32_bits((float)g.z) << 32) | (uint32_t)(j * Ws + i);
        for (int b = g.b0; b <= g.b1; ++b)
          for (int a = g.a0; a <= g.a1; ++a)
            if (cover_d2(&g, a, b) <= g.R2) {
              uint64_t *zp = &zbuf[(size_t)b * Wt + a];
              if (key < *zp) *zp = key;
            }
      }
    /* the winner's depth in the working precision (the key holds its FP32
     * rounding, which orders the z-test) */
    for (size_t p = 0; p < nt; ++p) {
      zwin[p] = 0;
      if (zbuf[p] == UINT64_MAX) continue;
      const uint32_t qw = (uint32_t)(zbuf[p] & 0xffffffffu);
      orc_splat_geom g;
      splat_geom(H, c, sscale, rmax2, sp, (int)(qw % (uint32_t)Ws), (int)(qw / (uint32_t)Ws),
                 dk[qw], Wt, Ht, &g);
      zwin[p] = g.z;
    }
    /* pass 2: band blend in ascending q */
    for (int j = 0; j < Hs; ++j)
      for (int i = 0; i < Ws; ++i) {
        orc_splat_geom g;
        const size_t q = (size_t)j * Ws + i;
        splat_geom(H, c, sscale, rmax2, sp, i, j, dk[q], Wt, Ht, &g);
        if (!g.ok) continue;
        for (int b = g.b0; b <= g.b1; ++b)
          for (int a = g.a0; a <= g.a1; ++a) {
            const real d2 = cover_d2(&g, a, b);
            if (!(d2 <= g.R2)) continue;
            const size_t p = (size_t)b * Wt + a;
            if (!(g.z <= zwin[p] * band)) continue;
            const real G = REXP(((real)-0.5 * d2) / g.s2);
            nrm[p] = nrm[p] + G;
            for (int ch = 0; ch < 3; ++ch)
              prgb[ch * nt + p] = prgb[ch * nt + p] + G * ((real)ck[q * 3 + ch] / (real)255);
            if (mask) msum[p] = msum[p] + G * (real)mask[ns * k + q];
            prod[p] = prod[p] * ((real)1 - G);
            if (G < (real)1)
              lsum[p] = lsum[p] + RLOG((real)1 - G);
            else
              ones[p] = ones[p] + 1;
          }
      }
    for (size_t p = 0; p < nt; ++p) {
      const size_t o = nt * k + p;
      if (zbuf[p] == UINT64_MAX) {
        win_idx[o] = -1;
        out_depth[o] = 0;
        out_alpha[o] = 0;
      } else {
        win_idx[o] = (int32_t)(uint32_t)(zbuf[p] & 0xffffffffu);
        out_depth[o] = zwin[p];
        for (int ch = 0; ch < 3; ++ch) prgb[ch * nt + p] = prgb[ch * nt + p] / nrm[p];
        out_alpha[o] = (real)1 - prod[p];
      }
      if (mask) {
        const real m = zbuf[p] == UINT64_MAX ? (real)0 : msum[p] / nrm[p];
        if (out_mask) out_mask[o] = m;
        if (out_mask_max && m > out_mask_max[p]) out_mask_max[p] = m;
      }
      if (tape) {
        tape[nt * 3 * k + p] = nrm[p];
        tape[nt * 3 * k + nt + p] = lsum[p];
        tape[nt * 3 * k + 2 * nt + p] = ones[p];
      }
    }
  }
  free(zbuf);
  free(nrm);
  free(prod);
  free(lsum);
  free(ones);
  free(zwin);
  free(msum);
  return 0;
}

int orc_splat(const orc_camera *src, int K, const float *depth, const uint8_t *rgb,
              const orc_camera *tgt, const orc_splat_params *sp, int32_t *win_idx,
              real *out_depth, real *out_rgb, real *out_alpha, real *tape) {
  return orc_splat_masked(src, K, depth, rgb, tgt, sp, win_idx, out_depth, out_rgb, out_alpha,
                          tape, NULL, NULL, NULL);
}

/* ------------------------------------------------------------------------
 * exp(x) in FP32 by Cody and Waite's argument reduction (1980) with a
 * degree-6 Taylor polynomial: n = rint(x log2 e), r = x - n ln2 with ln2
 * split into a 16-bit head and a tail (two fused multiply-adds), e^r by
 * Horner's rule with fused multiply-adds, scaled by 2^n.  0 below x = -86
 * (no subnormal results).  For x <= 0, within 3 ulp of e^x.  Every step is
 * an explicitly rounded FP32 operation, so the function is reproducible
 * bit for bit wherever it is implemented in this order.
 * ---------------------------------------------------------------------- */
float orc_exp_cw(float x) {
  if (!(x >= -86.0f)) return 0.0f;
  const float n = rintf(x * 1.44269504f);
  float r = fmaf(-n, 0.693145752f, x);
  r = fmaf(-n, 1.42860677e-6f, r);
  float p = 1.0f / 720.0f;
  p = fmaf(p, r, 1.0f / 120.0f);
  p = fmaf(p, r, 1.0f / 24.0f);
  p = fmaf(p, r, 1.0f / 6.0f);
  p = fmaf(p, r, 0.5f);
  p = fmaf(p, r, 1.0f);
  p = fmaf(p, r, 1.0f);
  return ldexpf(p, (int)n);
}

/* Threads of the OpenMP loops (for timing the oracle on n cores). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}

void orc_exp_cw_n(const float *x, float *y, size_t n) {
  for (size_t i = 0; i < n; ++i) y[i] = orc_exp_cw(x[i]);
}

/* ------------------------------------------------------------------------
 * EWA pixel Gaussians composited front to back (§3.1: the paper renders the
 * per-pixel Gaussians with the 3D Gaussian splatting rasteriser).  The
 * Gaussians are those of orc_splat: isotropic in 3D, centred on the
 * back-projected pixel, fully opaque, coloured u8 / 255, with standard
 * deviation sigma_px D / f_k so that their footprint in the source image is
 * one pixel.  Here they are projected with the local affine (EWA)
 * approximation of the perspective map instead of an isotropic disc.
 *
 * Readings (the paper names the renderer, not its constants):
 *   - image covariance of the Gaussian with target mean (u, v) = (x, y) / z:
 *     with a = (u - cx) / fx, b = (v - cy) / fy and sig = sscale (D / z)
 *     (sscale = sigma_px fx_T / f_k, as in orc_splat),
 *       S = sig^2 [[1 + a^2, r a b], [r a b, r^2 (1 + b^2)]] + lowpass I,
 *     r = fy / fx: J J^T of the perspective Jacobian times the isotropic 3D
 *     covariance, plus the renderer's 0.3 px^2 screen-space low-pass;
 *   - opacity at a pixel centre: alpha = min(0.99, G), G = exp(power),
 *     power = -d^T S^-1 d / 2, d = pixel centre - (u, v); terms with
 *     power > 0 or alpha < 1/255 are skipped;
 *   - footprints are clipped to |dx| <= r_max, |dy| <= r_max (r_max_px of
 *     the splat parameters), which bounds the tiles a Gaussian can touch;
 *   - per target pixel the terms are taken in ascending (z, source index)
 *     order (z is the FP32 target depth of the mean); compositing stops
 *     before the first term that would bring the transmittance below 1e-4;
 *   - outputs per view: colour sum c alpha T, opacity 1 - T, and depth
 *     sum z alpha T / (1 - T) (0 where no term was taken).
 * Splats with z <= z_min are dropped, as in orc_splat.
 *
 * Operation order (FP32 build): inv = 1 / z, u = x inv, v = y inv,
 * sig = sscale (D inv), s2 = sig sig,
 * sxx = s2 (1 + a a) + lowpass, syy = s2 (r2 (1 + b b)) + lowpass,
 * sxy = s2 (r (a b)) with r, r2 = (fy / fx)^2 rounded once from FP64;
 * det = sxx syy - sxy sxy; Ah = (-0.5 syy) / det, Bn = sxy / det,
 * Ch = (-0.5 sxx) / det; power = fma(Bn, dx dy, fma(Ah, dx dx, Ch (dy dy)));
 * G = orc_exp_cw(power); w = alpha T; colour = fma(c, w, colour);
 * depth sum = fma(z, w, sum); T = T (1 - alpha) (the product computed for
 * the stopping test).
 * out_rgb K x 3 x Ht x Wt, out_alpha and out_depth K x Ht x Wt; with
 * pixel_mask (Ht x Wt, nullable) only the pixels it marks are rendered (the
 * others read as nothing drawn).
 * ---------------------------------------------------------------------- */
typedef struct {
  uint64_t key;
  real u, v, Ah, Bn, Ch, z, c[3];
} orc_ewa_entry;

static int ewa_cmp(const void *x, const void *y) {
  const uint64_t a = ((const orc_ewa_entry *)x)->key, b = ((const orc_ewa_entry *)y)->key;
  return a < b ? -1 : (a > b ? 1 : 0);
}

int orc_splat_ewa(const orc_camera *src, int K, const float *depth, const uint8_t *rgb,
                  const orc_camera *tgt, const orc_splat_params *sp, float lowpass,
                  const uint8_t *pixel_mask, real *out_rgb, real *out_alpha, real *out_depth) {
  const int Ws = src[0].width, Hs = src[0].height, Wt = tgt->width, Ht = tgt->height;
  const size_t ns = (size_t)Ws * Hs, nt = (size_t)Wt * Ht;
  const real fx = (real)tgt->fx, fy = (real)tgt->fy, cx = (real)tgt->cx, cy = (real)tgt->cy;
  const double rd = (double)tgt->fy / (double)tgt->fx;
  const real ry = (real)rd, ry2 = (real)(rd * rd), lp = (real)lowpass;
  const real rmax = (real)sp->r_max_px;
  const real amin = (real)1 / (real)255;
  size_t *cnt = (size_t *)malloc(sizeof(size_t) * (nt + 1));
  if (!cnt) return -2;
  for (int k = 0; k < K; ++k) {
    real H[9], c[3];
    relproj(&src[k], tgt, H, c);
    const real sscale = (real)((double)sp->sigma_px * (double)tgt->fx / (double)src[k].fx);
    const float *dk = depth + ns * k;
    const uint8_t *ck = rgb + ns * 3 * k;
    orc_ewa_entry *g = (orc_ewa_entry *)malloc(sizeof(orc_ewa_entry) * (ns ? ns : 1));
    int *box = (int *)malloc(sizeof(int) * (ns ? ns : 1) * 4);
    if (!g || !box) return -2;
    /* the Gaussians of view k */
    for (size_t q = 0; q < ns; ++q) {
      g[q].key = UINT64_MAX;
      const float D = dk[q];
      if (!depth_ok(D)) continue;
      real h[3], X[3];
      ray_of(H, (real)(int)(q % Ws) + (real)0.5, (real)(int)(q / Ws) + (real)0.5, h);
      point_at(h, c, (real)D, X);
      if (!(X[2] > (real)sp->z_min)) continue;
      const real inv = (real)1 / X[2];
      const real u = X[0] * inv, v = X[1] * inv;
      const real a = (u - cx) / fx, b = (v - cy) / fy;
      const real sig = sscale * ((real)D * inv), s2 = sig * sig;
      const real sxx = s2 * ((real)1 + a * a) + lp;
      const real syy = s2 * (ry2 * ((real)1 + b * b)) + lp;
      const real sxy = s2 * (ry * (a * b));
      const real det = sxx * syy - sxy * sxy;
      g[q].Ah = ((real)-0.5 * syy) / det;
      g[q].Bn = sxy / det;
      g[q].Ch = ((real)-0.5 * sxx) / det;
      g[q].u = u;
      g[q].v = v;
      g[q].z = X[2];
      for (int ch = 0; ch < 3; ++ch) g[q].c[ch] = (real)ck[q * 3 + ch] / (real)255;
      g[q].key = ((uint64_t)f32_bits((float)X[2]) << 32) | (uint32_t)q;
      /* a box holding every pixel that can take a term: alpha >= 1/255
       * needs d^T S^-1 d <= 2 ln 255 < 12, which bounds |dx| by
       * sqrt(12 sxx) and |dy| by sqrt(12 syy); the clip bounds both by
       * r_max; one pixel of margin for the rounding of the bounds */
      const double ud = (double)u, vd = (double)v;
      const double rx = fmin(sqrt(12.0 * (double)sxx), (double)rmax) + 1;
      const double rv = fmin(sqrt(12.0 * (double)syy), (double)rmax) + 1;
      int x0 = (int)fmax(floor(ud - 0.5 - rx), -1.0), x1 = (int)fmin(ceil(ud - 0.5 + rx), 1e9);
      int y0 = (int)fmax(floor(vd - 0.5 - rv), -1.0), y1 = (int)fmin(ceil(vd - 0.5 + rv), 1e9);
      box[4 * q] = x0 < 0 ? 0 : x0;
      box[4 * q + 1] = x1 > Wt - 1 ? Wt - 1 : x1;
      box[4 * q + 2] = y0 < 0 ? 0 : y0;
      box[4 * q + 3] = y1 > Ht - 1 ? Ht - 1 : y1;
    }
    /* per-pixel candidate lists (counting sort by pixel) */
    for (size_t p = 0; p <= nt; ++p) cnt[p] = 0;
    for (size_t q = 0; q < ns; ++q) {
      if (g[q].key == UINT64_MAX) continue;
      for (int y = box[4 * q + 2]; y <= box[4 * q + 3]; ++y)
        for (int x = box[4 * q]; x <= box[4 * q + 1]; ++x)
          if (!pixel_mask || pixel_mask[(size_t)y * Wt + x]) cnt[(size_t)y * Wt + x + 1]++;
    }
    for (size_t p = 0; p < nt; ++p) cnt[p + 1] += cnt[p];
    uint32_t *lst = (uint32_t *)malloc(sizeof(uint32_t) * (cnt[nt] ? cnt[nt] : 1));
    size_t *cur = (size_t *)malloc(sizeof(size_t) * (nt ? nt : 1));
    if (!lst || !cur) return -2;
    memcpy(cur, cnt, sizeof(size_t) * nt);
    for (size_t q = 0; q < ns; ++q) {
      if (g[q].key == UINT64_MAX) continue;
      for (int y = box[4 * q + 2]; y <= box[4 * q + 3]; ++y)
        for (int x = box[4 * q]; x <= box[4 * q + 1]; ++x)
          if (!pixel_mask || pixel_mask[(size_t)y * Wt + x])
            lst[cur[(size_t)y * Wt + x]++] = (uint32_t)q;
    }
    int oom = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (size_t p = 0; p < nt; ++p) {
      const size_t m = cnt[p + 1] - cnt[p];
      orc_ewa_entry *e = (orc_ewa_entry *)malloc(sizeof(orc_ewa_entry) * (m ? m : 1));
      if (!e) {
        oom = 1;
        continue;
      }
      for (size_t t = 0; t < m; ++t) e[t] = g[lst[cnt[p] + t]];
      qsort(e, m, sizeof(orc_ewa_entry), ewa_cmp);
      const real px = (real)(int)(p % Wt) + (real)0.5, py = (real)(int)(p / Wt) + (real)0.5;
      real T = 1, col[3] = {0, 0, 0}, zs = 0;
      for (size_t t = 0; t < m; ++t) {
        const real dx = px - e[t].u, dy = py - e[t].v;
        if (!(RABS(dx) <= rmax && RABS(dy) <= rmax)) continue;
        const real power = RFMA(e[t].Bn, dx * dy, RFMA(e[t].Ah, dx * dx, e[t].Ch * (dy * dy)));
        if (power > 0) continue;
#ifdef ORC_DOUBLE
        const real G = exp(power);
#else
        const real G = orc_exp_cw(power);
#endif
        const real al = RMIN((real)0.99, G);
        if (al < amin) continue;
        const real tt = T * ((real)1 - al);
        if (tt < (real)1e-4) break;
        const real w = al * T;
        for (int ch = 0; ch < 3; ++ch) col[ch] = RFMA(e[t].c[ch], w, col[ch]);
        zs = RFMA(e[t].z, w, zs);
        T = tt;
      }
      for (int ch = 0; ch < 3; ++ch) out_rgb[(3 * (size_t)k + ch) * nt + p] = col[ch];
      out_alpha[(size_t)k * nt + p] = (real)1 - T;
      out_depth[(size_t)k * nt + p] = T < 1 ? zs / ((real)1 - T) : (real)0;
      free(e);
    }
    free(lst);
    free(cur);
    free(g);
    free(box);
    if (oom) {
      free(cnt);
      return -2;
    }
  }
  free(cnt);
  return 0;
}

/* ------------------------------------------------------------------------
 * Soft difference mask of one view between consecutive frames (Eq. 1, §3.2):
 * M = min(|I^t - I^{t-1}| / lambda_t + beta, 1), computed at quarter
 * resolution, max-pooled over 3 x 3 and upsampled bilinearly to full size.
 *
 * Readings: "quarter resolution" is a factor x factor box (factor = 4)
 * mean of the colours c = u8 / 255, the box clipped at the image border
 * (Wq = ceil(W / factor)); |I^t - I^{t-1}| of an RGB image is the mean over
 * its three channels of the absolute difference; the max-pool window is
 * clipped at the border; upsampling samples the low-resolution image at the
 * full-resolution pixel centre, x = (i + 1/2) / factor - 1/2, clamped to
 * [0, Wq - 1] (likewise y).
 * Operation order: per box the channel sums of u8 are exact integers, so
 * dI = (sum over channels of |S^t - S^{t-1}|) / (765 n) is one rounding
 * (n pixels in the box); then t = dI / lambda_t, M = min(t + beta, 1).
 * Bilinear: x0 = floor(x), x1 = min(x0 + 1, Wq - 1), fx = x - x0;
 * top = m00 + fx (m10 - m00), bottom = m01 + fx (m11 - m01),
 * M = top + fy (bottom - top), no fused multiply-adds.
 * rgb, rgb_prev: H x W x 3 u8.  mask: H x W.
 * ---------------------------------------------------------------------- */
int orc_difference_mask(const uint8_t *rgb, const uint8_t *rgb_prev, int W, int H, int factor,
                        float beta, float lambda_t, real *mask) {
  const int Wq = (W + factor - 1) / factor, Hq = (H + factor - 1) / factor;
  real *low = (real *)malloc(sizeof(real) * Wq * Hq);
  real *pool = (real *)malloc(sizeof(real) * Wq * Hq);
  if (!low || !pool) return -2;
  for (int b = 0; b < Hq; ++b)
    for (int a = 0; a < Wq; ++a) {
      long st[3] = {0, 0, 0}, sp[3] = {0, 0, 0};
      int n = 0;
      for (int j = b * factor; j < (b + 1) * factor && j < H; ++j)
        for (int i = a * factor; i < (a + 1) * factor && i < W; ++i) {
          for (int ch = 0; ch < 3; ++ch) {
            st[ch] += rgb[((size_t)j * W + i) * 3 + ch];
            sp[ch] += rgb_prev[((size_t)j * W + i) * 3 + ch];
          }
          ++n;
        }
      const long d = labs(st[0] - sp[0]) + labs(st[1] - sp[1]) + labs(st[2] - sp[2]);
      const real dI = (real)d / (real)(765 * n);
      const real t = dI / (real)lambda_t;
      low[(size_t)b * Wq + a] = RMIN(t + (real)beta, (real)1);
    }
  for (int b = 0; b < Hq; ++b)
    for (int a = 0; a < Wq; ++a) {
      real m = low[(size_t)b * Wq + a];
      for (int bb = b - 1; bb <= b + 1; ++bb)
        for (int aa = a - 1; aa <= a + 1; ++aa)
          if (aa >= 0 && aa < Wq && bb >= 0 && bb < Hq && low[(size_t)bb * Wq + aa] > m)
            m = low[(size_t)bb * Wq + aa];
      pool[(size_t)b * Wq + a] = m;
    }
  for (int j = 0; j < H; ++j)
    for (int i = 0; i < W; ++i) {
      real x = ((real)i + (real)0.5) / (real)factor - (real)0.5;
      real y = ((real)j + (real)0.5) / (real)factor - (real)0.5;
      if (x < 0) x = 0;
      if (y < 0) y = 0;
      if (x > (real)(Wq - 1)) x = (real)(Wq - 1);
      if (y > (real)(Hq - 1)) y = (real)(Hq - 1);
      const int x0 = (int)floor((double)x), y0 = (int)floor((double)y);
      const int x1 = x0 + 1 < Wq ? x0 + 1 : Wq - 1, y1 = y0 + 1 < Hq ? y0 + 1 : Hq - 1;
      const real fx = x - (real)x0, fy = y - (real)y0;
      const real m00 = pool[(size_t)y0 * Wq + x0], m10 = pool[(size_t)y0 * Wq + x1];
      const real m01 = pool[(size_t)y1 * Wq + x0], m11 = pool[(size_t)y1 * Wq + x1];
      const real top = m00 + fx * (m10 - m00);
      const real bot = m01 + fx * (m11 - m01);
      mask[(size_t)j * W + i] = top + fy * (bot - top);
    }
  free(low);
  free(pool);
  return 0;
}

/* ------------------------------------------------------------------------
 * Temporally filtered depth (Eq. 2, §3.2): Dd^t = M D^t + (1 - M) Dd^{t-1},
 * evaluated as fma(M, D^t, (1 - M) Dd^{t-1}).  Readings: a hole in D^t
 * stays a hole (0, so the fusion drops it); where there is no usable
 * previous filtered depth (first frame: prev NULL, or a hole) Dd^t = D^t.
 * ---------------------------------------------------------------------- */
void orc_temporal_filter(const float *depth, const real *mask, const real *prev, size_t n,
                         real *out) {
  for (size_t p = 0; p < n; ++p) {
    const float D = depth[p];
    if (!depth_ok(D)) {
      out[p] = 0;
    } else if (!prev || !(prev[p] > 0 && prev[p] < INFINITY)) {
      out[p] = (real)D;
    } else {
      const real a = (real)1 - mask[p];
      out[p] = RFMA(mask[p], (real)D, a * prev[p]);
    }
  }
}

/* ------------------------------------------------------------------------
 * Adjoint of the splat with respect to source depth and colour.
 *
 * L = <g_rgb, rgb> + <g_depth, depth> + <g_alpha, alpha>.  Discrete choices
 * (coverage, band, winner) are held fixed.  With G = exp(-d2 / (2 s2)):
 *   d rgb_c / d c_q = G_q / n,  d rgb_c / d G_q = (c_q - rgb_c) / n,
 *   d alpha / d G_q = prod over the other band members of (1 - G_j),
 *   d depth / d D_q = h_2 (dz_T/dD) for the winner.
 * G depends on D through x, y (X = D h + c) and sigma = s_k D / z_T:
 *   dx/dD = (h0 z_T - X0 h2) / z_T^2, likewise y; dsigma/dD = s_k c2 / z_T^2
 *   dG/dD = G * ( (dx * dx/dD + dy * dy/dD) / s2 + d2 (dsigma/dD) / (sigma s2) )
 * with dx = centre - x.  Gradients are overwritten, not accumulated.
 * The forward outputs (winners, depth, rgb) are recomputed here.
 * Error-bound outputs (optional, for the tests' tolerance): m_depth_in and
 * m_rgb_in are the same sums over the terms' magnitudes (factors replaced
 * by their magnitudes, differences of computed values by the sums of their
 * magnitudes), cnt_in the number of terms of each depth gradient.
 * ---------------------------------------------------------------------- */
int orc_splat_backward_mag(const orc_camera *src, int K, const float *depth,
                           const uint8_t *rgb, const orc_camera *tgt, const orc_splat_params *sp,
                           const real *g_rgb, const real *g_depth, const real *g_alpha,
                           real *g_depth_in, real *g_rgb_in, real *m_depth_in, real *m_rgb_in,
                           int32_t *cnt_in) {
  const int Ws = src[0].width, Hs = src[0].height, Wt = tgt->width, Ht = tgt->height;
  const size_t ns = (size_t)Ws * Hs, nt = (size_t)Wt * Ht;
  int32_t *win = (int32_t *)malloc(sizeof(int32_t) * nt * K);
  real *od = (real *)malloc(sizeof(real) * nt * K), *orgb = (real *)malloc(sizeof(real) * nt * 3 * K);
  real *oa = (real *)malloc(sizeof(real) * nt * K), *tape = (real *)malloc(sizeof(real) * nt * 3 * K);
  size_t *start = (size_t *)malloc(sizeof(size_t) * (nt + 1)), *fill = (size_t *)malloc(sizeof(size_t) * nt);
  real *band_G = NULL;
  size_t *band_q = NULL;
  if (!win || !od || !orgb || !oa || !tape || !start || !fill) return -2;
  orc_splat(src, K, depth, rgb, tgt, sp, win, od, orgb, oa, tape);
  const real rmax2 = (real)sp->r_max_px * (real)sp->r_max_px;
  const real band = (real)1 + (real)sp->band_rel;
  for (size_t n = 0; n < ns * K; ++n) g_depth_in[n] = 0;
  for (size_t n = 0; n < ns * K * 3; ++n) g_rgb_in[n] = 0;
  if (m_depth_in)
    for (size_t n = 0; n < ns * K; ++n) m_depth_in[n] = 0;
  if (m_rgb_in)
    for (size_t n = 0; n < ns * K * 3; ++n) m_rgb_in[n] = 0;
  if (cnt_in)
    for (size_t n = 0; n < ns * K; ++n) cnt_in[n] = 0;
  for (int k = 0; k < K; ++k) {
    real H[9], c[3];
    relproj(&src[k], tgt, H, c);
    const real sscale = (real)((double)sp->sigma_px * (double)tgt->fx / (double)src[k].fx);
    const float *dk = depth + ns * k;
    const uint8_t *ck = rgb + ns * 3 * k;
    const real *nrm = tape + nt * 3 * k;
    /* band members of every target pixel, in ascending source index */
    for (size_t p = 0; p <= nt; ++p) start[p] = 0;
    for (int pass = 0; pass < 2; ++pass) {
      for (size_t p = 0; p < nt; ++p) fill[p] = 0;
      for (int j = 0; j < Hs; ++j)
        for (int i = 0; i < Ws; ++i) {
          orc_splat_geom g;
          splat_geom(H, c, sscale, rmax2, sp, i, j, dk[(size_t)j * Ws + i], Wt, Ht, &g);
          if (!g.ok) continue;
          for (int b = g.b0; b <= g.b1; ++b)
            for (int a = g.a0; a <= g.a1; ++a) {
              const real d2 = cover_d2(&g, a, b);
              const size_t p = (size_t)b * Wt + a;
              if (!(d2 <= g.R2) || win[nt * k + p] < 0 || !(g.z <= od[nt * k + p] * band)) continue;
              if (pass == 0) {
                start[p + 1]++;
              } else {
                band_G[start[p] + fill[p]] = REXP(((real)-0.5 * d2) / g.s2);
                band_q[start[p] + fill[p]] = (size_t)j * Ws + i;
              }
              fill[p]++;
            }
        }
      if (pass == 0) {
        for (size_t p = 0; p < nt; ++p) start[p + 1] += start[p];
        free(band_G);
        free(band_q);
        band_G = (real *)malloc(sizeof(real) * (start[nt] + 1));
        band_q = (size_t *)malloc(sizeof(size_t) * (start[nt] + 1));
        if (!band_G || !band_q) return -2;
      }
    }
    for (int j = 0; j < Hs; ++j)
      for (int i = 0; i < Ws; ++i) {
        const size_t q = (size_t)j * Ws + i;
        orc_splat_geom g;
        splat_geom(H, c, sscale, rmax2, sp, i, j, dk[q], Wt, Ht, &g);
        if (!g.ok) continue;
        real h[3], X[3];
        ray_of(H, (real)i + (real)0.5, (real)j + (real)0.5, h);
        point_at(h, c, (real)dk[q], X);
        const real Z = X[2], Z2 = Z * Z;
        const real dxdD = (h[0] * Z - X[0] * h[2]) / Z2;
        const real dydD = (h[1] * Z - X[1] * h[2]) / Z2;
        const real sig = sscale * ((real)dk[q] / Z);
        const real dsdD = sscale * c[2] / Z2;
        /* magnitudes of the same factors (differences as sums of magnitudes) */
        const real mxdD = (RABS(h[0]) * Z + RABS(X[0]) * RABS(h[2])) / Z2;
        const real mydD = (RABS(h[1]) * Z + RABS(X[1]) * RABS(h[2])) / Z2;
        real gD = 0, gc[3] = {0, 0, 0}, mD = 0, mc[3] = {0, 0, 0};
        int32_t nD = 0;
        for (int b = g.b0; b <= g.b1; ++b)
          for (int a = g.a0; a <= g.a1; ++a) {
            const real d2 = cover_d2(&g, a, b);
            if (!(d2 <= g.R2)) continue;
            const size_t p = (size_t)b * Wt + a, o = nt * k + p;
            if (win[o] < 0 || !(g.z <= od[o] * band)) continue;
            const real G = REXP(((real)-0.5 * d2) / g.s2);
            const real n = nrm[p];
            real dLdG = 0, mLdG = 0;
            for (int ch = 0; ch < 3; ++ch) {
              const real gr = g_rgb[(nt * 3 * k) + ch * nt + p];
              const real cq = (real)ck[q * 3 + ch] / (real)255;
              const real orc = orgb[nt * 3 * k + ch * nt + p];
              gc[ch] += gr * G / n;
              mc[ch] += RABS(gr) * G / n;
              dLdG += gr * (cq - orc) / n;
              mLdG += RABS(gr) * (cq + RABS(orc)) / n;
            }
            /* product of (1 - G_j) over the other band members, directly */
            real others = 1;
            for (size_t e = start[p]; e < start[p + 1]; ++e)
              if (band_q[e] != q) others = others * ((real)1 - band_G[e]);
            dLdG += g_alpha[o] * others;
            mLdG += RABS(g_alpha[o]) * others;
            const real dx = ((real)a + (real)0.5) - g.x, dy = ((real)b + (real)0.5) - g.y;
            const real dGdD = G * ((dx * dxdD + dy * dydD) / g.s2 + d2 * dsdD / (sig * g.s2));
            const real mGdD = G * ((RABS(dx) * mxdD + RABS(dy) * mydD) / g.s2 +
                                   d2 * RABS(dsdD) / (sig * g.s2));
            gD += dLdG * dGdD;
            mD += mLdG * mGdD;
            nD += 1;
            if (win[o] == (int32_t)q) {
              gD += g_depth[o] * h[2];
              mD += RABS(g_depth[o]) * RABS(h[2]);
              nD += 1;
            }
          }
        g_depth_in[ns * k + q] = gD;
        for (int ch = 0; ch < 3; ++ch) g_rgb_in[(ns * k + q) * 3 + ch] = gc[ch];
        if (m_depth_in) m_depth_in[ns * k + q] = mD;
        if (m_rgb_in)
          for (int ch = 0; ch < 3; ++ch) m_rgb_in[(ns * k + q) * 3 + ch] = mc[ch];
        if (cnt_in) cnt_in[ns * k + q] = nD;
      }
  }
  free(win);
  free(od);
  free(orgb);
  free(oa);
  free(tape);
  free(start);
  free(fill);
  free(band_G);
  free(band_q);
  return 0;
}

int orc_splat_backward(const orc_camera *src, int K, const float *depth, const uint8_t *rgb,
                       const orc_camera *tgt, const orc_splat_params *sp, const real *g_rgb,
                       const real *g_depth, const real *g_alpha, real *g_depth_in,
                       real *g_rgb_in) {
  return orc_splat_backward_mag(src, K, depth, rgb, tgt, sp, g_rgb, g_depth, g_alpha, g_depth_in,
                                g_rgb_in, NULL, NULL, NULL);
}

/* ------------------------------------------------------------------------
 * Adjoint of extraction + fusion with respect to the input depths.
 *
 * L = <g, depth_tsdf>.  With d = bin(p), Delta = F_d - F_{d+1}, dz = z_{d+1}-z_d:
 *   d depth / d F_d = -dz F_{d+1} / Delta^2,  d depth / d F_{d+1} = dz F_d / Delta^2.
 * At a voxel, F = (omega_tmp F_prev + sum omega_k c_k) / W:
 *   dF/dc_k = omega_k / W,  dF/domega_k = (c_k - F) / W,
 *   dc_k/dD_k[q] = 1 if s_k < tau (unclamped), else 0.
 * omega_k[q] = min(scale (nu/w^2)^(-1/2), 1):
 *   domega/dnu = -0.5 scale w^-2 (nu/w^2)^(-3/2) where the min is not active
 *   and nu > 0, else 0;
 *   dnu/dD_q = sum_n 2 (D_q - D_n) [ (D_q - D_n)^2 < tau_w^2 ],
 *   dnu/dD_n = -2 (D_q - D_n) [ same ]   (valid in-bounds neighbours n).
 * No gradient reaches the carried state, the mask or the cameras.  The two
 * voxels per pixel are recomputed from the inputs (the volume is not kept).
 *
 * With a pixel list, only the listed target pixels carry an upstream
 * gradient (g_out per list entry); every other pixel's is zero and adds
 * nothing, so only the listed pixels' voxels are formed.
 * Error-bound outputs (optional, for the tests' tolerance): g_mag[q] is the
 * same sum over the magnitudes of its terms, each term's factors replaced
 * by their magnitudes, and a difference of computed values by the sum of
 * their magnitudes (running error analysis: a sum of n terms rounded in
 * any order lies within about (n + c) 2^-24 g_mag of the exact sum);
 * g_cnt[q] counts the terms of g_depth_in[q], *conf_cnt_max the most terms
 * of any dL/domega entry (which feeds the window terms).  For a sum formed
 * in fixed point (every term rounded to one quantum Q): g_qsens[q] bounds
 * the error of g_depth_in[q] in units of Q (half a quantum per term, and a
 * window term's sensitivity to its dL/domega sum), and *term_bound is the
 * largest |term| any listed voxel can produce, |gF| max(1, tau + |F|) / W.
 * ---------------------------------------------------------------------- */
int orc_tsdf_backward_px(const orc_camera *src, int K, const float *depth,
                         const orc_camera *tgt, const orc_tsdf_params *p, const float *mask,
                         const real *F_prev, const real *W_prev, const real *g_out,
                         const int32_t *pixels, int npx, real *g_depth_in, real *g_mag,
                         int32_t *g_cnt, int32_t *conf_cnt_max, real *g_qsens,
                         double *term_bound) {
  const int D = p->num_bins;
  const int Ws = src[0].width, Hs = src[0].height, Wt = tgt->width, Ht = tgt->height;
  const size_t ns = (size_t)Ws * Hs;
  /* the voxels of the listed pixels (all pixels, row-major, without a list);
   * g_out, F_prev and W_prev follow the list */
  const size_t nt = pixels ? (size_t)npx : (size_t)Wt * Ht;
  real *conf = (real *)calloc(ns * K, sizeof(real));
  real *gconf = (real *)calloc(ns * K, sizeof(real));
  real *mconf = (real *)calloc(ns * K, sizeof(real));
  int32_t *nconf = (int32_t *)calloc(ns * K, sizeof(int32_t));
  real *F = (real *)malloc(sizeof(real) * nt * D), *W = (real *)malloc(sizeof(real) * nt * D);
  real *dep = (real *)malloc(sizeof(real) * nt);
  int32_t *bin = (int32_t *)malloc(sizeof(int32_t) * nt);
  real *zb = (real *)malloc(sizeof(real) * D), *tb = (real *)malloc(sizeof(real) * D);
  if (!conf || !gconf || !mconf || !nconf || !F || !W || !dep || !bin || !zb || !tb) return -2;
  for (int k = 0; k < K; ++k) orc_confidence(depth + ns * k, Ws, Hs, p, conf + ns * k);
  orc_integrate(src, K, depth, conf, tgt, p, mask, F_prev, W_prev, F, W, pixels,
                pixels ? npx : 0);
  orc_extract(p, F, W, (int)nt, dep, bin);
  orc_bins(p, zb, tb);
  real Hk[16][9], ck[16][3];
  for (int k = 0; k < K; ++k) relproj(tgt, &src[k], Hk[k], ck[k]);
  for (size_t n = 0; n < ns * K; ++n) g_depth_in[n] = 0;
  if (g_mag)
    for (size_t n = 0; n < ns * K; ++n) g_mag[n] = 0;
  if (g_cnt)
    for (size_t n = 0; n < ns * K; ++n) g_cnt[n] = 0;
  if (g_qsens)
    for (size_t n = 0; n < ns * K; ++n) g_qsens[n] = 0;
  double tb_max = 0;
  for (size_t i = 0; i < nt; ++i) {
    const size_t pix = pixels ? (size_t)pixels[i] : i;
    const int d = bin[i];
    if (d < 0) continue;
    const real *f = F + i * D;
    const real delta = f[d] - f[d + 1], dz = zb[d + 1] - zb[d];
    const real gF[2] = {g_out[i] * (-dz * f[d + 1] / (delta * delta)),
                        g_out[i] * (dz * f[d] / (delta * delta))};
    /* magnitudes (running error bound): dz and delta are exact differences
     * of shared values (Sterbenz; opposite signs), so they enter as is */
    const real aF[2] = {RABS(g_out[i]) * (dz * RABS(f[d + 1]) / (delta * delta)),
                        RABS(g_out[i]) * (dz * RABS(f[d]) / (delta * delta))};
    const int x = (int)(pix % Wt), y = (int)(pix / Wt);
    for (int e = 0; e < 2; ++e) {
      const int dd = d + e;
      const real z = zb[dd], tau = tb[dd];
      const real Wn = W[i * D + dd], Fv = F[i * D + dd];
      {
        /* largest term this voxel can produce: |gF| / W times max(1, tau + |F|)
         * (fusion weights are at most 1, clamped distances at most tau) */
        const double gb = fabs((double)gF[e]) / (double)Wn;
        const double m = gb * fmax(1.0, (double)tau + fabs((double)Fv));
        if (m > tb_max) tb_max = m;
      }
      for (int k = 0; k < K; ++k) {
        real h[3], X[3];
        ray_of(Hk[k], (real)x + (real)0.5, (real)y + (real)0.5, h);
        point_at(h, ck[k], z, X);
        if (!(X[2] > 0)) continue;
        const real inv = (real)1 / X[2];
        const real u = X[0] * inv, v = X[1] * inv;
        if (!(u >= 0 && u < (real)Ws && v >= 0 && v < (real)Hs)) continue;
        const size_t q = (size_t)(int)v * Ws + (size_t)(int)u;
        const float Dk = depth[ns * k + q];
        if (!depth_ok(Dk)) continue;
        const real s = (real)Dk - X[2];
        if (s < -tau) continue;
        const real cval = RMIN(s, tau);
        const real w = conf[ns * k + q];
        if (s < tau) {
          g_depth_in[ns * k + q] += gF[e] * w / Wn;
          if (g_mag) g_mag[ns * k + q] += aF[e] * w / Wn;
          if (g_cnt) g_cnt[ns * k + q] += 1;
          if (g_qsens) g_qsens[ns * k + q] += (real)0.5;
        }
        gconf[ns * k + q] += gF[e] * (cval - Fv) / Wn;
        mconf[ns * k + q] += aF[e] * (RABS(cval) + RABS(Fv)) / Wn;
        nconf[ns * k + q] += 1;
      }
    }
  }
  if (term_bound) *term_bound = tb_max;
  if (conf_cnt_max) {
    int32_t m = 0;
    for (size_t n = 0; n < ns * K; ++n) m = nconf[n] > m ? nconf[n] : m;
    *conf_cnt_max = m;
  }
  /* chain through the window statistic */
  const int r = (p->conf_window - 1) / 2;
  const real tw2 = (real)p->conf_tau * (real)p->conf_tau;
  const real n2 = (real)(p->conf_window * p->conf_window);
  for (int k = 0; k < K; ++k) {
    const float *dk = depth + ns * k;
    for (int j = 0; j < Hs; ++j)
      for (int i = 0; i < Ws; ++i) {
        const size_t q = (size_t)j * Ws + i;
        const real gq = gconf[ns * k + q];
        if (gq == 0 || !depth_ok(dk[q])) continue;
        real nu = 0;
        for (int dy = -r; dy <= r; ++dy)
          for (int dx = -r; dx <= r; ++dx) {
            const int ii = i + dx, jj = j + dy;
            if (ii < 0 || ii >= Ws || jj < 0 || jj >= Hs) continue;
            const float dn = dk[(size_t)jj * Ws + ii];
            if (depth_ok(dn)) {
              const real dd = (real)dk[q] - (real)dn;
              nu = nu + RMIN(dd * dd, tw2);
            } else {
              nu = nu + tw2;
            }
          }
        if (!(nu > 0)) continue;
        const real raw = (real)p->conf_scale / RSQRT(nu / n2);
        if (!(raw < 1)) continue; /* min(., 1) active */
        const real dwdnu = (real)-0.5 * raw / nu;
        const real gnu = gq * dwdnu;
        const real agnu = mconf[ns * k + q] * ((real)0.5 * raw / nu);
        for (int dy = -r; dy <= r; ++dy)
          for (int dx = -r; dx <= r; ++dx) {
            const int ii = i + dx, jj = j + dy;
            if (ii < 0 || ii >= Ws || jj < 0 || jj >= Hs || (dx == 0 && dy == 0)) continue;
            const size_t n = (size_t)jj * Ws + ii;
            if (!depth_ok(dk[n])) continue;
            const real dd = (real)dk[q] - (real)dk[n];
            if (!(dd * dd < tw2)) continue;
            g_depth_in[ns * k + q] += gnu * (real)2 * dd;
            g_depth_in[ns * k + n] -= gnu * (real)2 * dd;
            if (g_mag) {
              g_mag[ns * k + q] += agnu * (real)2 * RABS(dd);
              g_mag[ns * k + n] += agnu * (real)2 * RABS(dd);
            }
            if (g_cnt) {
              g_cnt[ns * k + q] += 1;
              g_cnt[ns * k + n] += 1;
            }
            if (g_qsens) {
              /* an absolute error e in dL/domega_q moves this term by
               * e |domega/dnu| 2 |dd|; a sum of nconf terms each rounded to a
               * quantum carries at most nconf / 2 quanta */
              const real qs = (real)0.5 * (real)nconf[ns * k + q] * ((real)0.5 * raw / nu) *
                              (real)2 * RABS(dd);
              g_qsens[ns * k + q] += qs;
              g_qsens[ns * k + n] += qs;
            }
          }
      }
  }
  free(conf);
  free(gconf);
  free(mconf);
  free(nconf);
  free(F);
  free(W);
  free(dep);
  free(bin);
  free(zb);
  free(tb);
  return 0;
}

int orc_tsdf_backward(const orc_camera *src, int K, const float *depth, const orc_camera *tgt,
                      const orc_tsdf_params *p, const float *mask, const real *F_prev,
                      const real *W_prev, const real *g_out, real *g_depth_in) {
  return orc_tsdf_backward_px(src, K, depth, tgt, p, mask, F_prev, W_prev, g_out, NULL, 0,
                              g_depth_in, NULL, NULL, NULL, NULL, NULL);
}
