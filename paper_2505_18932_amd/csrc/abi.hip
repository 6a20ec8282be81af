// C ABI of the geometry stage: argument validation (before anything is
// enqueued), workspace layout, the relative projection of camera pairs, and
// the launches.  See include/ggeom.h for the contract of each entry point.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "batch_internal.h"
#include "ggeom_internal.h"
#include "ewa_internal.h"

namespace gg {

// ---------------------------------------------------------------------------
// errors

static thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int check_hip(hipError_t e, const char *what) {
  if (e == hipSuccess) return GG_OK;
  return fail(GG_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// kernel timing

namespace {
struct TimedLaunch {
  std::string name;
  hipEvent_t start, stop;
};
std::mutex g_tmu;
bool g_timing = false;
std::string g_timing_only;  // time only kernels whose name contains this (empty: all)
std::vector<TimedLaunch> g_launches;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t take_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

KernelTimer::KernelTimer(const char *name, hipStream_t s) : name_(name), stream_(s), slot_(-1) {
  std::lock_guard<std::mutex> lk(g_tmu);
  if (!g_timing) return;
  if (!g_timing_only.empty() && !strstr(name, g_timing_only.c_str())) return;
  TimedLaunch t{name, take_event(), take_event()};
  if (!t.start || !t.stop) return;
  if (hipEventRecord(t.start, s) != hipSuccess) return;
  g_launches.push_back(t);
  slot_ = (int)g_launches.size() - 1;
}

KernelTimer::~KernelTimer() {
  if (slot_ < 0) return;
  std::lock_guard<std::mutex> lk(g_tmu);
  if (slot_ < (int)g_launches.size()) (void)hipEventRecord(g_launches[slot_].stop, stream_);
}

// ---------------------------------------------------------------------------
// helpers

// m = floor(2^32 / d) (2^32 - 1 for d = 1) underestimates n / d by less
// than one for every n < 2^32, which the single correction in fdiv() fixes.
FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  f.s = 0;
  f.m = d <= 1 ? 0xffffffffu : (uint32_t)((1ull << 32) / d);
  return f;
}

// The FP32 value nearest v, a binary128 evaluation whose error lies far
// below 2^-100 m (m: the summed magnitudes of the terms it adds).  A v
// within 2^-100 m of the midpoint of the two floats around it is taken to
// be that midpoint, an exact tie, and rounds to the float with the even
// significand: cameras aligned with the axes make exact ties common, and
// the last binary128 bits of a tie are noise of the evaluation order.
static float nearest_f32(__float128 v, __float128 m) {
  const float f = (float)v;
  const float g = std::nextafter(f, (__float128)f <= v ? INFINITY : -INFINITY);
  const float lo = std::min(f, g), hi = std::max(f, g);
  const __float128 d = v - ((__float128)lo + (__float128)hi) * 0.5Q;
  if ((d < 0 ? -d : d) <= 0x1p-100Q * m) {
    uint32_t bits;
    std::memcpy(&bits, &lo, sizeof bits);
    return (bits & 1u) ? hi : lo;
  }
  return f;
}

// H = K_b R_b R_a^T K_a^{-1}, c = K_b (t_b - R_b R_a^T t_a): M = R_b R_a^T
// and e = t_b - M t_a first, then the intrinsics of b on the left and those
// of a on the right, in binary128 (113-bit significand), rounded once to
// FP32 (nearest_f32).  binary128 keeps every entry far below an FP32
// rounding step of its exact value, also entries that are small differences
// of large terms, so the rounding is that of the exact product whatever the
// evaluation order, exact ties included.
// An entry below 2^-50 of the summed magnitudes of its monomials (the same
// formulas over magnitudes, carried beside the values) is cancellation
// residue and becomes 0, so that it is not left to the evaluation order.
void relproj(const gg_camera &a, const gg_camera &b, Proj &out) {
  typedef __float128 q;
  auto qa = [](q x) { return x < 0 ? -x : x; };
  q M[3][3], Mm[3][3], e[3], em[3], A[3][3], Am[3][3], H[9], Hm[9], c[3], cm[3];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      const q b0 = b.R[3 * r + 0], b1 = b.R[3 * r + 1], b2 = b.R[3 * r + 2];
      const q a0 = a.R[3 * k + 0], a1 = a.R[3 * k + 1], a2 = a.R[3 * k + 2];
      M[r][k] = (b0 * a0 + b1 * a1) + b2 * a2;
      Mm[r][k] = (qa(b0) * qa(a0) + qa(b1) * qa(a1)) + qa(b2) * qa(a2);
    }
  for (int r = 0; r < 3; ++r) {
    e[r] = (q)b.t[r] - ((M[r][0] * (q)a.t[0] + M[r][1] * (q)a.t[1]) + M[r][2] * (q)a.t[2]);
    em[r] = qa(b.t[r]) +
            ((Mm[r][0] * qa(a.t[0]) + Mm[r][1] * qa(a.t[1])) + Mm[r][2] * qa(a.t[2]));
  }
  const q bfx = b.fx, bfy = b.fy, bcx = b.cx, bcy = b.cy;
  for (int k = 0; k < 3; ++k) {
    A[0][k] = bfx * M[0][k] + bcx * M[2][k];
    A[1][k] = bfy * M[1][k] + bcy * M[2][k];
    A[2][k] = M[2][k];
    Am[0][k] = bfx * Mm[0][k] + qa(bcx) * Mm[2][k];
    Am[1][k] = bfy * Mm[1][k] + qa(bcy) * Mm[2][k];
    Am[2][k] = Mm[2][k];
  }
  c[0] = bfx * e[0] + bcx * e[2];
  c[1] = bfy * e[1] + bcy * e[2];
  c[2] = e[2];
  cm[0] = bfx * em[0] + qa(bcx) * em[2];
  cm[1] = bfy * em[1] + qa(bcy) * em[2];
  cm[2] = em[2];
  const q afx = a.fx, afy = a.fy, acx = a.cx, acy = a.cy;
  for (int r = 0; r < 3; ++r) {
    const q h0 = A[r][0] / afx, h1 = A[r][1] / afy;
    const q m0 = Am[r][0] / afx, m1 = Am[r][1] / afy;
    H[3 * r + 0] = h0;
    H[3 * r + 1] = h1;
    H[3 * r + 2] = (A[r][2] - h0 * acx) - h1 * acy;
    Hm[3 * r + 0] = m0;
    Hm[3 * r + 1] = m1;
    Hm[3 * r + 2] = (Am[r][2] + m0 * qa(acx)) + m1 * qa(acy);
  }
  const q tiny = 0x1p-50Q;
  for (int i = 0; i < 9; ++i) out.H[i] = qa(H[i]) < tiny * Hm[i] ? 0.0f : nearest_f32(H[i], Hm[i]);
  for (int i = 0; i < 3; ++i) out.c[i] = qa(c[i]) < tiny * cm[i] ? 0.0f : nearest_f32(c[i], cm[i]);
}

static bool finite_f(float v) { return std::isfinite(v); }

static int check_camera(const gg_camera *c, const char *what) {
  if (!c) return fail(GG_ERR_INVALID, "%s: camera is NULL", what);
  if (!(c->fx > 0.0f) || !(c->fy > 0.0f) || !finite_f(c->fx) || !finite_f(c->fy) ||
      !finite_f(c->cx) || !finite_f(c->cy))
    return fail(GG_ERR_INVALID, "%s: intrinsics must be finite with fx, fy > 0", what);
  for (float v : c->R)
    if (!finite_f(v)) return fail(GG_ERR_INVALID, "%s: rotation is not finite", what);
  for (float v : c->t)
    if (!finite_f(v)) return fail(GG_ERR_INVALID, "%s: translation is not finite", what);
  if (c->width < 1 || c->height < 1 || c->width > 16384 || c->height > 16384)
    return fail(GG_ERR_INVALID, "%s: size %dx%d outside 1..16384", what, c->width, c->height);
  return GG_OK;
}

static int check_sources(const gg_camera *src, int32_t K, const char *what) {
  if (!src) return fail(GG_ERR_INVALID, "%s: src is NULL", what);
  if (K < 1) return fail(GG_ERR_INVALID, "%s: K = %d, need K >= 1", what, K);
  if (K > GG_MAX_VIEWS)
    return fail(GG_ERR_UNSUPPORTED, "%s: K = %d exceeds %d views", what, K, GG_MAX_VIEWS);
  for (int k = 0; k < K; ++k) {
    if (int rc = check_camera(&src[k], what)) return rc;
    if (src[k].width != src[0].width || src[k].height != src[0].height)
      return fail(GG_ERR_INVALID, "%s: source views differ in size", what);
  }
  return GG_OK;
}

static int check_tsdf(const gg_tsdf_params *p, const char *what) {
  if (!p) return fail(GG_ERR_INVALID, "%s: params NULL", what);
  if (!(p->z_near > 0.0f) || !(p->z_far > p->z_near) || !finite_f(p->z_far))
    return fail(GG_ERR_INVALID, "%s: need 0 < z_near < z_far < inf", what);
  if (p->num_bins < 2) return fail(GG_ERR_INVALID, "%s: num_bins = %d < 2", what, p->num_bins);
  if (p->num_bins > GG_MAX_BINS)
    return fail(GG_ERR_UNSUPPORTED, "%s: num_bins = %d > %d", what, p->num_bins, GG_MAX_BINS);
  if (!(p->trunc > 0.0f) || !finite_f(p->trunc))
    return fail(GG_ERR_INVALID, "%s: trunc must be > 0", what);
  if (!(p->conf_tau >= 0.0f) || !(p->conf_scale >= 0.0f) || !finite_f(p->conf_tau) ||
      !finite_f(p->conf_scale))
    return fail(GG_ERR_INVALID, "%s: conf_tau, conf_scale must be >= 0", what);
  if (p->conf_window < 1 || p->conf_window % 2 == 0 || p->conf_window > GG_MAX_WINDOW)
    return fail(GG_ERR_INVALID, "%s: conf_window must be odd in 1..%d", what, GG_MAX_WINDOW);
  if (!(p->decay >= 0.0f && p->decay <= 1.0f) || !(p->weight_cap >= 0.0f) ||
      !finite_f(p->weight_cap))
    return fail(GG_ERR_INVALID, "%s: need decay in [0,1], weight_cap >= 0", what);
  return GG_OK;
}

static int check_splat(const gg_splat_params *p, const char *what) {
  if (!p) return fail(GG_ERR_INVALID, "%s: params NULL", what);
  if (!(p->sigma_px > 0.0f) || !finite_f(p->sigma_px))
    return fail(GG_ERR_INVALID, "%s: sigma_px must be > 0", what);
  if (!(p->band_rel >= 0.0f) || !finite_f(p->band_rel))
    return fail(GG_ERR_INVALID, "%s: band_rel must be >= 0", what);
  if (!(p->z_min >= 0.0f) || !finite_f(p->z_min))
    return fail(GG_ERR_INVALID, "%s: z_min must be >= 0", what);
  if (!(p->r_max_px > 0.0f) || !(p->r_max_px <= 64.0f))
    return fail(GG_ERR_INVALID, "%s: r_max_px must be in (0, 64]", what);
  return GG_OK;
}

static bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

static size_t up256(size_t n) { return (n + 255) & ~(size_t)255; }

// ---------------------------------------------------------------------------
// workspace layouts

struct SplatLayout {
  uint32_t ntx, nty, ntiles, cap;
  size_t count, offset, cursor, list, total;
};

// Workspace of difference_masks: the low-resolution mask and its 3 x 3
// maximum, K planes each.
static size_t mask_ws_bytes(int32_t K, int32_t w, int32_t h, int32_t factor) {
  const size_t wq = (size_t)((w + factor - 1) / factor), hq = (size_t)((h + factor - 1) / factor);
  return 2 * up256(sizeof(float) * wq * hq * (size_t)K);
}

static SplatLayout splat_layout(int K, int sw, int sh, int tw, int th, const gg_splat_params *sp) {
  SplatLayout L{};
  L.ntx = (uint32_t)((tw + kTile - 1) / kTile);
  L.nty = (uint32_t)((th + kTile - 1) / kTile);
  L.ntiles = L.ntx * L.nty;
  const size_t n = (size_t)K * L.ntiles;
  const size_t cap = (size_t)K * sw * sh * splat_tiles_per_splat(sp->r_max_px);
  L.cap = cap > 0xffffffffull ? 0xffffffffu : (uint32_t)cap;
  size_t o = 0;
  L.count = o;
  o += up256(4 * (n + 1));
  L.offset = o;
  o += up256(4 * (n + 1));
  L.cursor = o;
  o += up256(4 * (n + 1));
  L.list = o;
  o += up256(4 * cap);
  L.total = o;
  return L;
}

struct EwaLayout {
  uint32_t ntx, nty, ntiles, cap;
  size_t count, offset, cursor, keys, keys_alt, rec, total;
};

static EwaLayout ewa_layout(int K, int sw, int sh, int tw, int th, const gg_splat_params *sp) {
  EwaLayout L{};
  L.ntx = (uint32_t)((tw + kEwaTile - 1) / kEwaTile);
  L.nty = (uint32_t)((th + kEwaTile - 1) / kEwaTile);
  L.ntiles = L.ntx * L.nty;
  const size_t n = (size_t)K * L.ntiles;
  const size_t cap = (size_t)K * sw * sh * ewa_tiles_per_splat(sp->r_max_px);
  L.cap = cap > 0xffffffffull ? 0xffffffffu : (uint32_t)cap;
  size_t o = 0;
  L.count = o;
  o += up256(4 * (n + 1));
  L.offset = o;
  o += up256(4 * (n + 1));
  L.cursor = o;
  o += up256(4 * (n + 1));
  L.keys = o;
  o += up256(8 * cap);
  L.keys_alt = o;
  o += up256(8 * cap);
  L.rec = o;
  o += up256(32 * (size_t)K * sw * sh);
  L.total = o;
  return L;
}

struct TsdfLayout {
  size_t table, bins, acc, gnu, total;
};

static TsdfLayout tsdf_layout(int K, int sw, int sh, int D, bool backward) {
  TsdfLayout L{};
  const size_t ns = (size_t)sw * sh;
  size_t o = 0;
  L.table = o;
  o += up256(8 * table_view_records(sw, sh) * K);
  L.bins = o;
  o += up256(8 * (size_t)D);
  if (backward) {
    L.acc = o;  // acc_D, acc_w, max: contiguous
    o += up256(8 * (2 * ns * K + 1));
    L.gnu = o;
    o += up256(4 * ns * K);
  }
  L.total = o;
  return L;
}

static int check_ws(void *ws, size_t have, size_t need, const char *what) {
  if (need == 0) return GG_OK;
  if (!ws) return fail(GG_ERR_WORKSPACE, "%s: ws is NULL, need %zu bytes", what, need);
  if (have < need) return fail(GG_ERR_WORKSPACE, "%s: ws has %zu bytes, need %zu", what, have, need);
  if (!aligned(ws, 256)) return fail(GG_ERR_WORKSPACE, "%s: ws must be 256-byte aligned", what);
  return GG_OK;
}

// Launch shape of the volume kernels: V bins per thread, whole pixels per
// workgroup, neighbouring pixels per wavefront row (the caller's
// gg_volume_tuning, per call; NULL or zero fields: the defaults).
static int check_tuning(const gg_volume_tuning *t, const char *what) {
  if (!t) return GG_OK;
  if (t->pixels_per_block < 0 || t->pixels_per_block > 1024)
    return fail(GG_ERR_INVALID, "%s: pixels_per_block %d outside 0..1024", what,
                t->pixels_per_block);
  if (t->pixels_per_row < 0 || t->pixels_per_row > 64)
    return fail(GG_ERR_INVALID, "%s: pixels_per_row %d outside 0..64", what, t->pixels_per_row);
  const int v = t->bins_per_thread;
  if (v != 0 && v != 1 && v != 2 && v != 4 && v != 8)
    return fail(GG_ERR_INVALID, "%s: bins_per_thread %d not in {0, 1, 2, 4, 8}", what, v);
  if (t->band_width < 0 || t->band_width > 65536)
    return fail(GG_ERR_INVALID, "%s: band_width %d outside 0..65536", what, t->band_width);
  return GG_OK;
}

struct VolumeShape {
  int V;
  uint32_t cpp, ppb, threads, nblocks, pw_shift;
  uint32_t band_px;  // fusion tile order: band width in target pixels
};

constexpr uint32_t kDefaultBandPixels = 256;

// The fusion's tile order (IntegrateArgs::band_*) for a target of width x
// height pixels in tiles of ppb pixels: bands of band_px pixels across where
// whole tiles make up each row, else row-major.
static void set_band_order(IntegrateArgs &a, int width, int height, uint32_t ppb,
                           uint32_t band_px) {
  a.band_T = a.band_B = a.band_H = 0;
  if ((uint32_t)width % ppb != 0) return;
  const uint32_t T = (uint32_t)width / ppb;
  const uint32_t B = std::max(1u, band_px / ppb);
  if (B >= T) return;
  a.band_T = T;
  a.band_B = B;
  a.band_H = (uint32_t)height;
}

// Largest power of two <= cap (and <= 64) dividing ppb, as a shift.
static uint32_t pick_pw_shift(uint32_t ppb, int cap) {
  uint32_t sh = 0;
  while ((2u << sh) <= (uint32_t)cap && (2u << sh) <= 64u && ppb % (2u << sh) == 0) ++sh;
  return sh;
}

// Bins per thread: the tuning's choice where it divides D (and, for 8, the
// volumes are 32-byte aligned), else 4, 2 or 1, the largest dividing D.
static int volume_v(int D, bool aligned32, int o) {
  if (o > 0 && D % o == 0 && (o < 8 || aligned32)) return o;
  return (D % 4 == 0) ? 4 : (D % 2 == 0 ? 2 : 1);
}

static int volume_shape(int D, uint32_t npix, VolumeShape &s, const char *what,
                        bool aligned32, const gg_volume_tuning *tun) {
  if (int rc = check_tuning(tun, what)) return rc;
  const int ppb_t = tun ? tun->pixels_per_block : 0;
  const int pw_t = tun ? tun->pixels_per_row : 0;
  s.V = volume_v(D, aligned32, tun ? tun->bins_per_thread : 0);
  s.cpp = (uint32_t)(D / s.V);
  if (s.cpp > 1024) return fail(GG_ERR_UNSUPPORTED, "%s: D = %d too large", what, D);
  uint32_t ppb = ppb_t > 0 ? (uint32_t)ppb_t : 512u / s.cpp;
  if (ppb < 1) ppb = 1;
  while (ppb > 1 && ppb * s.cpp > 1024) --ppb;
  s.ppb = ppb;
  s.threads = ppb * s.cpp;
  s.nblocks = (npix + ppb - 1) / ppb;
  s.pw_shift = pick_pw_shift(ppb, pw_t > 0 ? pw_t : 16);
  s.band_px = (tun && tun->band_width > 0) ? (uint32_t)tun->band_width : kDefaultBandPixels;
  return GG_OK;
}

// Scratch of tsdf_integrate_noalloc: a file-scope device array, one copy per
// device the library runs on, held until the process ends.  Host code never
// uses the array's name as an address: its device address is looked up once
// per device (hipGetSymbolAddress, with that device current) and kept here.
constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

static int scratch_of_current_device(void **out, const char *what) {
  int dev = 0;
  if (int rc = check_hip(hipGetDevice(&dev), what)) return rc;
  if (dev < 0 || dev >= kMaxDevices)
    return fail(GG_ERR_UNSUPPORTED, "%s: device %d beyond %d", what, dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (int rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), what)) return rc;
    if (!p) return fail(GG_ERR_HIP, "%s: no device address for the scratch", what);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GG_OK;
}

}  // namespace gg

using namespace gg;

extern "C" {

const char *gg_last_error(void) { return g_err.c_str(); }

int gg_relative_projection(const gg_camera *a, const gg_camera *b, float *H, float *c) {
  if (int rc = check_camera(a, "gg_relative_projection")) return rc;
  if (int rc = check_camera(b, "gg_relative_projection")) return rc;
  if (!H || !c) return fail(GG_ERR_INVALID, "gg_relative_projection: NULL output");
  Proj P;
  relproj(*a, *b, P);
  memcpy(H, P.H, sizeof P.H);
  memcpy(c, P.c, sizeof P.c);
  return GG_OK;
}

size_t gg_workspace_size(int op, int32_t K, int32_t src_w, int32_t src_h, int32_t tgt_w,
                         int32_t tgt_h, int32_t num_bins, const gg_splat_params *sp) {
  if (K < 1 || K > GG_MAX_VIEWS || src_w < 1 || src_h < 1 || tgt_w < 1 || tgt_h < 1) return 0;
  switch (op) {
    case GG_OP_SPLAT:
      if (!sp || check_splat(sp, "gg_workspace_size")) return 0;
      return splat_layout(K, src_w, src_h, tgt_w, tgt_h, sp).total;
    case GG_OP_SPLAT_BACKWARD:
      return 0;
    case GG_OP_TSDF_INTEGRATE:
      if (num_bins < 2) return 0;
      return tsdf_layout(K, src_w, src_h, num_bins, false).total;
    case GG_OP_TSDF_INTEGRATE_BACKWARD:
      if (num_bins < 2) return 0;
      return tsdf_layout(K, src_w, src_h, num_bins, true).total;
    case GG_OP_SPLAT_EWA:
      if (!sp || check_splat(sp, "gg_workspace_size")) return 0;
      return ewa_layout(K, src_w, src_h, tgt_w, tgt_h, sp).total;
    case GG_OP_DIFFERENCE_MASKS:  // num_bins carries gg_mask_params.factor
      if (num_bins < 1 || num_bins > 16) return 0;
      return mask_ws_bytes(K, src_w, src_h, num_bins);
    default:
      return 0;
  }
}

// The splat kernels' arguments for K views of `src` into `tgt`, workspace
// laid out by L from base pointer w (NULL: backward, no workspace).
static void make_splat_args(SplatArgs &a, const gg_camera *src, int32_t K, const float *depth,
                            const uint8_t *rgb, const gg_camera &tgt, const gg_splat_params &prm,
                            const SplatLayout &L, char *w) {
  for (int k = 0; k < K; ++k) {
    relproj(src[k], tgt, a.views[k].P);
    a.views[k].sscale = (float)((double)prm.sigma_px * (double)tgt.fx / (double)src[k].fx);
  }
  const int sw = src[0].width, sh = src[0].height;
  a.depth = depth;
  a.rgb = rgb;
  a.K = K;
  a.Ws = sw;
  a.Hs = sh;
  a.Wt = tgt.width;
  a.Ht = tgt.height;
  a.ns = (uint32_t)(sw * sh);
  a.nt = (uint32_t)(tgt.width * tgt.height);
  a.ws_div = make_fastdiv((uint32_t)sw);
  a.ntx = (int)L.ntx;
  a.nty = (int)L.nty;
  a.ntiles = L.ntiles;
  a.zmin = prm.z_min;
  a.rmax2 = prm.r_max_px * prm.r_max_px;
  a.band = 1.0f + prm.band_rel;
  if (w) {
    a.tile_count = (uint32_t *)(w + L.count);
    a.tile_offset = (uint32_t *)(w + L.offset);
    a.tile_cursor = (uint32_t *)(w + L.cursor);
    a.list = (uint32_t *)(w + L.list);
    a.list_cap = L.cap;
  }
}

int splat_views(const gg_camera *src, int32_t K, const float *depth, const uint8_t *rgb,
                const gg_camera *tgt, const gg_splat_params *prm, int32_t *win_idx,
                float *out_depth, float *out_rgb, float *out_alpha, float *out_tape, void *ws,
                size_t ws_bytes, void *stream) {
  const char *W = "splat_views";
  if (int rc = check_sources(src, K, W)) return rc;
  if (int rc = check_camera(tgt, W)) return rc;
  if (int rc = check_splat(prm, W)) return rc;
  if (!depth || !rgb || !win_idx || !out_depth || !out_rgb || !out_alpha)
    return fail(GG_ERR_INVALID, "%s: NULL array argument", W);
  const int sw = src[0].width, sh = src[0].height;
  const SplatLayout L = splat_layout(K, sw, sh, tgt->width, tgt->height, prm);
  if ((size_t)K * sw * sh * splat_tiles_per_splat(prm->r_max_px) > 0xffffffffull)
    return fail(GG_ERR_UNSUPPORTED, "%s: too many source pixels", W);
  if (int rc = check_ws(ws, ws_bytes, L.total, W)) return rc;
  SplatArgs a{};
  make_splat_args(a, src, K, depth, rgb, *tgt, *prm, L, (char *)ws);
  a.win_idx = win_idx;
  a.out_depth = out_depth;
  a.out_rgb = out_rgb;
  a.out_alpha = out_alpha;
  a.out_tape = out_tape;
  return launch_splat_forward(a, (hipStream_t)stream);
}

int splat_views_masked(const gg_camera *src, int32_t K, const float *depth, const uint8_t *rgb,
                       const gg_camera *tgt, const gg_splat_params *prm, const float *mask,
                       int32_t *win_idx, float *out_depth, float *out_rgb, float *out_alpha,
                       float *out_tape, float *out_mask, float *out_mask_max, void *ws,
                       size_t ws_bytes, void *stream) {
  const char *W = "splat_views_masked";
  if (int rc = check_sources(src, K, W)) return rc;
  if (int rc = check_camera(tgt, W)) return rc;
  if (int rc = check_splat(prm, W)) return rc;
  if (!depth || !rgb || !mask || !win_idx || !out_depth || !out_rgb || !out_alpha)
    return fail(GG_ERR_INVALID, "%s: NULL array argument", W);
  if (!out_mask && !out_mask_max)
    return fail(GG_ERR_INVALID, "%s: need out_mask or out_mask_max", W);
  const int sw = src[0].width, sh = src[0].height;
  const SplatLayout L = splat_layout(K, sw, sh, tgt->width, tgt->height, prm);
  if ((size_t)K * sw * sh * splat_tiles_per_splat(prm->r_max_px) > 0xffffffffull)
    return fail(GG_ERR_UNSUPPORTED, "%s: too many source pixels", W);
  if (int rc = check_ws(ws, ws_bytes, L.total, W)) return rc;
  SplatArgs a{};
  make_splat_args(a, src, K, depth, rgb, *tgt, *prm, L, (char *)ws);
  a.win_idx = win_idx;
  a.out_depth = out_depth;
  a.out_rgb = out_rgb;
  a.out_alpha = out_alpha;
  a.out_tape = out_tape;
  a.mask_in = mask;
  a.out_mask = out_mask;
  a.out_mask_max = out_mask_max;
  return launch_splat_forward(a, (hipStream_t)stream);
}

int splat_views_ewa(const gg_camera *src, int32_t K, const float *depth, const uint8_t *rgb,
                    const gg_camera *tgt, const gg_splat_params *prm, float lowpass,
                    int32_t sort_limit, float *out_rgb, float *out_alpha, float *out_depth,
                    void *ws, size_t ws_bytes, void *stream) {
  const char *W = "splat_views_ewa";
  if (sort_limit != 0 && (sort_limit < 64 || sort_limit > (int)kEwaSortCap))
    return fail(GG_ERR_INVALID, "%s: sort_limit %d outside 64..%u", W, sort_limit, kEwaSortCap);
  if (int rc = check_sources(src, K, W)) return rc;
  if (int rc = check_camera(tgt, W)) return rc;
  if (int rc = check_splat(prm, W)) return rc;
  if (!(lowpass >= 0.0f) || !finite_f(lowpass))
    return fail(GG_ERR_INVALID, "%s: lowpass must be finite and >= 0", W);
  if (!depth || !rgb || !out_rgb || !out_alpha || !out_depth)
    return fail(GG_ERR_INVALID, "%s: NULL array argument", W);
  const int sw = src[0].width, sh = src[0].height;
  if ((size_t)K * sw * sh * ewa_tiles_per_splat(prm->r_max_px) > 0xffffffffull ||
      (size_t)K * sw * sh > 0x7fffffffull)
    return fail(GG_ERR_UNSUPPORTED, "%s: too many source pixels", W);
  const EwaLayout L = ewa_layout(K, sw, sh, tgt->width, tgt->height, prm);
  if (int rc = check_ws(ws, ws_bytes, L.total, W)) return rc;
  char *w = (char *)ws;
  EwaArgs a{};
  for (int k = 0; k < K; ++k) {
    relproj(src[k], *tgt, a.views[k].P);
    a.views[k].sscale = (float)((double)prm->sigma_px * (double)tgt->fx / (double)src[k].fx);
  }
  const double rd = (double)tgt->fy / (double)tgt->fx;
  a.depth = depth;
  a.rgb = rgb;
  a.K = K;
  a.Ws = sw;
  a.Hs = sh;
  a.Wt = tgt->width;
  a.Ht = tgt->height;
  a.ns = (uint32_t)(sw * sh);
  a.nt = (uint32_t)(tgt->width * tgt->height);
  a.ws_div = make_fastdiv((uint32_t)sw);
  a.ntx = (int)L.ntx;
  a.nty = (int)L.nty;
  a.ntiles = L.ntiles;
  a.fx = tgt->fx;
  a.fy = tgt->fy;
  a.cx = tgt->cx;
  a.cy = tgt->cy;
  a.ry = (float)rd;
  a.ry2 = (float)(rd * rd);
  a.lowpass = lowpass;
  a.zmin = prm->z_min;
  a.rmax = prm->r_max_px;
  a.tile_count = (uint32_t *)(w + L.count);
  a.tile_offset = (uint32_t *)(w + L.offset);
  a.tile_cursor = (uint32_t *)(w + L.cursor);
  a.keys = (unsigned long long *)(w + L.keys);
  a.keys_alt = (unsigned long long *)(w + L.keys_alt);
  a.cap = L.cap;
  a.rec = (float4 *)(w + L.rec);
  a.sort_limit = sort_limit == 0 ? kEwaSortCap : (uint32_t)sort_limit;
  a.out_rgb = out_rgb;
  a.out_alpha = out_alpha;
  a.out_depth = out_depth;
  return launch_splat_ewa(a, (hipStream_t)stream);
}

int difference_masks(int32_t K, int32_t width, int32_t height, const uint8_t *rgb,
                     const uint8_t *rgb_prev, const gg_mask_params *prm, float *mask,
                     const float *depth, const float *depth_filtered_prev,
                     float *depth_filtered, void *ws, size_t ws_bytes, void *stream) {
  const char *N = "difference_masks";
  if (K < 1 || K > GG_MAX_VIEWS)
    return fail(GG_ERR_INVALID, "%s: K = %d outside 1..%d", N, K, GG_MAX_VIEWS);
  if (width < 1 || height < 1 || width > 16384 || height > 16384)
    return fail(GG_ERR_INVALID, "%s: size %dx%d outside 1..16384", N, width, height);
  if (!prm) return fail(GG_ERR_INVALID, "%s: params NULL", N);
  if (!(prm->beta >= 0.0f && prm->beta <= 1.0f) || !(prm->lambda_t > 0.0f) ||
      !finite_f(prm->lambda_t) || prm->factor < 1 || prm->factor > 16)
    return fail(GG_ERR_INVALID, "%s: need beta in [0, 1], lambda_t > 0, factor in 1..16", N);
  if (!rgb || !rgb_prev || !mask) return fail(GG_ERR_INVALID, "%s: NULL array argument", N);
  if ((depth == nullptr) != (depth_filtered == nullptr))
    return fail(GG_ERR_INVALID, "%s: depth and depth_filtered go together", N);
  if (depth_filtered_prev && !depth)
    return fail(GG_ERR_INVALID, "%s: depth_filtered_prev needs depth", N);
  if (int rc = check_ws(ws, ws_bytes, mask_ws_bytes(K, width, height, prm->factor), N)) return rc;
  MaskArgs a{};
  a.rgb = rgb;
  a.rgb_prev = rgb_prev;
  a.K = K;
  a.W = width;
  a.H = height;
  a.factor = prm->factor;
  a.Wq = (width + prm->factor - 1) / prm->factor;
  a.Hq = (height + prm->factor - 1) / prm->factor;
  a.low = (float *)ws;
  a.pool = (float *)((char *)ws + up256(sizeof(float) * (size_t)a.Wq * a.Hq * K));
  a.mask = mask;
  a.depth = depth;
  a.prev = depth_filtered_prev;
  a.filtered = depth_filtered;
  a.beta = prm->beta;
  a.lambda_t = prm->lambda_t;
  return launch_difference_masks(a, (hipStream_t)stream);
}

int splat_views_backward(const gg_camera *src, int32_t K, const float *depth,
                         const uint8_t *rgb, const gg_camera *tgt, const gg_splat_params *prm,
                         const int32_t *win_idx, const float *out_depth, const float *out_rgb,
                         const float *out_tape, const float *g_rgb, const float *g_depth,
                         const float *g_alpha, float *g_depth_in, float *g_rgb_in, void *ws,
                         size_t ws_bytes, void *stream) {
  const char *W = "splat_views_backward";
  (void)ws;
  (void)ws_bytes;
  if (int rc = check_sources(src, K, W)) return rc;
  if (int rc = check_camera(tgt, W)) return rc;
  if (int rc = check_splat(prm, W)) return rc;
  if (!depth || !rgb || !win_idx || !out_depth || !out_rgb || !out_tape || !g_depth_in ||
      !g_rgb_in)
    return fail(GG_ERR_INVALID, "%s: NULL array argument", W);
  const int sw = src[0].width, sh = src[0].height;
  SplatArgs a{};
  const SplatLayout L = splat_layout(K, sw, sh, tgt->width, tgt->height, prm);
  make_splat_args(a, src, K, depth, rgb, *tgt, *prm, L, nullptr);
  a.fw_win = win_idx;
  a.fw_depth = out_depth;
  a.fw_rgb = out_rgb;
  a.fw_tape = out_tape;
  a.g_rgb = g_rgb;
  a.g_depth = g_depth;
  a.g_alpha = g_alpha;
  a.g_depth_in = g_depth_in;
  a.g_rgb_in = g_rgb_in;
  return launch_splat_backward(a, (hipStream_t)stream);
}

static int fill_views(const gg_camera *src, int32_t K, const gg_camera *tgt, Proj *views) {
  for (int k = 0; k < K; ++k) relproj(*tgt, src[k], views[k]);
  return GG_OK;
}

// True when every sample's view depth z_k = z h2 + c2 (z <= z_far, pixel
// centres inside the target) stays below 2^99, where the kernels' fast
// reciprocal is exact; otherwise they take IEEE division throughout.
static bool fast_reciprocal_safe(const Proj *views, int32_t K, const gg_camera &tgt,
                                 float z_far) {
  for (int k = 0; k < K; ++k) {
    const Proj &P = views[k];
    for (float v : P.H)
      if (!std::isfinite(v)) return false;
    for (float v : P.c)
      if (!std::isfinite(v)) return false;
    const double h2 = std::fabs((double)P.H[6]) * tgt.width + std::fabs((double)P.H[7]) * tgt.height +
                      std::fabs((double)P.H[8]);
    const double bound = (double)z_far * 1.01 * h2 + std::fabs((double)P.c[2]);
    if (!(bound < std::ldexp(1.0, 99))) return false;
  }
  return true;
}

static ConfArgs conf_args(const float *depth, float2 *table, int sw, int sh, int K,
                          const gg_tsdf_params *p) {
  ConfArgs c{};
  c.depth = depth;
  c.table = table;
  c.Ws = sw;
  c.Hs = sh;
  c.K = K;
  c.radius = (p->conf_window - 1) / 2;
  c.tw2 = p->conf_tau * p->conf_tau;
  c.n2 = (float)(p->conf_window * p->conf_window);
  c.scale = p->conf_scale;
  return c;
}

static void make_integrate_args(IntegrateArgs &a, const gg_camera *src, int32_t K,
                                const gg_camera &tgt, const gg_tsdf_params &prm,
                                const VolumeShape &vs, const float2 *table, const float2 *bins,
                                const float *mask, const float *F_prev, const float *W_prev,
                                float *F, float *W, float *out_depth, int32_t *out_bin) {
  fill_views(src, K, &tgt, a.views);
  const int sw = src[0].width, sh = src[0].height;
  a.table = table;
  a.bins = bins;
  a.mask = mask;
  a.F_prev = F_prev;
  a.W_prev = W_prev;
  a.F = F;
  a.W = W;
  a.out_depth = out_depth;
  a.out_bin = out_bin;
  a.K = K;
  a.Ws = sw;
  a.Hs = sh;
  a.D = prm.num_bins;
  a.npix = (uint32_t)(tgt.width * tgt.height);
  a.ns = (uint32_t)(sw * sh);
  a.wt_div = make_fastdiv((uint32_t)tgt.width);
  a.cpp_div = make_fastdiv(vs.cpp);
  a.cpp = vs.cpp;
  a.ppb = vs.ppb;
  a.pw_shift = vs.pw_shift;
  a.nblocks = vs.nblocks;
  set_band_order(a, tgt.width, tgt.height, vs.ppb, vs.band_px);
  a.decay = prm.decay;
  a.cap = prm.weight_cap;
  a.carry = F_prev != nullptr;
  a.exact_only = fast_reciprocal_safe(a.views, K, tgt, prm.z_far) ? 0 : 1;
  // Structured view-table loads take three vector instructions per sample off the carried
  // fusion, whose issue slots bound it at up to four views; at more views the texture address
  // unit is the tighter bound and they lose, and the forms without a carry would lose a
  // wavefront per SIMD to the extra address registers (measured; results are the same).
  a.rows = (table_rows_ok(sw) && F_prev != nullptr && K <= 4) ? 1 : 0;
}

// The view table (per source pixel: usable depth, fusion weight) and the
// bin depths into the workspace: the part of the fusion that depends on the
// depth maps only.
static int build_view_table(const gg_camera *src, int32_t K, const float *depth,
                            const gg_tsdf_params *prm, const TsdfLayout &L, char *w,
                            hipStream_t s) {
  const int sw = src[0].width, sh = src[0].height;
  if (int rc = launch_bins(*prm, (float2 *)(w + L.bins), s)) return rc;
  return launch_conf(conf_args(depth, (float2 *)(w + L.table), sw, sh, K, prm), s);
}

int tsdf_view_table(const gg_camera *src, int32_t K, const float *depth,
                    const gg_tsdf_params *prm, void *ws, size_t ws_bytes, void *stream) {
  const char *N = "tsdf_view_table";
  if (int rc = check_sources(src, K, N)) return rc;
  if (int rc = check_tsdf(prm, N)) return rc;
  if (!depth) return fail(GG_ERR_INVALID, "%s: NULL array argument", N);
  const TsdfLayout L = tsdf_layout(K, src[0].width, src[0].height, prm->num_bins, false);
  if (int rc = check_ws(ws, ws_bytes, L.total, N)) return rc;
  return build_view_table(src, K, depth, prm, L, (char *)ws, (hipStream_t)stream);
}

// depth NULL: the view table and bins are already in ws (tsdf_view_table).
static int integrate_impl(const char *N, bool tabled, const gg_camera *src, int32_t K,
                          const float *depth,
                          const gg_camera *tgt, const gg_tsdf_params *prm,
                          const float *temporal_mask, const float *F_prev, const float *W_prev,
                          float *F, float *W, float *out_depth, int32_t *out_bin,
                          const gg_volume_tuning *tuning, void *ws, size_t ws_bytes,
                          void *stream) {
  if (int rc = check_sources(src, K, N)) return rc;
  if (int rc = check_camera(tgt, N)) return rc;
  if (int rc = check_tsdf(prm, N)) return rc;
  if ((!tabled && !depth) || !F || !W) return fail(GG_ERR_INVALID, "%s: NULL array argument", N);
  if ((F_prev == nullptr) != (W_prev == nullptr))
    return fail(GG_ERR_INVALID, "%s: F_prev and W_prev go together", N);
  if ((out_depth == nullptr) != (out_bin == nullptr))
    return fail(GG_ERR_INVALID, "%s: out_depth and out_bin go together", N);
  const int sw = src[0].width, sh = src[0].height, D = prm->num_bins;
  const uint32_t npix = (uint32_t)(tgt->width * tgt->height);
  VolumeShape vs;
  const bool a32 = aligned(F, 32) && aligned(W, 32) && (!F_prev || (aligned(F_prev, 32) &&
                                                                     aligned(W_prev, 32)));
  if (int rc = volume_shape(D, npix, vs, N, a32, tuning)) return rc;
  const size_t va = 4 * (size_t)vs.V;
  if (!aligned(F, va) || !aligned(W, va) || (F_prev && (!aligned(F_prev, va) || !aligned(W_prev, va))))
    return fail(GG_ERR_INVALID, "%s: volumes must be %zu-byte aligned", N, va);
  if ((size_t)npix * D > (size_t)1 << 40) return fail(GG_ERR_UNSUPPORTED, "%s: volume too large", N);
  const TsdfLayout L = tsdf_layout(K, sw, sh, D, false);
  if (int rc = check_ws(ws, ws_bytes, L.total, N)) return rc;
  hipStream_t s = (hipStream_t)stream;
  char *w = (char *)ws;
  float2 *table = (float2 *)(w + L.table);
  float2 *bins = (float2 *)(w + L.bins);
  if (!tabled)
    if (int rc = build_view_table(src, K, depth, prm, L, w, s)) return rc;
  IntegrateArgs a{};
  make_integrate_args(a, src, K, *tgt, *prm, vs, table, bins, temporal_mask, F_prev, W_prev, F, W,
                      out_depth, out_bin);
  return launch_integrate(a, vs.V, vs.threads, s);
}

int tsdf_integrate(const gg_camera *src, int32_t K, const float *depth, const gg_camera *tgt,
                   const gg_tsdf_params *prm, const float *temporal_mask, const float *F_prev,
                   const float *W_prev, float *F, float *W, float *out_depth, int32_t *out_bin,
                   const gg_volume_tuning *tuning, void *ws, size_t ws_bytes, void *stream) {
  return integrate_impl("tsdf_integrate", false, src, K, depth, tgt, prm, temporal_mask, F_prev,
                        W_prev, F, W, out_depth, out_bin, tuning, ws, ws_bytes, stream);
}

int tsdf_integrate_tabled(const gg_camera *src, int32_t K, const gg_camera *tgt,
                          const gg_tsdf_params *prm, const float *temporal_mask,
                          const float *F_prev, const float *W_prev, float *F, float *W,
                          float *out_depth, int32_t *out_bin, const gg_volume_tuning *tuning,
                          void *ws, size_t ws_bytes, void *stream) {
  return integrate_impl("tsdf_integrate_tabled", true, src, K, nullptr, tgt, prm, temporal_mask,
                        F_prev, W_prev, F, W, out_depth, out_bin, tuning, ws, ws_bytes, stream);
}

int gg_fusion_stream_probe(const gg_camera *tgt, const gg_tsdf_params *prm,
                           const float *F_prev, const float *W_prev, float *F, float *W,
                           float *out_depth, int32_t *out_bin, const gg_volume_tuning *tuning,
                           void *ws, size_t ws_bytes, void *stream) {
  const char *N = "gg_fusion_stream_probe";
  if (int rc = check_camera(tgt, N)) return rc;
  if (int rc = check_tsdf(prm, N)) return rc;
  if (!F_prev || !W_prev || !F || !W || !out_depth || !out_bin)
    return fail(GG_ERR_INVALID, "%s: NULL array argument", N);
  const int D = prm->num_bins;
  const uint32_t npix = (uint32_t)(tgt->width * tgt->height);
  VolumeShape vs;
  const bool a32 = aligned(F, 32) && aligned(W, 32) && aligned(F_prev, 32) && aligned(W_prev, 32);
  if (int rc = volume_shape(D, npix, vs, N, a32, tuning)) return rc;
  const size_t va = 4 * (size_t)vs.V;
  if (!aligned(F, va) || !aligned(W, va) || !aligned(F_prev, va) || !aligned(W_prev, va))
    return fail(GG_ERR_INVALID, "%s: volumes must be %zu-byte aligned", N, va);
  if ((size_t)npix * D > (size_t)1 << 40) return fail(GG_ERR_UNSUPPORTED, "%s: volume too large", N);
  const TsdfLayout L = tsdf_layout(1, 1, 1, D, false);
  if (int rc = check_ws(ws, ws_bytes, L.total, N)) return rc;
  hipStream_t s = (hipStream_t)stream;
  float2 *bins = (float2 *)((char *)ws + L.bins);
  if (int rc = launch_bins(*prm, bins, s)) return rc;
  // the fusion kernel's own launch with no views: every voxel only decays
  // its carried weight (W = min(decay W_prev, cap), F = that weight times
  // F_prev over itself), so the kernel moves exactly its volume stream
  IntegrateArgs a{};
  a.table = (const float2 *)ws;
  a.bins = bins;
  a.F_prev = F_prev;
  a.W_prev = W_prev;
  a.F = F;
  a.W = W;
  a.out_depth = out_depth;
  a.out_bin = out_bin;
  a.K = 0;
  a.Ws = a.Hs = 1;
  a.D = D;
  a.npix = npix;
  a.ns = 1;
  a.wt_div = make_fastdiv((uint32_t)tgt->width);
  a.cpp_div = make_fastdiv(vs.cpp);
  a.cpp = vs.cpp;
  a.ppb = vs.ppb;
  a.pw_shift = vs.pw_shift;
  a.nblocks = vs.nblocks;
  a.decay = prm->decay;
  a.cap = prm->weight_cap;
  a.carry = 1;
  a.exact_only = 0;
  return launch_integrate(a, vs.V, vs.threads, s);
}

int tsdf_integrate_noalloc(const gg_camera *src, int32_t K, const float *depth,
                           const gg_camera *tgt, const gg_tsdf_params *prm,
                           const float *temporal_mask, const float *F_prev, const float *W_prev,
                           float *F, float *W, float *out_depth, int32_t *out_bin,
                           const gg_volume_tuning *tuning, void *stream) {
  const char *N = "tsdf_integrate_noalloc";
  if (int rc = check_sources(src, K, N)) return rc;
  if (int rc = check_tsdf(prm, N)) return rc;
  const size_t need = tsdf_layout(K, src[0].width, src[0].height, prm->num_bins, false).total;
  if (need > kScratchBytes)
    return fail(GG_ERR_UNSUPPORTED, "%s: needs %zu bytes of scratch, the static scratch holds %zu",
                N, need, kScratchBytes);
  void *ws = nullptr;
  if (int rc = scratch_of_current_device(&ws, N)) return rc;
  return integrate_impl(N, false, src, K, depth, tgt, prm, temporal_mask, F_prev, W_prev, F, W,
                        out_depth, out_bin, tuning, ws, kScratchBytes, stream);
}

int tsdf_raymarch(const gg_camera *src, int32_t K, const float *depth, const gg_camera *tgt,
                  const gg_tsdf_params *prm, const float *depth_prev, const float *acc_prev,
                  const float *temporal_mask, float *out_depth, float *out_acc,
                  int32_t *out_steps, void *ws, size_t ws_bytes, void *stream) {
  const char *N = "tsdf_raymarch";
  if (int rc = check_sources(src, K, N)) return rc;
  if (int rc = check_camera(tgt, N)) return rc;
  if (int rc = check_tsdf(prm, N)) return rc;
  if (!depth || !out_depth) return fail(GG_ERR_INVALID, "%s: NULL array argument", N);
  if ((depth_prev == nullptr) != (acc_prev == nullptr))
    return fail(GG_ERR_INVALID, "%s: depth_prev and acc_prev go together", N);
  if (temporal_mask && !depth_prev)
    return fail(GG_ERR_INVALID, "%s: temporal_mask needs depth_prev and acc_prev", N);
  const int sw = src[0].width, sh = src[0].height, D = prm->num_bins;
  const TsdfLayout L = tsdf_layout(K, sw, sh, D, false);
  if (int rc = check_ws(ws, ws_bytes, L.total, N)) return rc;
  hipStream_t s = (hipStream_t)stream;
  float2 *table = (float2 *)((char *)ws + L.table);
  if (int rc = launch_conf(conf_args(depth, table, sw, sh, K, prm), s)) return rc;
  RaymarchArgs a{};
  fill_views(src, K, tgt, a.views);
  a.table = table;
  a.K = K;
  a.Ws = sw;
  a.Hs = sh;
  a.ns = (uint32_t)(sw * sh);
  a.npix = (uint32_t)(tgt->width * tgt->height);
  a.wt_div = make_fastdiv((uint32_t)tgt->width);
  a.z_near = prm->z_near;
  a.z_far = prm->z_far;
  // bin width in inverse depth, formed as the bins are
  const float un = 1.0f / prm->z_near, uf = 1.0f / prm->z_far;
  a.du = (un - uf) / (float)(D - 1);
  a.trunc = prm->trunc;
  a.trunc_in_bins = prm->trunc_in_bins;
  a.decay = prm->decay;
  a.cap = prm->weight_cap;
  a.max_samples = 4 * D + 16;
  a.dprev = depth_prev;
  a.acc = acc_prev;
  a.mask = temporal_mask;
  a.out_depth = out_depth;
  a.out_acc = out_acc;
  a.out_steps = out_steps;
  a.exact_only = fast_reciprocal_safe(a.views, K, *tgt, prm->z_far) ? 0 : 1;
  return launch_raymarch(a, s);
}

static void centre_d(const gg_camera &c, double C[3]) {
  for (int r = 0; r < 3; ++r) {
    double v = 0;
    for (int k = 0; k < 3; ++k) v -= (double)c.R[3 * k + r] * (double)c.t[k];
    C[r] = v;
  }
}

int network_inputs(const gg_camera *src, int32_t K, const gg_camera *tgt,
                   const float *tsdf_depth, const float *rgb, const float *depth,
                   const float *alpha, float *out, void *stream) {
  const char *N = "network_inputs";
  if (int rc = check_sources(src, K, N)) return rc;
  if (int rc = check_camera(tgt, N)) return rc;
  if (!tsdf_depth || !rgb || !depth || !alpha || !out)
    return fail(GG_ERR_INVALID, "%s: NULL array argument", N);
  NetArgs a{};
  double Ct[3];
  centre_d(*tgt, Ct);
  const double Ki[9] = {1.0 / (double)tgt->fx, 0, -(double)tgt->cx / (double)tgt->fx,
                        0, 1.0 / (double)tgt->fy, -(double)tgt->cy / (double)tgt->fy, 0, 0, 1};
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) {
      double v = 0;
      for (int k = 0; k < 3; ++k) v += (double)tgt->R[3 * k + r] * Ki[3 * k + c];
      a.M.H[3 * r + c] = (float)v;
    }
    a.M.c[r] = (float)Ct[r];
  }
  for (int k = 0; k < K; ++k) {
    double Ck[3], d2 = 0, ax = 0;
    centre_d(src[k], Ck);
    for (int r = 0; r < 3; ++r) {
      a.Cs[k][r] = (float)Ck[r];
      d2 += (Ck[r] - Ct[r]) * (Ck[r] - Ct[r]);
      ax += (double)src[k].R[6 + r] * (double)tgt->R[6 + r];
    }
    a.dist[k] = (float)std::sqrt(d2);
    a.axd[k] = (float)ax;
  }
  a.K = K;
  a.W = tgt->width;
  a.H = tgt->height;
  a.tsdf_depth = tsdf_depth;
  a.rgb = rgb;
  a.depth = depth;
  a.alpha = alpha;
  a.out = out;
  return launch_network_inputs(a, (hipStream_t)stream);
}

int blend_views(int32_t K, int32_t width, int32_t height, const float *rgb, const float *depth,
                const float *alpha, const float *weights, const float *w_bg,
                const float *rgb_bg, float *out_rgb, float *out_depth, void *stream) {
  const char *N = "blend_views";
  if (K < 1 || K > GG_MAX_VIEWS)
    return fail(GG_ERR_INVALID, "%s: K = %d outside 1..%d", N, K, GG_MAX_VIEWS);
  if (width < 1 || height < 1 || width > 16384 || height > 16384)
    return fail(GG_ERR_INVALID, "%s: size %dx%d outside 1..16384", N, width, height);
  if (!rgb || !depth || !alpha || !weights || !w_bg || !rgb_bg || !out_rgb || !out_depth)
    return fail(GG_ERR_INVALID, "%s: NULL array argument", N);
  BlendArgs a{};
  a.K = K;
  a.W = width;
  a.H = height;
  a.rgb = rgb;
  a.depth = depth;
  a.alpha = alpha;
  a.w = weights;
  a.w_bg = w_bg;
  a.rgb_bg = rgb_bg;
  a.out_rgb = out_rgb;
  a.out_depth = out_depth;
  return launch_blend(a, (hipStream_t)stream);
}

int tsdf_extract_depth(const gg_camera *tgt, const gg_tsdf_params *prm, const float *F,
                       const float *W, float *out_depth, int32_t *out_bin,
                       const gg_volume_tuning *tuning, void *stream) {
  const char *N = "tsdf_extract_depth";
  if (int rc = check_camera(tgt, N)) return rc;
  if (int rc = check_tsdf(prm, N)) return rc;
  if (!F || !W || !out_depth || !out_bin) return fail(GG_ERR_INVALID, "%s: NULL argument", N);
  const uint32_t npix = (uint32_t)(tgt->width * tgt->height);
  VolumeShape vs;
  if (int rc = volume_shape(prm->num_bins, npix, vs, N, aligned(F, 32) && aligned(W, 32), tuning))
    return rc;
  const size_t va = 4 * (size_t)vs.V;
  if (!aligned(F, va) || !aligned(W, va))
    return fail(GG_ERR_INVALID, "%s: volumes must be %zu-byte aligned", N, va);
  ExtractArgs a{};
  a.F = F;
  a.W = W;
  a.out_depth = out_depth;
  a.out_bin = out_bin;
  a.npix = npix;
  a.D = prm->num_bins;
  a.cpp_div = make_fastdiv(vs.cpp);
  a.cpp = vs.cpp;
  a.ppb = vs.ppb;
  a.nblocks = vs.nblocks;
  a.z_near = prm->z_near;
  a.z_far = prm->z_far;
  return launch_extract(a, vs.V, vs.threads, (hipStream_t)stream);
}

int tsdf_extract_depth_backward(const gg_camera *tgt, const gg_tsdf_params *prm,
                                const float *F, const float *W, const int32_t *bin,
                                const float *g_depth, float *g_F2, void *stream) {
  const char *N = "tsdf_extract_depth_backward";
  if (int rc = check_camera(tgt, N)) return rc;
  if (int rc = check_tsdf(prm, N)) return rc;
  if (!F || !W || !bin || !g_depth || !g_F2) return fail(GG_ERR_INVALID, "%s: NULL argument", N);
  if (!aligned(g_F2, 8)) return fail(GG_ERR_INVALID, "%s: g_F2 must be 8-byte aligned", N);
  ExtractArgs a{};
  a.F = F;
  a.W = W;
  a.bin = bin;
  a.g_depth = g_depth;
  a.g_F2 = g_F2;
  a.npix = (uint32_t)(tgt->width * tgt->height);
  a.D = prm->num_bins;
  a.z_near = prm->z_near;
  a.z_far = prm->z_far;
  return launch_extract_backward(a, (hipStream_t)stream);
}

int tsdf_integrate_backward(const gg_camera *src, int32_t K, const float *depth,
                            const gg_camera *tgt, const gg_tsdf_params *prm, const float *F,
                            const float *W, const int32_t *bin, const float *g_F2,
                            float *g_depth_in, void *ws, size_t ws_bytes, void *stream) {
  const char *N = "tsdf_integrate_backward";
  if (int rc = check_sources(src, K, N)) return rc;
  if (int rc = check_camera(tgt, N)) return rc;
  if (int rc = check_tsdf(prm, N)) return rc;
  if (!depth || !F || !W || !bin || !g_F2 || !g_depth_in)
    return fail(GG_ERR_INVALID, "%s: NULL array argument", N);
  if (!aligned(g_F2, 8)) return fail(GG_ERR_INVALID, "%s: g_F2 must be 8-byte aligned", N);
  const int sw = src[0].width, sh = src[0].height, D = prm->num_bins;
  const TsdfLayout L = tsdf_layout(K, sw, sh, D, true);
  if (int rc = check_ws(ws, ws_bytes, L.total, N)) return rc;
  hipStream_t s = (hipStream_t)stream;
  char *w = (char *)ws;
  float2 *table = (float2 *)(w + L.table);
  float2 *bins = (float2 *)(w + L.bins);
  if (int rc = launch_bins(*prm, bins, s)) return rc;
  if (int rc = launch_conf(conf_args(depth, table, sw, sh, K, prm), s)) return rc;
  TsdfBackArgs a{};
  fill_views(src, K, tgt, a.views);
  const size_t ns = (size_t)sw * sh;
  a.table = table;
  a.bins = bins;
  a.depth = depth;
  a.F = F;
  a.W = W;
  a.bin = bin;
  a.g_F2 = g_F2;
  a.acc_D = (unsigned long long *)(w + L.acc);
  a.acc_w = a.acc_D + ns * K;
  a.maxbits = (uint32_t *)(a.acc_w + ns * K);
  a.gnu = (float *)(w + L.gnu);
  a.g_depth_in = g_depth_in;
  a.K = K;
  a.Ws = sw;
  a.Hs = sh;
  a.D = D;
  a.npix = (uint32_t)(tgt->width * tgt->height);
  a.ns = (uint32_t)ns;
  a.wt_div = make_fastdiv((uint32_t)tgt->width);
  a.radius = (prm->conf_window - 1) / 2;
  a.tw2 = prm->conf_tau * prm->conf_tau;
  a.n2 = (float)(prm->conf_window * prm->conf_window);
  a.scale = prm->conf_scale;
  return launch_tsdf_backward(a, s);
}

int gg_selftest_reciprocal(int32_t e_lo, int32_t e_hi, unsigned long long *mismatches,
                           void *stream) {
  if (e_lo < 1 || e_hi > 254 || e_lo > e_hi || !mismatches)
    return fail(GG_ERR_INVALID, "gg_selftest_reciprocal: need 1 <= e_lo <= e_hi <= 254");
  return launch_recip_selftest((uint32_t)e_lo, (uint32_t)(e_hi - e_lo + 1), mismatches,
                               (hipStream_t)stream);
}

int gg_fast_reciprocal(const float *in, float *out, int64_t n, void *stream) {
  if (!in || !out || n < 0) return fail(GG_ERR_INVALID, "gg_fast_reciprocal: bad arguments");
  if (n == 0) return GG_OK;
  return launch_fast_recip(in, out, n, (hipStream_t)stream);
}

int gg_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_tmu);
  g_timing = on != 0;
  return GG_OK;
}

int gg_timing_filter(const char *name) {
  std::lock_guard<std::mutex> lk(g_tmu);
  g_timing_only = name ? name : "";
  return GG_OK;
}

int gg_timing_reset(void) {
  std::lock_guard<std::mutex> lk(g_tmu);
  for (auto &t : g_launches) {
    g_event_pool.push_back(t.start);
    g_event_pool.push_back(t.stop);
  }
  g_launches.clear();
  return GG_OK;
}

int gg_timing_read(const char *name, double *total_ms, int64_t *launches) {
  std::lock_guard<std::mutex> lk(g_tmu);
  double sum = 0.0;
  int64_t n = 0;
  for (auto &t : g_launches) {
    if (name && !strstr(t.name.c_str(), name)) continue;
    if (int rc = check_hip(hipEventSynchronize(t.stop), "gg_timing_read")) return rc;
    float ms = 0.0f;
    if (int rc = check_hip(hipEventElapsedTime(&ms, t.start, t.stop), "gg_timing_read")) return rc;
    sum += ms;
    ++n;
  }
  if (total_ms) *total_ms = sum;
  if (launches) *launches = n;
  return GG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched path

struct gg_batch {
  BatchPlan P;
  std::vector<char> keep;  // nothing host-side is needed after creation
};

// Target pixels per fusion workgroup of a batch item by default (as the plain
// call's tuned launch shape takes them).
constexpr uint32_t kBatchPixelsPerBlock = 16;

// Bins per thread of a batch item (as for the plain call with that tuning).
static bool item_aligned32(const gg_batch_item &it) {
  return aligned(it.F, 32) && aligned(it.W, 32) &&
         (!it.F_prev || (aligned(it.F_prev, 32) && aligned(it.W_prev, 32)));
}

// Whether the item brings its own fusion launch shape.
static bool item_tuned(const gg_batch_item &it) {
  const gg_volume_tuning &t = it.volume;
  return t.pixels_per_block || t.pixels_per_row || t.bins_per_thread || t.band_width;
}

// Bins per thread of the item's fusion: as its own launch shape gives them
// (volume_shape), else as the plan's.
static int item_vec(const gg_batch_item &it, int vec) {
  return volume_v(it.tsdf.num_bins, item_aligned32(it),
                  item_tuned(it) ? it.volume.bins_per_thread : vec);
}

static int check_item(const gg_batch_item &it, int i, int vec) {
  char what[64];
  snprintf(what, sizeof what, "gg_batch_plan: item %d", i);
  if (int rc = check_sources(it.src, it.K, what)) return rc;
  if (int rc = check_camera(&it.tgt, what)) return rc;
  if (int rc = check_tsdf(&it.tsdf, what)) return rc;
  if (!it.depth || !it.F || !it.W) return fail(GG_ERR_INVALID, "%s: NULL array argument", what);
  if ((it.F_prev == nullptr) != (it.W_prev == nullptr))
    return fail(GG_ERR_INVALID, "%s: F_prev and W_prev go together", what);
  if ((it.out_depth == nullptr) != (it.out_bin == nullptr))
    return fail(GG_ERR_INVALID, "%s: out_depth and out_bin go together", what);
  if (it.rgb) {
    if (int rc = check_splat(&it.splat, what)) return rc;
    if (!it.win_idx || !it.sp_depth || !it.sp_rgb || !it.sp_alpha)
      return fail(GG_ERR_INVALID, "%s: splat outputs required with rgb", what);
  }
  if (int rc = check_tuning(&it.volume, what)) return rc;
  const int D = it.tsdf.num_bins;
  const int V = item_vec(it, vec);
  if (D / V > 1024) return fail(GG_ERR_UNSUPPORTED, "%s: D = %d too large", what, D);
  const size_t va = 4 * (size_t)V;
  if (!aligned(it.F, va) || !aligned(it.W, va) ||
      (it.F_prev && (!aligned(it.F_prev, va) || !aligned(it.W_prev, va))))
    return fail(GG_ERR_INVALID, "%s: volumes must be %zu-byte aligned", what, va);
  return GG_OK;
}

extern "C" int gg_batch_plan(const gg_batch_item *items, int32_t n, const gg_batch_tuning *tune,
                             gg_batch **out) {
  const char *N = "gg_batch_plan";
  if (!items || !out || n < 1) return fail(GG_ERR_INVALID, "%s: need items, n >= 1, out", N);
  if (n > 65535) return fail(GG_ERR_UNSUPPORTED, "%s: at most 65535 items", N);
  *out = nullptr;
  const int vec = tune ? tune->bins_per_thread : 0;
  if (vec != 0 && vec != 1 && vec != 2 && vec != 4 && vec != 8)
    return fail(GG_ERR_INVALID, "%s: bins_per_thread %d not in {0, 1, 2, 4, 8}", N, vec);
  for (int i = 0; i < n; ++i)
    if (int rc = check_item(items[i], i, vec)) return rc;
  const int ppb_t = tune ? tune->pixels_per_block : 0;
  const int per_cu = tune ? tune->blocks_per_cu : 0;
  const int branches = tune ? tune->branches : 0;
  if (ppb_t < 0 || ppb_t > 1024 || per_cu < 0 || per_cu > 64 || branches < 0 || branches > 2)
    return fail(GG_ERR_INVALID, "%s: pixels_per_block in 0..1024, blocks_per_cu in 0..64, "
                "branches in 0..2", N);
  int dev = 0, cus = 256;
  if (int rc = check_hip(hipGetDevice(&dev), N)) return rc;
  if (int rc = check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), N))
    return rc;

  // host descriptors, work lists and the device-memory layout
  std::vector<BatchItem> h(n);
  std::vector<WorkItem> conf, bin, raster;
  std::vector<IntegGroup> groups;              // fusion launches: (class, workgroup size)
  std::vector<std::vector<WorkItem>> integ;    // their work lists
  std::vector<uint32_t> splat_items;
  std::vector<VolumeShape> shapes(n);
  std::vector<SplatLayout> sl(n);
  size_t off = up256(sizeof(BatchItem) * n);
  std::vector<size_t> o_table(n), o_bins(n), o_splat(n);
  size_t count_words = 0;
  std::vector<size_t> o_count(n);
  for (int i = 0; i < n; ++i) {
    const gg_batch_item &it = items[i];
    const int sw = it.src[0].width, sh = it.src[0].height, K = it.K, D = it.tsdf.num_bins;
    const uint32_t npix = (uint32_t)(it.tgt.width * it.tgt.height);
    VolumeShape &vs = shapes[i];
    if (item_tuned(it)) {
      // the item's own launch shape, exactly as tsdf_integrate would take it
      char what[64];
      snprintf(what, sizeof what, "%s: item %d", N, i);
      if (int rc = volume_shape(D, npix, vs, what, item_aligned32(it), &it.volume)) return rc;
    } else {
      vs.V = item_vec(it, vec);
      vs.cpp = (uint32_t)(D / vs.V);
      // pixels per workgroup as the plain call's launch shape would give them
      vs.ppb = ppb_t > 0 ? (uint32_t)ppb_t : kBatchPixelsPerBlock;
      while (vs.ppb > 1 && vs.ppb * vs.cpp > 1024) --vs.ppb;
      vs.threads = vs.ppb * vs.cpp;
      vs.nblocks = (npix + vs.ppb - 1) / vs.ppb;
      vs.pw_shift = pick_pw_shift(vs.ppb, 16);
      vs.band_px = kDefaultBandPixels;
    }
    o_table[i] = off;
    off += up256(8 * table_view_records(sw, sh) * K);
    o_bins[i] = off;
    off += up256(8 * (size_t)D);
    if (it.rgb) {
      if ((size_t)K * sw * sh * splat_tiles_per_splat(it.splat.r_max_px) > 0xffffffffull)
        return fail(GG_ERR_UNSUPPORTED, "%s: item %d has too many source pixels", N, i);
      sl[i] = splat_layout(K, sw, sh, it.tgt.width, it.tgt.height, &it.splat);
      o_splat[i] = off;
      off += sl[i].total;
      o_count[i] = count_words;
      count_words += (size_t)K * sl[i].ntiles + 1;
    }
    const uint32_t ctx = (uint32_t)((sw + kConfTX - 1) / kConfTX),
                   cty = (uint32_t)((sh + kConfTY - 1) / kConfTY);
    if (ctx > 65535 || cty > 65535) return fail(GG_ERR_UNSUPPORTED, "%s: image too large", N);
    for (int k = 0; k < K; ++k)
      for (uint32_t y = 0; y < cty; ++y)
        for (uint32_t x = 0; x < ctx; ++x)
          conf.push_back(WorkItem{(uint16_t)i, (uint16_t)k, (uint16_t)x, (uint16_t)y});
    if (it.rgb) {
      splat_items.push_back((uint32_t)i);
      const uint32_t nb = splat_bin_blocks((uint32_t)sw, (uint32_t)sh);
      for (int k = 0; k < K; ++k) {
        for (uint32_t b = 0; b < nb; ++b)
          bin.push_back(WorkItem{(uint16_t)i, (uint16_t)k, (uint16_t)(b & 0xffff), (uint16_t)(b >> 16)});
        for (uint32_t t = 0; t < sl[i].ntiles; ++t)
          raster.push_back(WorkItem{(uint16_t)i, (uint16_t)k, (uint16_t)(t & 0xffff), (uint16_t)(t >> 16)});
      }
    }
    IntegrateArgs probe{};  // only for the view count class and the reciprocal's range
    make_integrate_args(probe, it.src, it.K, it.tgt, it.tsdf, vs, nullptr, nullptr, nullptr,
                        nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    // the volume stream through LDS where the plain call would take it too
    size_t stage_bytes = 0;
    if (vs.threads % 64 == 0 && vs.pw_shift == 4 && vs.cpp % 4 == 0) {
      if (vs.V == 8) stage_bytes = integrate_lds_bytes<8>(vs.threads, vs.ppb, D, true);
      if (vs.V == 4) stage_bytes = integrate_lds_bytes<4>(vs.threads, vs.ppb, D, true);
      if (stage_bytes > 65536) stage_bytes = 0;
    }
    const int mode = stage_bytes ? (it.F_prev ? 2 : 1) : 0;
    const int cls = integ_class(vs.V, K, probe.exact_only != 0, mode);
    size_t gi = 0;
    while (gi < groups.size() && !(groups[gi].cls == cls && groups[gi].threads == vs.threads)) ++gi;
    if (gi == groups.size()) {
      IntegGroup g;
      g.cls = cls;
      g.threads = vs.threads;
      groups.push_back(g);
      integ.emplace_back();
    }
    groups[gi].shm = std::max(groups[gi].shm,
                              stage_bytes ? stage_bytes : integrate_lds_head(vs.threads, vs.ppb));
    // the item's tiles in the plain launch's visiting order (bands)
    for (uint32_t s = 0; s < vs.nblocks; ++s) {
      const uint32_t t = band_tile(probe, s);
      integ[gi].push_back(WorkItem{(uint16_t)i, 0, (uint16_t)(t & 0xffff), (uint16_t)(t >> 16)});
    }
  }
  const size_t o_counts = off;
  off += up256(4 * (count_words + kBatchCounters));
  auto put = [&](size_t bytes) { const size_t o = off; off += up256(bytes ? bytes : 1); return o; };
  const size_t o_conf = put(sizeof(WorkItem) * conf.size()), o_bin = put(sizeof(WorkItem) * bin.size()),
               o_raster = put(sizeof(WorkItem) * raster.size());
  std::vector<size_t> o_integ(groups.size());
  for (size_t g = 0; g < groups.size(); ++g) o_integ[g] = put(sizeof(WorkItem) * integ[g].size());
  const size_t o_sitems = put(4 * splat_items.size());

  gg_batch *b = new gg_batch();
  BatchPlan &P = b->P;
  P.n_items = n;
  P.cus = cus;
  P.blocks_per_cu = per_cu;
  P.branches = branches ? branches : 2;
  P.dev_bytes = off;
  if (int rc = check_hip(hipMalloc(&P.dev, off), N)) {
    delete b;
    return rc;
  }
  char *dv = (char *)P.dev;
  for (int i = 0; i < n; ++i) {
    const gg_batch_item &it = items[i];
    BatchItem &d = h[i];
    const int sw = it.src[0].width, sh = it.src[0].height;
    float2 *table = (float2 *)(dv + o_table[i]);
    float2 *bins = (float2 *)(dv + o_bins[i]);
    d.conf = conf_args(it.depth, table, sw, sh, it.K, &it.tsdf);
    make_integrate_args(d.integ, it.src, it.K, it.tgt, it.tsdf, shapes[i], table, bins,
                        it.temporal_mask, it.F_prev, it.W_prev, it.F, it.W, it.out_depth,
                        it.out_bin);
    if (it.rgb) {
      make_splat_args(d.splat, it.src, it.K, it.depth, it.rgb, it.tgt, it.splat, sl[i],
                      dv + o_splat[i]);
      d.splat.tile_count = (uint32_t *)(dv + o_counts) + o_count[i];
      d.splat.win_idx = it.win_idx;
      d.splat.out_depth = it.sp_depth;
      d.splat.out_rgb = it.sp_rgb;
      d.splat.out_alpha = it.sp_alpha;
      d.splat.out_tape = it.sp_tape;
    }
    d.bins = bins;
    d.D = it.tsdf.num_bins;
    d.z_near = it.tsdf.z_near;
    d.z_far = it.tsdf.z_far;
    d.trunc = it.tsdf.trunc;
    d.trunc_in_bins = it.tsdf.trunc_in_bins;
  }
  P.d_items = (BatchItem *)dv;
  P.d_conf = (WorkItem *)(dv + o_conf);
  P.n_conf = (uint32_t)conf.size();
  P.d_bin = (WorkItem *)(dv + o_bin);
  P.n_bin = (uint32_t)bin.size();
  P.d_raster = (WorkItem *)(dv + o_raster);
  P.n_raster = (uint32_t)raster.size();
  P.integ = groups;
  for (size_t g = 0; g < groups.size(); ++g) {
    P.integ[g].list = (WorkItem *)(dv + o_integ[g]);
    P.integ[g].n = (uint32_t)integ[g].size();
  }
  P.d_splat_items = (uint32_t *)(dv + o_sitems);
  P.n_splat_items = (uint32_t)splat_items.size();
  P.zero_ptr = (uint32_t *)(dv + o_counts);
  P.zero_words = count_words + kBatchCounters;
  P.d_ctr = P.zero_ptr + count_words;
  int rc = GG_OK;
  auto cp = [&](size_t o, const void *src, size_t bytes) {
    if (rc == GG_OK && bytes) rc = check_hip(hipMemcpy(dv + o, src, bytes, hipMemcpyHostToDevice), N);
  };
  cp(0, h.data(), sizeof(BatchItem) * n);
  cp(o_conf, conf.data(), sizeof(WorkItem) * conf.size());
  cp(o_bin, bin.data(), sizeof(WorkItem) * bin.size());
  cp(o_raster, raster.data(), sizeof(WorkItem) * raster.size());
  for (size_t g = 0; g < groups.size(); ++g)
    cp(o_integ[g], integ[g].data(), sizeof(WorkItem) * integ[g].size());
  if (rc == GG_OK) rc = batch_occupancy(P);
  cp(o_sitems, splat_items.data(), 4 * splat_items.size());
  // capture every phase into one graph
  hipStream_t cs = nullptr, side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  if (rc == GG_OK) rc = check_hip(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), N);
  if (rc == GG_OK) rc = check_hip(hipStreamCreateWithFlags(&side, hipStreamNonBlocking), N);
  if (rc == GG_OK) rc = check_hip(hipEventCreateWithFlags(&fork, hipEventDisableTiming), N);
  if (rc == GG_OK) rc = check_hip(hipEventCreateWithFlags(&join, hipEventDisableTiming), N);
  if (rc == GG_OK) rc = check_hip(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), N);
  if (rc == GG_OK) {
    const int rr = batch_record(P, cs, side, fork, join);
    const int re = check_hip(hipStreamEndCapture(cs, &P.graph), N);
    rc = rr ? rr : re;
  }
  if (rc == GG_OK) rc = check_hip(hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0), N);
  if (fork) (void)hipEventDestroy(fork);
  if (join) (void)hipEventDestroy(join);
  if (side) (void)hipStreamDestroy(side);
  if (cs) (void)hipStreamDestroy(cs);
  if (rc != GG_OK) {
    gg_batch_free(b);
    return rc;
  }
  *out = b;
  return GG_OK;
}

extern "C" int gg_batch_launch(gg_batch *plan, void *stream) {
  if (!plan || !plan->P.exec) return fail(GG_ERR_INVALID, "gg_batch_launch: no plan");
  KernelTimer t("batch_graph", (hipStream_t)stream);
  return check_hip(hipGraphLaunch(plan->P.exec, (hipStream_t)stream), "gg_batch_launch");
}

extern "C" size_t gg_batch_device_bytes(const gg_batch *plan) { return plan ? plan->P.dev_bytes : 0; }

extern "C" int gg_batch_free(gg_batch *plan) {
  if (!plan) return GG_OK;
  BatchPlan &P = plan->P;
  if (P.exec) (void)hipGraphExecDestroy(P.exec);
  if (P.graph) (void)hipGraphDestroy(P.graph);
  if (P.dev) (void)hipFree(P.dev);
  delete plan;
  return GG_OK;
}
