// Device functions of the fusion (Suppl. A.1, A.2) shared by the plain
// kernels (tsdf.hip) and the batched persistent kernels (batch.hip): one
// definition, so both paths perform the identical operation sequence.
#pragma once

#include <climits>

#include "ggeom_internal.h"

namespace gg {

// depth bins: z_d = 1 / (1/z_near - d du)
__device__ __forceinline__ float bin_depth(int d, int D, float z_near, float z_far) {
  const float un = 1.0f / z_near;
  const float uf = 1.0f / z_far;
  const float du = (un - uf) / (float)(D - 1);
  const float u = un - (float)d * du;
  return 1.0f / u;
}

// ---------------------------------------------------------------------------
// fusion weight (Suppl. A.1)

constexpr int kConfTX = 32, kConfTY = 8, kMaxR = (GG_MAX_WINDOW - 1) / 2;
constexpr int kConfLW = kConfTX + 2 * kMaxR, kConfLH = kConfTY + 2 * kMaxR;

// nu of Suppl. A.1 at pixel (i, j) with centre depth dq, reading the staged
// tile (origin at image (i0 - r, j0 - r)); row-major over the window.
__device__ __forceinline__ float window_nu(const float *tile, int li, int lj, int i, int j,
                                           float dq, const ConfArgs &a) {
  const int r = a.radius;
  float nu = 0.0f;
  for (int dy = -r; dy <= r; ++dy) {
    const int jj = j + dy;
    if (jj < 0 || jj >= a.Hs) continue;
    for (int dx = -r; dx <= r; ++dx) {
      const int ii = i + dx;
      if (ii < 0 || ii >= a.Ws) continue;
      const float dn = tile[(lj + dy) * kConfLW + (li + dx)];
      float term;
      if (depth_ok(dn)) {
        const float dd = dq - dn;
        term = fminf(dd * dd, a.tw2);
      } else {
        term = a.tw2;
      }
      nu = nu + term;
    }
  }
  return nu;
}

// nu for a pixel whose whole window lies inside the image (radius R known
// at compile time): the same terms in the same row-major order, with holes
// staged as NaN -- d_q - NaN is NaN and fminf(NaN, tau^2) = tau^2, which is
// exactly a hole's term -- so no test is needed per neighbour.
template <int R>
__device__ __forceinline__ float window_nu_interior(const float *tile, int li, int lj, float dq,
                                                    float tw2) {
  const float *w = tile + (lj - R) * kConfLW + (li - R);
  float nu = 0.0f;
#pragma unroll
  for (int dy = 0; dy <= 2 * R; ++dy)
#pragma unroll
    for (int dx = 0; dx <= 2 * R; ++dx) {
      const float dd = dq - w[dy * kConfLW + dx];
      nu = nu + fminf(dd * dd, tw2);
    }
  return nu;
}

__device__ __forceinline__ float window_nu_fast(const float *tile, int li, int lj, float dq,
                                                const ConfArgs &a) {
  switch (a.radius) {
    case 0: return window_nu_interior<0>(tile, li, lj, dq, a.tw2);
    case 1: return window_nu_interior<1>(tile, li, lj, dq, a.tw2);
    case 2: return window_nu_interior<2>(tile, li, lj, dq, a.tw2);
    case 3: return window_nu_interior<3>(tile, li, lj, dq, a.tw2);
    case 4: return window_nu_interior<4>(tile, li, lj, dq, a.tw2);
    case 5: return window_nu_interior<5>(tile, li, lj, dq, a.tw2);
    case 6: return window_nu_interior<6>(tile, li, lj, dq, a.tw2);
    default: return window_nu_interior<kMaxR>(tile, li, lj, dq, a.tw2);
  }
}

// The window's tile staged in LDS; pixels without a usable depth are staged
// as NaN (both window forms treat NaN as a hole), pixels outside the image
// as 0 (only the bounds-checked form can reach them, and it skips them).
// A staged row is at most 46 floats: one wavefront's lanes take its columns
// and the workgroup's wavefronts (blockDim a multiple of 64) step down the
// rows, so no lane divides by the row width.  kDepth: the source is a depth
// map, whose holes are staged as NaN; otherwise values are staged as read.
template <bool kDepth>
__device__ __forceinline__ void stage_rows(float *tile, const float *src, int i0, int j0,
                                           const ConfArgs &a) {
  static_assert(kConfTX + 2 * kMaxR <= 64, "a staged row fits one wavefront");
  const int r = a.radius;
  const int tw = kConfTX + 2 * r, th = kConfTY + 2 * r;
  const int lx = (int)(threadIdx.x & 63u), waves = (int)(blockDim.x >> 6);
  const int gi = i0 - r + lx;
  const bool in_col = gi >= 0 && gi < a.Ws;
  // stored at (ly + kMaxR - r, lx + kMaxR - r) so that window offsets are
  // relative to the fixed centre origin
  float *dst = tile + (kMaxR - r) * kConfLW + (lx + kMaxR - r);
  if (lx < tw) {
    for (int ly = (int)(threadIdx.x >> 6); ly < th; ly += waves) {
      const int gj = j0 - r + ly;
      float v = 0.0f;
      if (in_col && gj >= 0 && gj < a.Hs) {
        v = gmem(src)[(size_t)gj * a.Ws + gi];
        if (kDepth && !depth_ok(v)) v = __builtin_nanf("");
      }
      dst[ly * kConfLW] = v;
    }
  }
}

__device__ __forceinline__ void stage_tile(float *tile, const float *dk, int i0, int j0,
                                           const ConfArgs &a) {
  stage_rows<true>(tile, dk, i0, j0, a);
}

// One 32 x 8 tile (bx, by) of view k; tile: LDS of kConfLH x kConfLW floats.
__device__ __forceinline__ void conf_tile(const ConfArgs &a, int k, int bx, int by, float *tile) {
  const int i0 = bx * kConfTX, j0 = by * kConfTY;
  const float *dk = a.depth + (size_t)k * a.Ws * a.Hs;
  stage_tile(tile, dk, i0, j0, a);
  __syncthreads();
  const int lx = threadIdx.x & (kConfTX - 1), ly = threadIdx.x / kConfTX;
  const int i = i0 + lx, j = j0 + ly;
  // every window of the tile inside the image: the unchecked form
  const bool interior = i0 >= a.radius && j0 >= a.radius &&
                        i0 + kConfTX + a.radius <= a.Ws && j0 + kConfTY + a.radius <= a.Hs;
  if (ly < kConfTY && i < a.Ws && j < a.Hs) {
    const int li = lx + kMaxR, lj = ly + kMaxR;
    const float dq = tile[lj * kConfLW + li];
    float2 rec = make_float2(-INFINITY, 0.0f);
    if (depth_ok(dq)) {
      const float nu = interior ? window_nu_fast(tile, li, lj, dq, a)
                                : window_nu(tile, li, lj, i, j, dq, a);
      const float om = (nu == 0.0f) ? 1.0f : fminf(a.scale / sqrtf(nu / a.n2), 1.0f);
      rec = make_float2(dq, om);
    }
    float2 *row = a.table + (size_t)k * table_view_records(a.Ws, a.Hs) + (size_t)j * table_pitch(a.Ws);
    gstore2(row + i, rec);
    if (i == a.Ws - 1) gstore2(row + a.Ws, make_float2(0.0f, 0.0f));  // the row's closing record
  }
  __syncthreads();  // the tile may be restaged by the caller's next iteration
}

// Fusion tile at position s of the launch's visiting order.  Far source
// views see a target ray as a long epipolar segment spanning many source
// rows, so one target row gathers from a large part of each view table;
// the rows below it gather from nearly the same lines.  Visiting vertical
// bands of band_B tiles across, each row by row from the top, keeps the
// lines that the tiles in flight share within cache, where row-major order
// would have walked the whole target width before returning to them.
// Every full band comes before the narrower last one (band_T = 0:
// row-major order).
__host__ __device__ __forceinline__ uint32_t band_tile(const IntegrateArgs &a, uint32_t s) {
  if (a.band_T == 0) return s;
  const uint32_t span = a.band_B * a.band_H;  // tiles of a full band
  const uint32_t b = s / span;
  const uint32_t b0 = b * a.band_B;
  const uint32_t w = a.band_T - b0 < a.band_B ? a.band_T - b0 : a.band_B;
  const uint32_t rem = s - b * span;
  const uint32_t r = rem / w;
  return r * a.band_T + b0 + (rem - r * w);
}

// ---------------------------------------------------------------------------
// Volume stream access of V consecutive floats (V = 8, 4, 2, 1).  The volume
// is read and written once per launch: its accesses are non-temporal, so
// that they pass through the caches without evicting the view-table lines
// that the gathers of neighbouring tiles reuse.

template <int V>
__device__ __forceinline__ void loadv(const float *p, float (&o)[V]) {
  if constexpr (V == 8) {
    const gg_v4f a = __builtin_nontemporal_load((const GG_GLOBAL gg_v4f *)p),
                 b = __builtin_nontemporal_load((const GG_GLOBAL gg_v4f *)(p + 4));
    o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
    o[4] = b.x; o[5] = b.y; o[6] = b.z; o[7] = b.w;
  } else if constexpr (V == 4) {
    const gg_v4f v = __builtin_nontemporal_load((const GG_GLOBAL gg_v4f *)p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  } else if constexpr (V == 2) {
    const gg_v2f v = __builtin_nontemporal_load((const GG_GLOBAL gg_v2f *)p);
    o[0] = v.x; o[1] = v.y;
  } else {
    o[0] = __builtin_nontemporal_load(gmem(p));
  }
}

template <int V>
__device__ __forceinline__ void storev(float *p, const float (&o)[V]) {
  if constexpr (V == 8) {
    __builtin_nontemporal_store((gg_v4f){o[0], o[1], o[2], o[3]}, (GG_GLOBAL gg_v4f *)p);
    __builtin_nontemporal_store((gg_v4f){o[4], o[5], o[6], o[7]}, (GG_GLOBAL gg_v4f *)(p + 4));
  } else if constexpr (V == 4) {
    __builtin_nontemporal_store((gg_v4f){o[0], o[1], o[2], o[3]}, (GG_GLOBAL gg_v4f *)p);
  } else if constexpr (V == 2) {
    __builtin_nontemporal_store((gg_v2f){o[0], o[1]}, (GG_GLOBAL gg_v2f *)p);
  } else {
    __builtin_nontemporal_store(o[0], gmem(p));
  }
}

// First crossing inside this thread's V bins, given the next chunk's first
// bin (F, W); INT_MAX if none.
template <int V>
__device__ __forceinline__ int local_crossing(const float (&F)[V], const float (&W)[V], float nF,
                                              float nW, int d0, int D) {
  int cand = INT_MAX;
#pragma unroll
  for (int v = V - 1; v >= 0; --v) {
    const float f1 = (v + 1 < V) ? F[(v + 1) % V] : nF;
    const float w1 = (v + 1 < V) ? W[(v + 1) % V] : nW;
    if (d0 + v + 1 < D && W[v] > 0.0f && w1 > 0.0f && F[v] > 0.0f && f1 <= 0.0f) cand = d0 + v;
  }
  return cand;
}

// Extraction across the workgroup: each thread holds V bins of one pixel;
// the chunk's first bin is exchanged through LDS, the smallest crossing per
// pixel is an LDS atomic minimum (order-free), and the owning thread
// interpolates.  zf(d) returns z_d for the owning thread.
template <int V, typename ZF>
__device__ __forceinline__ void extract_block(const float (&F)[V], const float (&W)[V],
                                              bool lane, bool active, uint32_t pix, uint32_t lp,
                                              uint32_t chunk, uint32_t cpp, uint32_t next_off,
                                              int d0, int D,
                                              float *sF, float *sW, int *sBest,
                                              float *out_depth, int32_t *out_bin, ZF zf) {
  // lane: this thread maps to a chunk of one of the workgroup's pixels
  // (threads past ppb * cpp idle but take part in the barriers).
  const uint32_t t = threadIdx.x;
  if (lane) {
    sF[t] = F[0];
    sW[t] = W[0];
    if (chunk == 0) sBest[lp] = INT_MAX;
  }
  __syncthreads();
  const bool has_next = lane && chunk + 1 < cpp;
  const float nF = has_next ? sF[t + next_off] : 0.0f;
  const float nW = has_next ? sW[t + next_off] : 0.0f;
  if (active) {
    const int cand = local_crossing<V>(F, W, nF, nW, d0, D);
    if (cand != INT_MAX) atomicMin(&sBest[lp], cand);
  }
  __syncthreads();
  if (active) {
    const int best = sBest[lp];
    if (best == INT_MAX) {
      if (chunk == 0) {
        gmem(out_depth)[pix] = 0.0f;
        gmem(out_bin)[pix] = -1;
      }
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) {
        if (best == d0 + v) {
          const float f0 = F[v];
          const float f1 = (v + 1 < V) ? F[(v + 1) % V] : nF;
          const float za = zf(best), zb = zf(best + 1);
          const float frac = f0 / (f0 - f1);
          gmem(out_depth)[pix] = za + (zb - za) * frac;
          gmem(out_bin)[pix] = best;
        }
      }
    }
  }
  __syncthreads();  // LDS reused by the caller's next tile
}

// ---------------------------------------------------------------------------
// fused integrate + extraction.  Workgroup = ppb whole pixels; thread = V
// consecutive bins of one pixel (the volume is D-innermost, so a wavefront
// reads and writes one contiguous span of F and W: fully coalesced).
//
// Per voxel and view the work is branch-free: the sample pixel of every
// (view, bin) pair the thread owns is computed first, then all their view-
// table records (8 bytes: depth, weight) are gathered at once, then they are
// accumulated in view order.  The gathers of a thread are independent, so
// their L2 latencies overlap.

// How a view's samples of the thread's bins find their pixels.  The pixel
// of the point (X0, X1, Z) (homogeneous pixel coordinates) is
// (floor(X0 / Z), floor(X1 / Z)) with the quotient evaluated as X * (1 / Z),
// none if Z <= 0 or outside the image.  1 / Z is correctly rounded in every
// mode: by recip_rn where it is exact (0 < Z < 2^100; the upper end is
// checked on the host), by IEEE division where a depth may lie in
// (0, 2^-100].
enum : int {
  kInFront = 0,  // every sample has Z > 2^-100: no depth test per sample
  kChecked = 1,  // no sample has Z in (0, 2^-100]: recip_rn, Z tested
  kDivide = 2,   // IEEE division
};

// Byte offset of the sample's view-table record within the view's table
// (rows of `pitch` records), kOutOfRange if none.
template <int kMode>
__device__ __forceinline__ uint32_t sample_offset(float X0, float X1, float Z, uint32_t Ws,
                                                  uint32_t Hs, uint32_t pitch, float fWs,
                                                  float fHs) {
  if constexpr (kMode == kDivide) {
    uint32_t off = kOutOfRange;
    if (Z > 0.0f) {
      const float iv = 1.0f / Z;
      const float u = X0 * iv, w = X1 * iv;
      if (u >= 0.0f && u < fWs && w >= 0.0f && w < fHs)
        off = ((uint32_t)w * pitch + (uint32_t)u) << 3;
    }
    return off;
  } else {
    const float inv = recip_rn(Z);
    const uint32_t i = (uint32_t)floor_i32(X0 * inv), j = (uint32_t)floor_i32(X1 * inv);
    bool ok = i < Ws && j < Hs;
    if constexpr (kMode == kChecked) ok = ok && (Z > kRecipLo);
    // sizes are at most 16384 (host check): pitch * 8 < 2^24, the offset < 2^31
    return ok ? __umul24(j, pitch << 3) + (i << 3) : kOutOfRange;
  }
}

// The sample's record as (row, byte offset in the row) for a structured
// load: a row outside [0, Hs) -- a negative floor is a huge unsigned row --
// is dropped by the load's range check, and a column outside [0, Ws) is
// clamped to Ws, the row's closing record (0, 0).  Either way the sample
// reads (0, 0), exactly what the range-checked raw load gives it, with no
// test of its own.
template <int kMode>
__device__ __forceinline__ void sample_row(float X0, float X1, float Z, uint32_t Ws, float fWs,
                                           float fHs, uint32_t &row, uint32_t &off) {
  if constexpr (kMode == kDivide) {
    row = 0xffffffffu;
    off = 0u;
    if (Z > 0.0f) {
      const float iv = 1.0f / Z;
      const float u = X0 * iv, w = X1 * iv;
      if (u >= 0.0f && u < fWs && w >= 0.0f && w < fHs) {
        row = (uint32_t)w;
        off = (uint32_t)u << 3;
      }
    }
  } else {
    const float inv = recip_rn(Z);
    const uint32_t i = (uint32_t)floor_i32(X0 * inv), j = (uint32_t)floor_i32(X1 * inv);
    row = j;
    if constexpr (kMode == kChecked) row = (Z > kRecipLo) ? j : 0xffffffffu;
    off = min(i, Ws) << 3;
  }
}

// The view's depth over the thread's bins, fma(z, h2, c2), is monotone in z
// and the bin depths increase with the bin index, so the end bins bound it.
template <int V>
__device__ __forceinline__ void view_depth_range(const Proj &P, float px, float py,
                                                 const float (&z)[V], float &lo, float &hi) {
  float h0, h1, h2;
  ray_of(P, px, py, h0, h1, h2);
  const float Za = fmaf(z[0], h2, P.c[2]), Zb = fmaf(z[V - 1], h2, P.c[2]);
  lo = fminf(Za, Zb);
  hi = fmaxf(Za, Zb);
}

// Wave-uniform mode for one view.
template <int V>
__device__ __forceinline__ int view_mode(const Proj &P, float px, float py, const float (&z)[V]) {
  float lo, hi;
  view_depth_range<V>(P, px, py, z, lo, hi);
  if (__all(lo > kRecipLo)) return kInFront;
  // a lane whose bins straddle the camera plane may have a depth in (0, 2^-100]
  return __any(hi > 0.0f && !(lo > kRecipLo)) ? kDivide : kChecked;
}

// One view's samples of the V voxels: depths and table gathers (left in
// flight for the caller).  A sample with no pixel reads the record (0, 0)
// from the range-checked load, whose zero weight drops it.
// kRows: the view's table read with structured loads (rows of at most 2047
// records), else with range-checked raw loads.
template <int V, int kMode, bool kRows>
__device__ __forceinline__ void view_samples(const IntegrateArgs &a, int k, float px, float py,
                                             const float (&z)[V], float (&Z)[V],
                                             float2 (&e)[V]) {
  const Proj &P = a.views[k];
  float h0, h1, h2;
  ray_of(P, px, py, h0, h1, h2);
  const uint32_t pitch = table_pitch(a.Ws);
  const float2 *view = a.table + (size_t)k * table_view_records(a.Ws, a.Hs);
  const float fWs = (float)a.Ws, fHs = (float)a.Hs;
  if constexpr (kRows) {
    const __amdgpu_buffer_rsrc_t tab = rows_of(view, pitch * 8u, (uint32_t)a.Hs);
    uint32_t row[V], off[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const float X0 = fmaf(z[v], h0, P.c[0]);
      const float X1 = fmaf(z[v], h1, P.c[1]);
      Z[v] = fmaf(z[v], h2, P.c[2]);
      sample_row<kMode>(X0, X1, Z[v], (uint32_t)a.Ws, fWs, fHs, row[v], off[v]);
    }
#pragma unroll
    for (int v = 0; v < V; ++v) e[v] = rload2(tab, row[v], off[v]);
  } else {
    const __amdgpu_buffer_rsrc_t tab =
        buffer_of(view, (uint32_t)(table_view_records(a.Ws, a.Hs) * 8u));
    uint32_t off[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const float X0 = fmaf(z[v], h0, P.c[0]);
      const float X1 = fmaf(z[v], h1, P.c[1]);
      Z[v] = fmaf(z[v], h2, P.c[2]);
      off[v] = sample_offset<kMode>(X0, X1, Z[v], (uint32_t)a.Ws, (uint32_t)a.Hs, pitch, fWs,
                                    fHs);
    }
#pragma unroll
    for (int v = 0; v < V; ++v) e[v] = bload2(tab, off[v]);
  }
}

// Accumulate one view's samples: s = D_k - z_k, occlusion cut (s < -tau:
// dropped), clamp min(s, tau).  Branch-free: the clamp to [-tau, tau] equals
// min(s, tau) for every kept sample and stays finite for dropped ones (a
// hole's depth is -inf), which add (+0) * c and +0 and so leave S and Wo
// bitwise unchanged (both start at +0 and never become -0).
template <int V>
__device__ __forceinline__ void view_accumulate(const float (&Z)[V], const float2 (&e)[V],
                                                const float (&tau)[V], float (&S)[V],
                                                float (&Wo)[V]) {
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const float s = e[v].x - Z[v];
    const float c = __builtin_amdgcn_fmed3f(s, -tau[v], tau[v]);
    const float w = (s < -tau[v]) ? 0.0f : e[v].y;
    S[v] = fmaf(w, c, S[v]);
    Wo[v] = Wo[v] + w;
  }
}

// G views k0 .. k0+G-1: every gather of the group is issued, then
// after_issue() (the caller's own loads, so that in-order load completion
// lets the gathers be consumed while those are still in flight), then the
// samples are accumulated in view order.
template <int V, int G, int kMode, bool kRows, typename AfterIssue>
__device__ __forceinline__ void fuse_group(const IntegrateArgs &a, int k0, float px, float py,
                                           const float (&z)[V], const float (&tau)[V],
                                           float (&S)[V], float (&Wo)[V],
                                           AfterIssue &&after_issue) {
  float Z[G][V];
  float2 e[G][V];
#pragma unroll
  for (int g = 0; g < G; ++g) view_samples<V, kMode, kRows>(a, k0 + g, px, py, z, Z[g], e[g]);
  after_issue();
#pragma unroll
  for (int g = 0; g < G; ++g) view_accumulate<V>(Z[g], e[g], tau, S, Wo);
}

// Views per group for a compile-time view count: at most 16 samples (and
// 4 views) in flight, the group size dividing KC.
template <int KC, int V>
constexpr int view_group() {
  constexpr int m = (16 / V < 4) ? (16 / V < 1 ? 1 : 16 / V) : 4;
  int g = KC < m ? KC : m;
  while (g > 1 && KC % g != 0) --g;
  return g;
}

// View count KC > 0 known at compile time, every sample in front of its
// view: views in unrolled groups, the caller's loads issued after the first
// group's gathers.
template <int V, int KC, bool kRows, typename AfterIssue>
__device__ __forceinline__ void fuse_views_in_front(const IntegrateArgs &a, float px, float py,
                                                    const float (&z)[V], const float (&tau)[V],
                                                    float (&S)[V], float (&Wo)[V],
                                                    AfterIssue &&after_issue) {
  constexpr int G = view_group<KC, V>();
  fuse_group<V, G, kInFront, kRows>(a, 0, px, py, z, tau, S, Wo, after_issue);
#pragma unroll
  for (int k0 = G; k0 < KC; k0 += G)
    fuse_group<V, G, kInFront, kRows>(a, k0, px, py, z, tau, S, Wo, [] {});
}

// KC > 0 and every sample of the wave in front of every view (one
// wave-uniform test): the unrolled straight-line variant.  Otherwise (and
// for a runtime view count, KC == 0, or under kExact) one view at a time in
// a loop, each in its own wave-uniform mode, the caller's loads first.
//
// kRows: every view table read with structured loads (rows_of / rload2),
// which replace the per-sample bounds tests with the row index's range check
// and a clamp of the column onto the row's closing record: three vector
// instructions fewer per sample, for two registers per address in flight and
// more work at the texture address unit (the host picks it where that pays).
template <int V, int KC, bool kExact, bool kRows, typename AfterIssue>
__device__ __forceinline__ void fuse_voxels(const IntegrateArgs &a, float px, float py,
                                            const float (&z)[V], const float (&tau)[V],
                                            float (&S)[V], float (&Wo)[V],
                                            AfterIssue &&after_issue) {
  if constexpr (KC > 0 && !kExact) {
    bool front = true;
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      float lo, hi;
      view_depth_range<V>(a.views[k], px, py, z, lo, hi);
      front = front && lo > kRecipLo;
    }
    if (__builtin_expect(__all(front), 1)) {
      fuse_views_in_front<V, KC, kRows>(a, px, py, z, tau, S, Wo, after_issue);
      return;
    }
  }
  after_issue();
  const int K = KC > 0 ? KC : a.K;
#pragma nounroll
  for (int k = 0; k < K; ++k) {
    const int mode = kExact ? kDivide : view_mode<V>(a.views[k], px, py, z);
    if (mode == kInFront)
      fuse_group<V, 1, kInFront, kRows>(a, k, px, py, z, tau, S, Wo, [] {});
    else if (mode == kChecked)
      fuse_group<V, 1, kChecked, kRows>(a, k, px, py, z, tau, S, Wo, [] {});
    else
      fuse_group<V, 1, kDivide, kRows>(a, k, px, py, z, tau, S, Wo, [] {});
  }
}


// ---------------------------------------------------------------------------
// The volume stream through LDS.  In the compute layout a wavefront holds 16
// neighbouring pixels x 4 consecutive chunks (lane = chunk * 16 + pixel), so
// a lane quad of a direct F / W access touches four pixels, i.e. four cache
// lines, and the vector-memory unit takes one pass per line.  Per pixel the
// wavefront's 4 chunks are one contiguous run of 4V floats, so instead the
// loads and stores move each run with lane quads inside one 64-byte piece
// (one line per quad), and the wavefront's own LDS slice exchanges the data
// with the compute layout.  Needs V = 4 or 8, 16 pixels per wavefront row and
// a chunk count per pixel that is a multiple of 4 (the launcher checks).

template <int V>
struct VolStage {
  static constexpr int kRowF4 = V + 1;              // float4 per pixel row (+1 pad: no bank conflicts)
  static constexpr int kArray = 16 * kRowF4 * 4;    // floats per array per wavefront
  static constexpr int kWave = 2 * kArray;          // F and W
  static constexpr int kIssues = V / 4;             // float4 per lane per array
};

// Orders one wavefront's LDS writes before its following LDS reads of other
// lanes' data (LDS executes a wavefront's instructions in order; this keeps
// the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void lds_put4(float *p, gg_v4f v) { *(gg_v4f *)p = v; }
__device__ __forceinline__ gg_v4f lds_get4(const float *p) { return *(const gg_v4f *)p; }

// Stream position of issue h of this lane: pixel row p (0..15) of the
// wavefront and float4 j (0..V-1) of that pixel's run.
template <int V>
__device__ __forceinline__ void stage_pos(int h, uint32_t lane, uint32_t &p, uint32_t &j) {
  const uint32_t f = (uint32_t)h * 64u + lane;
  p = f / V;
  j = f % V;
}

// Loads of the stream, unconditional (a pixel past the image reads the last
// pixel's run, which nothing stores back): no branch separates them from the
// view gathers, so the compiler's in-order wait counts need not assume that
// these long-latency loads precede every gather.  Non-temporal, as loadv.
template <int V>
__device__ __forceinline__ void stage_load(const float *src, uint32_t pix0, uint32_t npix,
                                           size_t run0, int D, gg_v4f (&r)[VolStage<V>::kIssues]) {
  const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
  for (int h = 0; h < VolStage<V>::kIssues; ++h) {
    uint32_t p, j;
    stage_pos<V>(h, lane, p, j);
    const uint32_t pp = min(pix0 + p, npix - 1u);
    r[h] = __builtin_nontemporal_load((const GG_GLOBAL gg_v4f *)(src + (size_t)pp * D + run0 + 4u * j));
  }
}

template <int V>
__device__ __forceinline__ void stage_put_stream(float *st, const gg_v4f (&r)[VolStage<V>::kIssues]) {
  const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
  for (int h = 0; h < VolStage<V>::kIssues; ++h) {
    uint32_t p, j;
    stage_pos<V>(h, lane, p, j);
    lds_put4(st + (p * VolStage<V>::kRowF4 + j) * 4, r[h]);
  }
}

// compute layout: lane = c * 16 + p holds floats [c V, c V + V) of row p
template <int V>
__device__ __forceinline__ void stage_get_compute(const float *st, float (&o)[V]) {
  const uint32_t lane = threadIdx.x & 63u, p = lane & 15u, c = lane >> 4;
#pragma unroll
  for (int e = 0; e < V / 4; ++e) {
    const gg_v4f v = lds_get4(st + (p * VolStage<V>::kRowF4 + c * (V / 4) + e) * 4);
    o[4 * e] = v.x; o[4 * e + 1] = v.y; o[4 * e + 2] = v.z; o[4 * e + 3] = v.w;
  }
}

template <int V>
__device__ __forceinline__ void stage_put_compute(float *st, const float (&o)[V]) {
  const uint32_t lane = threadIdx.x & 63u, p = lane & 15u, c = lane >> 4;
#pragma unroll
  for (int e = 0; e < V / 4; ++e)
    lds_put4(st + (p * VolStage<V>::kRowF4 + c * (V / 4) + e) * 4,
             (gg_v4f){o[4 * e], o[4 * e + 1], o[4 * e + 2], o[4 * e + 3]});
}

template <int V>
__device__ __forceinline__ void stage_store(const float *st, float *dst, uint32_t pix0,
                                            uint32_t npix, size_t run0, int D) {
  const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
  for (int h = 0; h < VolStage<V>::kIssues; ++h) {
    uint32_t p, j;
    stage_pos<V>(h, lane, p, j);
    const gg_v4f v = lds_get4(st + (p * VolStage<V>::kRowF4 + j) * 4);
    if (pix0 + p < npix)
      __builtin_nontemporal_store(v, (GG_GLOBAL gg_v4f *)(dst + (size_t)(pix0 + p) * D + run0 + 4u * j));
  }
}

// Dynamic LDS of integrate_tile: sF, sW (one float per thread), sBest (one
// int per pixel); with kStage also the bin table (D float2) and the
// wavefronts' volume slices.
__host__ __device__ constexpr size_t integrate_lds_head(uint32_t threads, uint32_t ppb) {
  return ((sizeof(float) * 2 * threads + sizeof(int) * ppb) + 15u) & ~(size_t)15u;
}

template <int V>
__host__ __device__ constexpr size_t integrate_lds_bytes(uint32_t threads, uint32_t ppb, int D,
                                                         bool stage) {
  return integrate_lds_head(threads, ppb) +
         (stage ? (size_t)8 * D + sizeof(float) * VolStage<V>::kWave * (threads / 64u) : 0);
}

// kCarry: 1 the previous volume is carried, 0 it is not, -1 a.carry decides
// at run time (the staged form takes it at compile time).  kRows: structured
// view-table loads (see fuse_voxels; rows of at most 2047 records).
template <int V, int KC, bool kExact, bool kStage = false, int kCarry = -1, bool kRows = false>
__device__ __forceinline__ void integrate_tile(const IntegrateArgs &a, uint32_t tile, float *smem) {
  static_assert(!kStage || V == 4 || V == 8, "staged volume stream needs V = 4 or 8");
  static_assert(!kStage || kCarry >= 0, "the staged form takes the carry at compile time");
  static_assert(!kRows || KC > 0, "structured loads in the compile-time view-count forms only");
  float *sF = smem;
  float *sW = smem + blockDim.x;
  int *sBest = reinterpret_cast<int *>(smem + 2 * blockDim.x);
  float2 *sBins = nullptr;
  float *sVol = nullptr;

  // thread -> (pixel lp, chunk of V bins): 2^pw_shift neighbouring pixels
  // of a row interleave in each wavefront, so one gather instruction reads
  // neighbouring source pixels at a few depths (few cache lines) while each
  // pixel's chunks still form contiguous runs of the volume
  const uint32_t t = threadIdx.x;
  const uint32_t pw = t & ((1u << a.pw_shift) - 1u), rest = t >> a.pw_shift;
  const uint32_t grp = fdiv(rest, a.cpp_div);
  const uint32_t chunk = rest - grp * a.cpp;
  const uint32_t lp = (grp << a.pw_shift) + pw;
  const bool lane = lp < a.ppb;
  const uint32_t pix = tile * a.ppb + lp;
  const bool active = lane && pix < a.npix;
  const int d0 = lane ? (int)chunk * V : 0;
  const size_t base = (size_t)pix * a.D + d0;

  float z[V], tau[V], S[V], Wo[V];
  if constexpr (kStage) {
    // the bin table once per workgroup in LDS
    char *head = reinterpret_cast<char *>(smem) + integrate_lds_head(blockDim.x, a.ppb);
    sBins = reinterpret_cast<float2 *>(head);
    sVol = reinterpret_cast<float *>(head + 8 * (size_t)a.D) +
           (size_t)(t >> 6) * VolStage<V>::kWave;
    for (int d = (int)t; d < a.D; d += (int)blockDim.x) sBins[d] = gload2(a.bins + d);
    __syncthreads();
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const float2 b = sBins[d0 + v];
      z[v] = b.x;
      tau[v] = b.y;
      S[v] = 0.0f;
      Wo[v] = 0.0f;
    }
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const float2 b = gload2(a.bins + d0 + v);
      z[v] = b.x;
      tau[v] = b.y;
      S[v] = 0.0f;
      Wo[v] = 0.0f;
    }
  }
  // the carried volume streams from HBM; its loads are issued after the
  // first views' gathers (see fuse_voxels)
  float Fp[V], Wp[V];
#pragma unroll
  for (int v = 0; v < V; ++v) Fp[v] = Wp[v] = 0.0f;
  const bool carry = active && a.carry;
  float mraw = 0.0f;
  // staged stream: the wavefront's first pixel and the offset of its runs
  // (every lane of a wavefront shares the pixel group and the 4 chunks)
  const uint32_t rest0 = (t & ~63u) >> 4;
  const uint32_t grp0 = fdiv(rest0, a.cpp_div);
  const uint32_t pix0 = tile * a.ppb + (grp0 << 4);
  const size_t run0 = (size_t)(rest0 - grp0 * a.cpp) * V;
  gg_v4f rF[kStage ? VolStage<V>::kIssues : 1], rW[kStage ? VolStage<V>::kIssues : 1];
  auto load_volume = [&] {
    if constexpr (kStage) {
      // kept at this point of the program: after the first views' gathers,
      // before the others (the scheduler would otherwise sink them to the end)
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (kCarry == 1) {
        stage_load<V>(a.F_prev, pix0, a.npix, run0, a.D, rF);
        stage_load<V>(a.W_prev, pix0, a.npix, run0, a.D, rW);
      }
      // unconditional as well (without a mask it reads a bin, unused)
      const float *mb = a.mask ? a.mask : reinterpret_cast<const float *>(a.bins);
      mraw = gmem(mb)[a.mask ? min(pix, a.npix - 1u) : 0u];
      __builtin_amdgcn_sched_barrier(0);
    } else {
      if (carry) {
        loadv<V>(a.F_prev + base, Fp);
        loadv<V>(a.W_prev + base, Wp);
      }
      if (active && a.mask) mraw = gmem(a.mask)[pix];
    }
  };
  float Fn[V], Wn[V];
  if constexpr (kStage) {
    // every lane fuses (a pixel past the image samples nothing in range and
    // stores nothing) and takes part in the wavefront's exchanges
    const uint32_t y = fdiv(pix, a.wt_div);
    const uint32_t x = pix - y * a.wt_div.d;
    fuse_voxels<V, KC, kExact, kRows>(a, (float)x + 0.5f, (float)y + 0.5f, z, tau, S, Wo,
                                        load_volume);
    if constexpr (kCarry == 1) {
      stage_put_stream<V>(sVol, rF);
      stage_put_stream<V>(sVol + VolStage<V>::kArray, rW);
      wave_lds_sync();
      stage_get_compute<V>(sVol, Fp);
      stage_get_compute<V>(sVol + VolStage<V>::kArray, Wp);
    }
    const float m = a.mask ? fmaxf(1.0f - mraw, 0.0f) : 1.0f;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const float wp = (kCarry == 1) ? fminf((a.decay * Wp[v]) * m, a.cap) : 0.0f;
      const float wn = wp + Wo[v];
      Fn[v] = (active && wn > 0.0f) ? fmaf(wp, Fp[v], S[v]) / wn : 0.0f;
      Wn[v] = active ? wn : 0.0f;
    }
    wave_lds_sync();
    stage_put_compute<V>(sVol, Fn);
    stage_put_compute<V>(sVol + VolStage<V>::kArray, Wn);
    wave_lds_sync();
    stage_store<V>(sVol, a.F, pix0, a.npix, run0, a.D);
    stage_store<V>(sVol + VolStage<V>::kArray, a.W, pix0, a.npix, run0, a.D);
  } else if (active) {
    const uint32_t y = fdiv(pix, a.wt_div);
    const uint32_t x = pix - y * a.wt_div.d;
    fuse_voxels<V, KC, kExact, kRows>(a, (float)x + 0.5f, (float)y + 0.5f, z, tau, S, Wo,
                                        load_volume);
    const float m = a.mask ? fmaxf(1.0f - mraw, 0.0f) : 1.0f;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const float wp = a.carry ? fminf((a.decay * Wp[v]) * m, a.cap) : 0.0f;
      const float wn = wp + Wo[v];
      Fn[v] = (wn > 0.0f) ? fmaf(wp, Fp[v], S[v]) / wn : 0.0f;
      Wn[v] = wn;
    }
    storev<V>(a.F + base, Fn);
    storev<V>(a.W + base, Wn);
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) Fn[v] = Wn[v] = 0.0f;
  }
  if (a.out_depth) {
    if constexpr (kStage) {
      const float2 *bins = sBins;
      extract_block<V>(Fn, Wn, lane, active, pix, lp, chunk, a.cpp, 1u << a.pw_shift, d0, a.D,
                       sF, sW, sBest, a.out_depth, a.out_bin,
                       [bins](int d) { return bins[d].x; });
    } else {
      const float2 *bins = a.bins;
      extract_block<V>(Fn, Wn, lane, active, pix, lp, chunk, a.cpp, 1u << a.pw_shift, d0, a.D,
                       sF, sW, sBest, a.out_depth, a.out_bin,
                       [bins](int d) { return gload2(bins + d).x; });
    }
  }
}

}  // namespace gg
