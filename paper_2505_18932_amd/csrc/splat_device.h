// Device functions of the z-buffered splat (§3.1, Suppl. A.3) shared by the
// plain kernels (splat.hip) and the batched persistent kernels (batch.hip).
#pragma once

#include "ggeom_internal.h"

namespace gg {

struct SplatGeom {
  bool ok;
  float x, y, z, s2, R2;
  int a0, a1, b0, b1;  // candidate window (superset of covered pixels)
};

// Footprint of source pixel (i, j) at depth D in the target.
__device__ __forceinline__ SplatGeom splat_geom(const SplatView &V, float D, uint32_t i,
                                                uint32_t j, const SplatArgs &a) {
  SplatGeom g;
  g.ok = false;
  if (!depth_ok(D)) return g;
  float h0, h1, h2;
  ray_of(V.P, (float)i + 0.5f, (float)j + 0.5f, h0, h1, h2);
  const float X0 = fmaf(D, h0, V.P.c[0]);
  const float X1 = fmaf(D, h1, V.P.c[1]);
  const float Z = fmaf(D, h2, V.P.c[2]);
  if (!(Z > a.zmin)) return g;
  const float inv = recip_pos(Z);  // the correctly rounded 1 / Z
  g.x = X0 * inv;
  g.y = X1 * inv;
  g.z = Z;
  const float sig = V.sscale * (D * inv);
  g.s2 = sig * sig;
  g.R2 = fminf(2.0f * g.s2, a.rmax2);
  // candidate window: covered pixels have |a + 0.5 - x| <= r (1 + 2^-21)
  // (the rounded d2 is at least the rounded dx^2); the hardware square root
  // (within an ulp) and the float bounds below carry at most 4 ulps of
  // |x| + r, which is below 2^15 wherever a pixel is covered (images of at
  // most 16384 pixels, r_max at most 64): at most 2^-7, inside the margin
  const float r = __builtin_amdgcn_sqrtf(g.R2) + 0x1p-6f;
  float ax0 = ceilf(g.x - 0.5f - r), ax1 = floorf(g.x - 0.5f + r);
  float by0 = ceilf(g.y - 0.5f - r), by1 = floorf(g.y - 0.5f + r);
  ax0 = fmaxf(ax0, 0.0f);
  by0 = fmaxf(by0, 0.0f);
  ax1 = fminf(ax1, (float)(a.Wt - 1));
  by1 = fminf(by1, (float)(a.Ht - 1));
  if (!(ax0 <= ax1 && by0 <= by1)) return g;
  g.a0 = (int)ax0;
  g.a1 = (int)ax1;
  g.b0 = (int)by0;
  g.b1 = (int)by1;
  g.ok = true;
  return g;
}

__device__ __forceinline__ float cover_d2(const SplatGeom &g, int aa, int b) {
  const float dx = ((float)aa + 0.5f) - g.x;
  const float dy = ((float)b + 0.5f) - g.y;
  return fmaf(dx, dx, dy * dy);
}

// Wavefront-aggregated atomicAdd: lanes with the same key share one atomic;
// each gets a distinct slot base + rank.  The lanes are grouped by key with
// ballots only (no memory traffic); then every group's leader issues its
// atomic in one instruction and each lane reads its leader's base with one
// cross-lane permute, so a wavefront waits for one atomic round trip.
// kReturn = false (counting) issues the atomics without a return value.
template <bool kReturn>
__device__ __forceinline__ uint32_t aggregated_slot(uint32_t *counters, uint32_t key, bool has) {
  const int lane = __lane_id();
  unsigned long long pending = __ballot(has);
  int leader = lane;
  uint32_t rank = 0, count = 0;
  while (pending) {
    const int l = __ffsll((unsigned long long)pending) - 1;
    const uint32_t lkey = __shfl(key, l);
    const bool mine = has && key == lkey;
    const unsigned long long grp = __ballot(mine);
    if (mine) {
      leader = l;
      rank = (uint32_t)__popcll(grp & ((1ull << lane) - 1ull));
    }
    if (lane == l) count = (uint32_t)__popcll(grp);
    pending &= ~grp;
  }
  const bool lead = has && lane == leader;
  if (!kReturn) {
    if (lead)
      __hip_atomic_fetch_add(gmem(&counters[key]), count, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  uint32_t base = 0;
  if (lead) base = gatomic_add(&counters[key], count);
  base = (uint32_t)__shfl((int)base, leader);
  return base + rank;
}

// Source pixels of one binning workgroup (256 threads): four wavefronts of
// kBinWave x kBinWave pixels side by side.  A square of neighbouring source
// pixels lands on a compact target region, which touches fewer distinct
// tiles than a run of 64 pixels along a row: fewer rounds of the
// wavefront's per-tile grouping (aggregated_slot).  The order in which a
// tile's list receives its entries changes nothing downstream: the z-test
// keeps the minimum key and the blend sums integers.
constexpr uint32_t kBinWave = 8;
constexpr uint32_t kBinBlockW = 4 * kBinWave, kBinBlockH = kBinWave;

__host__ __device__ constexpr uint32_t splat_bin_blocks_x(uint32_t Ws) {
  return (Ws + kBinBlockW - 1) / kBinBlockW;
}
__host__ __device__ constexpr uint32_t splat_bin_blocks(uint32_t Ws, uint32_t Hs) {
  return splat_bin_blocks_x(Ws) * ((Hs + kBinBlockH - 1) / kBinBlockH);
}

// Count (kFill = false) or list (kFill = true) the target tiles touched by
// the footprints of the source pixels of binning block blk of view k.
template <bool kFill>
__device__ __forceinline__ void splat_bin_block(const SplatArgs &a, int k, uint32_t blk) {
  const uint32_t nbx = splat_bin_blocks_x((uint32_t)a.Ws);
  const uint32_t by = blk / nbx, bx = blk - by * nbx;  // wave-uniform
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const uint32_t i = bx * kBinBlockW + wv * kBinWave + (lane % kBinWave);
  const uint32_t j = by * kBinBlockH + lane / kBinWave;
  const uint32_t q = j * (uint32_t)a.Ws + i;
  int tx0 = 0, ty0 = 0, nx = 0, n = 0;
  if (i < (uint32_t)a.Ws && j < (uint32_t)a.Hs) {
    const SplatGeom g = splat_geom(a.views[k], gmem(a.depth)[(size_t)k * a.ns + q], i, j, a);
    if (g.ok) {
      tx0 = g.a0 / kTile;
      ty0 = g.b0 / kTile;
      nx = g.a1 / kTile - tx0 + 1;
      n = nx * (g.b1 / kTile - ty0 + 1);
    }
  }
  uint32_t *cnt = (kFill ? a.tile_cursor : a.tile_count) + (size_t)k * a.ntiles;
  // the covered tiles in row-major order: column sx, row sy of the range
  int sx = 0, sy = 0;
  for (int s = 0;; ++s) {
    const bool has = s < n;
    if (__ballot(has) == 0ull) break;
    const uint32_t tile = has ? (uint32_t)((ty0 + sy) * a.ntx + (tx0 + sx)) : 0u;
    if (++sx == nx) {
      sx = 0;
      ++sy;
    }
    const uint32_t slot = aggregated_slot<kFill>(cnt, tile, has);
    if (kFill && has) {
      const uint32_t pos = gmem(a.tile_offset)[(size_t)k * a.ntiles + tile] + slot;
      if (pos < a.list_cap) gmem(a.list)[pos] = q;
    }
  }
}

// Exclusive scan of n counters by one workgroup of 1024 threads; also
// clears the cursors.  off has n + 1 entries (the last is the total).
// Chunks of kScanChunk counters are staged through LDS so that global loads
// and stores are coalesced; each thread scans 8 consecutive entries, the
// 1024 partial sums are scanned with wavefront shuffles.
constexpr uint32_t kScanChunk = 8192;
struct ScanLds {
  uint32_t buf[kScanChunk];
  uint32_t wave[16];
  uint32_t part[1024];
};

__device__ __forceinline__ void tile_scan_block(const uint32_t *cnt, uint32_t *off,
                                                uint32_t *cursor, uint32_t n, ScanLds &L) {
  const uint32_t t = threadIdx.x, lane = t & 63u, wv = t >> 6;
  uint32_t carry = 0;
  for (uint32_t base = 0; base < n; base += kScanChunk) {
#pragma unroll
    for (uint32_t i = 0; i < 8; ++i) {
      const uint32_t g = base + t + 1024u * i;
      L.buf[t + 1024u * i] = g < n ? gmem(cnt)[g] : 0u;
    }
    __syncthreads();
    uint32_t sum = 0;
#pragma unroll
    for (uint32_t i = 0; i < 8; ++i) sum += L.buf[8u * t + i];
    // inclusive scan of the partial sums within the wavefront
    uint32_t inc = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t v = __shfl_up(inc, d);
      if ((int)lane >= d) inc += v;
    }
    if (lane == 63) L.wave[wv] = inc;
    __syncthreads();
    uint32_t wbase = 0, total = 0;
    for (uint32_t w = 0; w < 16; ++w) {
      const uint32_t x = L.wave[w];
      wbase += w < wv ? x : 0u;
      total += x;
    }
    uint32_t run = carry + wbase + inc - sum;
#pragma unroll
    for (uint32_t i = 0; i < 8; ++i) {
      const uint32_t c = L.buf[8u * t + i];
      L.buf[8u * t + i] = run;
      run += c;
    }
    __syncthreads();
#pragma unroll
    for (uint32_t i = 0; i < 8; ++i) {
      const uint32_t g = base + t + 1024u * i;
      if (g < n) {
        gmem(off)[g] = L.buf[t + 1024u * i];
        gmem(cursor)[g] = 0u;
      }
    }
    carry += total;
    __syncthreads();
  }
  if (t == 0) gmem(off)[n] = carry;
  __syncthreads();
}

constexpr double kFixG = 1099511627776.0;  // 2^40: sums of G and G c
constexpr double kFixL = 4294967296.0;     // 2^32: sums of log(1 - G)

// A fixed-point term round(t 2^32) (round half to even) for 0 <= t < 2^32,
// in FP32 operations that are exact but for the one rounding: hi = floor(t)
// and the fraction f = t - hi are exact (f keeps a subset of t's
// significand bits), f 2^32 is exact, and round(t 2^32) = hi 2^32 +
// round(f 2^32) because hi 2^32 is an integer; f <= 1 - 2^-24 keeps
// round(f 2^32) below 2^32, so the low word never carries.  Bitwise what
// the FP64 product and a 64-bit rint give, at a fraction of their cost.
// (For t < 0 the fraction 1 - |t| of a small |t| is not exact; rounding
// half to even is symmetric, so negative terms go through -t.)
__device__ __forceinline__ unsigned long long fix_nonneg(float t) {
  const float hi = floorf(t);
  const float lo = rintf((t - hi) * 4294967296.0f);
  return ((unsigned long long)(uint32_t)hi << 32) + (unsigned long long)(uint32_t)lo;
}
// round(t 2^32) of either sign, as a two's complement word
__device__ __forceinline__ unsigned long long fix_signed(float t) {
  const unsigned long long m = fix_nonneg(fabsf(t));
  return t < 0.0f ? 0ull - m : m;
}
// round(x kFixG) = round((x 2^8) 2^32) (x 2^8 exact) for x >= 0
__device__ __forceinline__ unsigned long long fix_g(float x) { return fix_nonneg(x * 256.0f); }
// round(L kFixL) for L <= 0
__device__ __forceinline__ unsigned long long fix_l(float L) { return 0ull - fix_nonneg(-L); }

// LDS of one raster tile.
struct RasterLds {
  unsigned long long zkey[kTile * kTile];
  unsigned long long sG[kTile * kTile], sR[kTile * kTile], sGr[kTile * kTile], sB[kTile * kTile],
      sL[kTile * kTile], sM[kTile * kTile];
  uint32_t sOnes[kTile * kTile];
};

__device__ __forceinline__ void raster_output(const SplatArgs &a, int k, int px, int py,
                                              const RasterLds &lds, uint32_t t) {
  const unsigned long long *sG = lds.sG, *sR = lds.sR, *sGr = lds.sGr, *sB = lds.sB,
                           *sL = lds.sL;
  const uint32_t *sOnes = lds.sOnes;
  const unsigned long long *zkey = lds.zkey;
  const size_t p = (size_t)py * a.Wt + px;
  const size_t o = (size_t)k * a.nt + p;
  const unsigned long long wk = zkey[t];
  // The weighted means divide the fixed-point sums in FP32: each sum is
  // rounded to FP32 (through FP64, whose conversion of a 64-bit integer is
  // short), and 1 / (sum of G) multiplies the numerators.  Each result is
  // within a few ulps of the exact quotient.
  const float inv_g = wk == ~0ull ? 0.0f : 1.0f / (float)(double)(long long)sG[t];
  if (a.mask_in) {
    // the mask channel, like the colours; its maximum over the views as
    // float bits (non-negative floats order as unsigned integers)
    const float m = wk == ~0ull ? 0.0f : (float)(double)(long long)lds.sM[t] * inv_g;
    if (a.out_mask) gmem(a.out_mask)[o] = m;
    if (a.out_mask_max)
      __hip_atomic_fetch_max(reinterpret_cast<GG_GLOBAL uint32_t *>(gmem(a.out_mask_max) + p),
                             __float_as_uint(m), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  GG_GLOBAL float *rgb = gmem(a.out_rgb + (size_t)k * 3 * a.nt);
  GG_GLOBAL int32_t *win = gmem(a.win_idx);
  GG_GLOBAL float *dep = gmem(a.out_depth), *alp = gmem(a.out_alpha);
  if (wk == ~0ull) {
    win[o] = -1;
    dep[o] = 0.0f;
    alp[o] = 0.0f;
    rgb[p] = rgb[a.nt + p] = rgb[2 * a.nt + p] = 0.0f;
    if (a.out_tape) {
      GG_GLOBAL float *tp = gmem(a.out_tape + (size_t)k * 3 * a.nt);
      tp[p] = tp[a.nt + p] = tp[2 * a.nt + p] = 0.0f;
    }
    return;
  }
  win[o] = (int32_t)(uint32_t)(wk & 0xffffffffull);
  dep[o] = __uint_as_float((uint32_t)(wk >> 32));
  rgb[p] = (float)(double)(long long)sR[t] * inv_g;
  rgb[a.nt + p] = (float)(double)(long long)sGr[t] * inv_g;
  rgb[2 * a.nt + p] = (float)(double)(long long)sB[t] * inv_g;
  const double L = (double)(long long)sL[t] / kFixL;  // power-of-two scalings: exact
  // alpha = 1 - prod(1 - G) = -(exp(L) - 1), with expm1 accurate where alpha is small
  alp[o] = sOnes[t] ? 1.0f : -expm1f((float)L);
  if (a.out_tape) {
    GG_GLOBAL float *tp = gmem(a.out_tape + (size_t)k * 3 * a.nt);
    tp[p] = (float)((double)(long long)sG[t] / kFixG);
    tp[a.nt + p] = (float)L;
    tp[2 * a.nt + p] = (float)sOnes[t];
  }
}

// Z-test and band blend of target tile `tile` of view k (kTile * kTile
// threads).
// kKeepFirst: carry the thread's first entry from the z-test to the blend in
// registers (more VGPRs, fewer loads); the results are the same either way.
template <bool kKeepFirst>
__device__ __forceinline__ void raster_tile(const SplatArgs &a, int k, uint32_t tile,
                                            RasterLds &lds) {
  unsigned long long *zkey = lds.zkey, *sG = lds.sG, *sR = lds.sR, *sGr = lds.sGr, *sB = lds.sB,
                     *sL = lds.sL, *sM = lds.sM;
  uint32_t *sOnes = lds.sOnes;
  const int tyi = (int)(tile / (uint32_t)a.ntx), txi = (int)tile - tyi * a.ntx;
  const int ax0 = txi * kTile, by0 = tyi * kTile;
  const uint32_t t = threadIdx.x;
  zkey[t] = ~0ull;
  sG[t] = sR[t] = sGr[t] = sB[t] = sL[t] = sM[t] = 0ull;
  sOnes[t] = 0u;
  __syncthreads();
  const size_t ti = (size_t)k * a.ntiles + tile;
  const uint32_t beg = gmem(a.tile_offset)[ti], end = min(gmem(a.tile_offset)[ti + 1], a.list_cap);
  const SplatView &V = a.views[k];
  const float *dk = a.depth + (size_t)k * a.ns;
  const uint8_t *ck = a.rgb + (size_t)k * a.ns * 3;
  // z-test.  With kKeepFirst the thread's first entry (most threads have one
  // or two) keeps its index and footprint in registers for the blend pass.
  uint32_t q_first = 0xffffffffu;
  SplatGeom g_first;
  g_first.ok = false;
  for (uint32_t e = beg + t; e < end; e += blockDim.x) {
    const uint32_t q = gmem(a.list)[e];
    if (q >= a.ns) continue;
    const uint32_t j = fdiv(q, a.ws_div), i = q - j * (uint32_t)a.Ws;
    const SplatGeom g = splat_geom(V, gmem(dk)[q], i, j, a);
    if (kKeepFirst && e == beg + t) {
      q_first = q;
      g_first = g;
    }
    if (!g.ok) continue;
    const unsigned long long key = ((unsigned long long)__float_as_uint(g.z) << 32) | q;
    const int a0 = max(g.a0, ax0), a1 = min(g.a1, ax0 + kTile - 1);
    const int b0 = max(g.b0, by0), b1 = min(g.b1, by0 + kTile - 1);
    for (int b = b0; b <= b1; ++b)
      for (int aa = a0; aa <= a1; ++aa)
        if (cover_d2(g, aa, b) <= g.R2) atomicMin(&zkey[(b - by0) * kTile + (aa - ax0)], key);
  }
  __syncthreads();
  // band blend
  for (uint32_t e = beg + t; e < end; e += blockDim.x) {
    const bool first = kKeepFirst && e == beg + t;
    const uint32_t q = first ? q_first : gmem(a.list)[e];
    if (q >= a.ns) continue;
    SplatGeom g;
    if (first) {
      g = g_first;
    } else {
      const uint32_t j = fdiv(q, a.ws_div), i = q - j * (uint32_t)a.Ws;
      g = splat_geom(V, gmem(dk)[q], i, j, a);
    }
    if (!g.ok) continue;
    // the entry's colour (c = u8 / 255) and mask, once for all its pixels
    const float c0 = unorm8(gmem(ck)[3 * (size_t)q + 0]);
    const float c1 = unorm8(gmem(ck)[3 * (size_t)q + 1]);
    const float c2 = unorm8(gmem(ck)[3 * (size_t)q + 2]);
    const float m = a.mask_in ? gmem(a.mask_in)[(size_t)k * a.ns + q] : 0.0f;
    const int a0 = max(g.a0, ax0), a1 = min(g.a1, ax0 + kTile - 1);
    const int b0 = max(g.b0, by0), b1 = min(g.b1, by0 + kTile - 1);
    for (int b = b0; b <= b1; ++b)
      for (int aa = a0; aa <= a1; ++aa) {
        const float d2 = cover_d2(g, aa, b);
        if (!(d2 <= g.R2)) continue;
        const int lp = (b - by0) * kTile + (aa - ax0);
        const float zw = __uint_as_float((uint32_t)(zkey[lp] >> 32));
        if (!(g.z <= zw * a.band)) continue;
        const float G = expf((-0.5f * d2) / g.s2);
        atomicAdd(&sG[lp], fix_g(G));
        atomicAdd(&sR[lp], fix_g(G * c0));
        atomicAdd(&sGr[lp], fix_g(G * c1));
        atomicAdd(&sB[lp], fix_g(G * c2));
        if (a.mask_in) atomicAdd(&sM[lp], fix_signed((G * m) * 256.0f));
        if (G < 1.0f)
          atomicAdd(&sL[lp], fix_l(logf(1.0f - G)));
        else
          atomicAdd(&sOnes[lp], 1u);
      }
  }
  __syncthreads();
  const int px = ax0 + (int)(t % kTile), py = by0 + (int)(t / kTile);
  if (px < a.Wt && py < a.Ht) raster_output(a, k, px, py, lds, t);
  __syncthreads();  // LDS reused by the caller's next tile
}

}  // namespace gg
