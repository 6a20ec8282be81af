// EWA pixel Gaussians composited front to back for gfx950 (§3.1: the paper
// renders each view's per-pixel Gaussians with the 3D Gaussian splatting
// rasteriser; the Gaussians are isotropic in 3D, fully opaque and one source
// pixel wide).
//
// Pipeline per call (all views at once):
//   count  - every source pixel builds its Gaussian (target mean, conic,
//            colour) into a record and counts the 8 x 8 target tiles its
//            candidate window touches (wavefront-aggregated atomics);
//   alloc  - a list segment per tile (wavefront prefix sums, one atomic per
//            wavefront on an allocator; segments in atomic order);
//   fill   - the same walk writes the key bits(z) << 32 | source index into
//            each touched tile's segment (in arrival order);
//   raster - one wavefront per (view, tile): the tile's keys are sorted in
//            ascending (z, source index) order -- a bitonic sort in LDS for
//            lists of up to sort_limit keys, else LDS-sorted runs merged
//            pairwise in global memory -- and each lane composites its pixel
//            front to back over the sorted list, 64 records at a time staged
//            through LDS, until every lane has stopped.
// The order of the terms is fixed by the keys, so the arrival order of the
// fill does not matter: outputs are bitwise reproducible.  Every
// floating-point step follows the operation order of the definition (the
// header gives it), including the exponential, so the decisions alpha >=
// 1/255 and T >= 1e-4 are taken exactly as there.
#include "ewa_internal.h"
#include "splat_device.h"

namespace gg {

// exp(x) in FP32 by Cody and Waite's argument reduction with a degree-6
// Taylor polynomial, every step an explicitly rounded FP32 operation:
// n = rint(x log2 e), r = x - n ln 2 (ln 2 as a 16-bit head plus a tail),
// e^r by Horner's rule with fused multiply-adds, times 2^n.  The definition
// returns 0 below -86; here x is clamped at -87 instead (which keeps n and r
// finite) and [-87, -86) gives at most 3e-38: every value below -86 is
// far under the opacity floor 1/255, so the terms taken are the same.
__device__ __forceinline__ float exp_alpha(float x) {
  const float xc = fmaxf(x, -87.0f);
  const float n = rintf(xc * 1.44269504f);
  float r = fmaf(-n, 0.693145752f, xc);
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

struct EwaGauss {
  bool ok;
  float u, v, z, Ah, Bn, Ch;
  int a0, a1, b0, b1;  // candidate window (superset of the pixels that can take a term)
};

// The Gaussian of source pixel (i, j) of view k at depth D.
__device__ __forceinline__ EwaGauss ewa_gauss(const EwaArgs &a, int k, float D, uint32_t i,
                                              uint32_t j) {
  EwaGauss g;
  g.ok = false;
  if (!depth_ok(D)) return g;
  const Proj &P = a.views[k].P;
  float h0, h1, h2;
  ray_of(P, (float)i + 0.5f, (float)j + 0.5f, h0, h1, h2);
  const float X0 = fmaf(D, h0, P.c[0]);
  const float X1 = fmaf(D, h1, P.c[1]);
  const float Z = fmaf(D, h2, P.c[2]);
  if (!(Z > a.zmin)) return g;
  const float inv = recip_pos(Z);  // the correctly rounded 1 / Z
  const float u = X0 * inv, v = X1 * inv;
  const float ca = (u - a.cx) / a.fx, cb = (v - a.cy) / a.fy;
  const float sig = a.views[k].sscale * (D * inv), s2 = sig * sig;
  const float sxx = s2 * (1.0f + ca * ca) + a.lowpass;
  const float syy = s2 * (a.ry2 * (1.0f + cb * cb)) + a.lowpass;
  const float sxy = s2 * (a.ry * (ca * cb));
  const float det = sxx * syy - sxy * sxy;
  g.Ah = (-0.5f * syy) / det;
  g.Bn = sxy / det;
  g.Ch = (-0.5f * sxx) / det;
  g.u = u;
  g.v = v;
  g.z = Z;
  // a term needs alpha >= 1/255, i.e. d^T S^-1 d <= 2 ln 255 < 11.1, so
  // |dx| <= sqrt(11.1 sxx) (the ellipse's extent along x), and the clip
  // bounds |dx| by rmax; 1/16 pixel of margin covers the rounding of u and
  // of the bound (the FP32 quadratic form differs from the exact one by a
  // few ulps, far inside the 0.2% between 2 ln 255 and 11.1)
  const float hx = fminf(sqrtf(11.1f * sxx), a.rmax) + 0.0625f;
  const float hy = fminf(sqrtf(11.1f * syy), a.rmax) + 0.0625f;
  float ax0 = ceilf(u - 0.5f - hx), ax1 = floorf(u - 0.5f + hx);
  float by0 = ceilf(v - 0.5f - hy), by1 = floorf(v - 0.5f + hy);
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

// Count (kFill = false: also writes the records) or list (kFill = true) the
// tiles touched by the Gaussians of the source pixels of binning block
// blockIdx.x of view blockIdx.y: 8 x 8 squares of source pixels per
// wavefront, as the splat's binning (the sort fixes the list order).
template <bool kFill>
__global__ __launch_bounds__(256) void ewa_bin_kernel(EwaArgs a) {
  const int k = blockIdx.y;
  const uint32_t nbx = splat_bin_blocks_x((uint32_t)a.Ws);
  const uint32_t by = blockIdx.x / nbx, bx = blockIdx.x - by * nbx;
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const uint32_t i = bx * kBinBlockW + wv * kBinWave + (lane % kBinWave);
  const uint32_t j = by * kBinBlockH + lane / kBinWave;
  const uint32_t q = j * (uint32_t)a.Ws + i;
  int tx0 = 0, ty0 = 0, nx = 0, n = 0;
  unsigned long long key = 0;
  if (i < (uint32_t)a.Ws && j < (uint32_t)a.Hs) {
    const size_t o = (size_t)k * a.ns + q;
    const EwaGauss g = ewa_gauss(a, k, gmem(a.depth)[o], i, j);
    if (g.ok) {
      tx0 = g.a0 / kEwaTile;
      ty0 = g.b0 / kEwaTile;
      nx = g.a1 / kEwaTile - tx0 + 1;
      n = nx * (g.b1 / kEwaTile - ty0 + 1);
      key = ((unsigned long long)__float_as_uint(g.z) << 32) | q;
      if (!kFill) {
        const GG_GLOBAL uint8_t *c = gmem(a.rgb) + 3 * o;
        const float4 r0 = make_float4(g.u, g.v, g.Ah, g.Bn);
        const float4 r1 = make_float4(g.Ch, unorm8(c[0]), unorm8(c[1]), unorm8(c[2]));
        *(GG_GLOBAL gg_v4f *)(a.rec + 2 * o) = (gg_v4f){r0.x, r0.y, r0.z, r0.w};
        *(GG_GLOBAL gg_v4f *)(a.rec + 2 * o + 1) = (gg_v4f){r1.x, r1.y, r1.z, r1.w};
      }
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
      if (pos < a.cap) gmem(a.keys)[pos] = key;
    }
  }
}

// A list segment per (view, tile): each wavefront takes an exclusive prefix
// of its 64 tiles' counts with shuffles and one atomic on the allocator
// count[n] for its total.  Segments are laid out in atomic order (a tile
// needs only its own range: offset and count); the fill's cursors are
// cleared.
__global__ __launch_bounds__(256) void ewa_alloc_kernel(uint32_t *count, uint32_t *off,
                                                        uint32_t *cursor, uint32_t n) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = __lane_id();
  const uint32_t c = t < n ? gmem(count)[t] : 0u;
  uint32_t inc = c;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t v = (uint32_t)__shfl_up((int)inc, d);
    if (lane >= d) inc += v;
  }
  const uint32_t total = (uint32_t)__shfl((int)inc, 63);
  uint32_t base = 0;
  if (lane == 63 && total) base = gatomic_add(&count[n], total);
  base = (uint32_t)__shfl((int)base, 63);
  if (t < n) {
    gmem(off)[t] = base + inc - c;
    gmem(cursor)[t] = 0u;
  }
}

__global__ void ewa_zero_kernel(uint32_t *p, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    gmem(p)[i] = 0u;
}

// v_writelane: `old` with lane `lane` set to the wave-uniform `value`.
extern "C" __device__ int gg_writelane(int value, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

// The raster's cull unit: the tile's pixels in blocks of kEwaBlock x
// kEwaBlock, each block's lanes walking their own list (2 x 2: sixteen
// blocks of four lanes; measured faster than four 4 x 4 quadrants, whose
// lists are longer, at the cost of 16 ballots per batch of records).
constexpr int kEwaBlock = 2;
constexpr int kEwaBlocksX = kEwaTile / kEwaBlock;
constexpr int kEwaBlocks = kEwaBlocksX * kEwaBlocksX;
constexpr int kEwaBlockLanes = kEwaBlock * kEwaBlock;

struct EwaLds {
  unsigned long long key[kEwaSortCap];
  float4 rec[2][64];
  float z[64];
  // per block of the tile: the staged entries that may reach it, in order;
  // slot 64 takes the writes of the lanes whose entry does not
  uint8_t idx[kEwaBlocks][65];
};

// Ascending bitonic sort of L.key[0 .. N) (N a power of two, 64 <= N <=
// kEwaSortCap) by the 64 lanes of the workgroup.
__device__ __forceinline__ void lds_bitonic(EwaLds &L, uint32_t N, uint32_t lane) {
  for (uint32_t size = 2; size <= N; size <<= 1)
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t t = lane; t < N / 2; t += 64) {
        const uint32_t i = 2 * t - (t & (stride - 1)), l = i + stride;
        const bool up = (i & size) == 0;
        const unsigned long long x = L.key[i], y = L.key[l];
        if ((x > y) == up) {
          L.key[i] = y;
          L.key[l] = x;
        }
      }
      __syncthreads();
    }
}

__device__ __forceinline__ uint32_t pow2_at_least(uint32_t n) {
  uint32_t N = 64;
  while (N < n) N <<= 1;
  return N;
}

// Sort keys[0 .. m) (m > sort_limit) in global memory: runs of `chunk`
// keys sorted in LDS, then pairwise merges between keys and alt, each lane
// producing an equal share of every merged run (merge path).  Returns the
// buffer that holds the sorted list.
__device__ const unsigned long long *global_sort(EwaLds &L, unsigned long long *keys,
                                                 unsigned long long *alt, uint32_t m,
                                                 uint32_t chunk, uint32_t lane) {
  for (uint32_t base = 0; base < m; base += chunk) {
    const uint32_t n = min(chunk, m - base);
    for (uint32_t t = lane; t < chunk; t += 64) L.key[t] = t < n ? gmem(keys)[base + t] : ~0ull;
    __syncthreads();
    lds_bitonic(L, chunk, lane);
    for (uint32_t t = lane; t < n; t += 64) gmem(keys)[base + t] = L.key[t];
    __syncthreads();
  }
  __threadfence();
  __syncthreads();
  unsigned long long *src = keys, *dst = alt;
  for (uint32_t w = chunk; w < m; w <<= 1) {
    for (uint32_t lo = 0; lo < m; lo += 2 * w) {
      const uint32_t na = min(w, m - lo);
      const uint32_t nb = m - lo > w ? min(w, m - lo - w) : 0u;
      const GG_GLOBAL unsigned long long *A = gmem(src) + lo, *B = A + na;
      GG_GLOBAL unsigned long long *out = gmem(dst) + lo;
      const uint32_t n = na + nb;
      const uint32_t d0 = (uint32_t)(((unsigned long long)n * lane) / 64u);
      const uint32_t d1 = (uint32_t)(((unsigned long long)n * (lane + 1)) / 64u);
      // A elements among the first d0 outputs
      uint32_t lo_i = d0 > nb ? d0 - nb : 0u, hi_i = min(d0, na);
      while (lo_i < hi_i) {
        const uint32_t mid = (lo_i + hi_i) >> 1;
        if (A[mid] < B[d0 - 1 - mid])
          lo_i = mid + 1;
        else
          hi_i = mid;
      }
      uint32_t ia = lo_i, ib = d0 - lo_i;
      for (uint32_t o = d0; o < d1; ++o) {
        const bool take_a = ib >= nb || (ia < na && A[ia] < B[ib]);
        out[o] = take_a ? A[ia++] : B[ib++];
      }
    }
    __threadfence();
    __syncthreads();
    unsigned long long *t = src;
    src = dst;
    dst = t;
  }
  return src;
}

// The blocks of the tile (origin (tx0, ty0)) at whose pixels the Gaussian of
// a staged record may take a term, as a bit mask (bit b: block b).  A term
// needs alpha >= 1/255, so d^T S^-1 d <= 2 ln 255 < 11.1 and |dx| <=
// sqrt(11.1 S_xx), and it needs |dx| <= rmax.  S_xx = M_yy / det M of the
// conic M = S^-1, whose entries the record holds as Ah = -M_xx / 2, Ch =
// -M_yy / 2, Bn = -M_xy; the extent takes 2% and a quarter pixel of margin
// for the rounding of this reconstruction (the hardware's reciprocal and
// square root, within an ulp or two, are well inside it) and of the tests
// (a conic so ill-conditioned that S_xx comes out negative, infinite or NaN
// falls back to rmax: fminf drops the NaN).  The test is a superset, so it
// never decides a term: skipping a record it rejects leaves every pixel of
// the block exactly as taking it would.  It is separable: a block's column
// decides the x half, its row the y half.
__device__ __forceinline__ uint32_t ewa_reach(float4 A, float4 B, float rmax, float tx0,
                                              float ty0) {
  const float det = 4.0f * (A.z * B.x) - A.w * A.w;
  const float rdet = __builtin_amdgcn_rcpf(det);
  const float sxx = (-2.0f * B.x) * rdet, syy = (-2.0f * A.z) * rdet;
  const float hx = fminf(__builtin_amdgcn_sqrtf(11.32f * sxx), rmax) + 0.25f;
  const float hy = fminf(__builtin_amdgcn_sqrtf(11.32f * syy), rmax) + 0.25f;
  // pixel centres q + 0.5 .. q + kEwaBlock - 0.5 against u +- h
  constexpr float kLast = (float)kEwaBlock - 0.5f;
  uint32_t cols = 0, rows = 0;
#pragma unroll
  for (int c = 0; c < kEwaBlocksX; ++c) {
    const float qx = tx0 + (float)(kEwaBlock * c), qy = ty0 + (float)(kEwaBlock * c);
    if ((qx + 0.5f) - A.x <= hx && A.x - (qx + kLast) <= hx) cols |= 1u << c;
    if ((qy + 0.5f) - A.y <= hy && A.y - (qy + kLast) <= hy) rows |= 1u << c;
  }
  uint32_t reach = 0;
#pragma unroll
  for (int r = 0; r < kEwaBlocksX; ++r)
    if ((rows >> r) & 1u) reach |= cols << (kEwaBlocksX * r);
  return reach;
}

// One wavefront per (view, tile); its 64 lanes are the tile's blocks of
// kEwaBlock x kEwaBlock pixels (the lanes of block b consecutive, row-major
// in the block; blocks row-major in the tile).  Each batch of 64 staged
// records is culled per block (ewa_reach) into an ordered list, and each
// block's lanes composite only their own list: the wavefront takes as many
// steps as the longest list instead of all 64, and every pixel still sees,
// front to back, every record that can touch it.
__global__ __launch_bounds__(64) void ewa_raster_kernel(EwaArgs a) {
  __shared__ EwaLds L;
  const int k = blockIdx.y;
  const uint32_t tile = xcd_tile(blockIdx.x, a.ntiles);
  const uint32_t lane = threadIdx.x;
  const uint32_t ty = tile / (uint32_t)a.ntx, tx = tile - ty * (uint32_t)a.ntx;
  const uint32_t blk = lane / kEwaBlockLanes, ql = lane % kEwaBlockLanes;
  const int qx0 = (int)tx * kEwaTile + kEwaBlock * (int)(blk % kEwaBlocksX);
  const int qy0 = (int)ty * kEwaTile + kEwaBlock * (int)(blk / kEwaBlocksX);
  const int x = qx0 + (int)(ql % kEwaBlock), y = qy0 + (int)(ql / kEwaBlock);
  const size_t seg = (size_t)k * a.ntiles + tile;
  const uint32_t off = min(gmem(a.tile_offset)[seg], a.cap);
  const uint32_t m = min(gmem(a.tile_count)[seg], a.cap - off);
  const unsigned long long *list = nullptr;
  const bool in_lds = m <= a.sort_limit;
  if (m > 0) {
    if (in_lds) {
      const uint32_t N = pow2_at_least(m);
      for (uint32_t t = lane; t < N; t += 64) L.key[t] = t < m ? gmem(a.keys)[off + t] : ~0ull;
      __syncthreads();
      lds_bitonic(L, N, lane);
    } else {
      uint32_t chunk = 64;
      while (chunk * 2 <= a.sort_limit) chunk <<= 1;
      list = global_sort(L, a.keys + off, a.keys_alt + off, m, chunk, lane);
    }
  }
  const float px = (float)x + 0.5f, py = (float)y + 0.5f;
  const float amin = 1.0f / 255.0f, rmax = a.rmax;
  float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, zs = 0.0f;
  bool done = x >= a.Wt || y >= a.Ht;
  const float4 *rec = a.rec + 2 * (size_t)k * a.ns;
  const float tx0 = (float)((int)tx * kEwaTile), ty0 = (float)((int)ty * kEwaTile);
  for (uint32_t base = 0; base < m; base += 64) {
    if (__all(done)) break;
    const uint32_t e = base + lane;
    uint32_t reach = 0;  // bit b: the record may reach block b
    if (e < m) {
      const unsigned long long key = in_lds ? L.key[e] : gmem(list)[e];
      const uint32_t q = (uint32_t)key;
      const gg_v4f r0 = *(const GG_GLOBAL gg_v4f *)(rec + 2 * (size_t)q);
      const gg_v4f r1 = *(const GG_GLOBAL gg_v4f *)(rec + 2 * (size_t)q + 1);
      const float4 A = make_float4(r0.x, r0.y, r0.z, r0.w), B = make_float4(r1.x, r1.y, r1.z, r1.w);
      L.rec[0][lane] = A;
      L.rec[1][lane] = B;
      L.z[lane] = __uint_as_float((uint32_t)(key >> 32));
      reach = ewa_reach(A, B, rmax, tx0, ty0);
    }
    // each block's list: the records that reach it, in staging (= front to back) order
    int counts = 0;  // lane b (< kEwaBlocks): the length of block b's list
#pragma unroll
    for (uint32_t qd = 0; qd < (uint32_t)kEwaBlocks; ++qd) {
      const bool hit = (reach & (1u << qd)) != 0u;
      const unsigned long long b = __builtin_amdgcn_ballot_w64(hit);
      // the lane's rank among the hits: set bits of b below the lane
      const uint32_t rank =
          __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
      // every lane stores (no branch): a hit at its rank, the others into the
      // row's spare slot, which nothing reads (relaxed atomic stores, as
      // several lanes store to it at once)
      __hip_atomic_store(&L.idx[qd][hit ? rank : 64u], (uint8_t)lane, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_WORKGROUP);
      counts = gg_writelane(__popcll(b), (int)qd, counts);
    }
    const uint32_t nq = (uint32_t)__shfl(counts, (int)blk);
    __syncthreads();
    // each block walks its own list; the wavefront runs as long as the longest
    for (uint32_t s = 0; s < nq; ++s) {
      const uint32_t t = L.idx[blk][s];
      const float4 A = L.rec[0][t], B = L.rec[1][t];
      const float dx = px - A.x, dy = py - A.y;
      const bool in = fabsf(dx) <= rmax && fabsf(dy) <= rmax;
      const float power = fmaf(A.w, dx * dy, fmaf(A.z, dx * dx, B.x * (dy * dy)));
      const float z = L.z[t];
      const float al = fminf(0.99f, exp_alpha(power));
      const float tt = T * (1.0f - al);
      const bool take = !done && in && !(power > 0.0f) && !(al < amin);
      const bool stop = take && tt < 1e-4f;
      if (take && !stop) {
        const float w = al * T;
        c0 = fmaf(B.y, w, c0);
        c1 = fmaf(B.z, w, c1);
        c2 = fmaf(B.w, w, c2);
        zs = fmaf(z, w, zs);
        T = tt;
      }
      done = done || stop;
    }
    __syncthreads();
  }
  if (x < a.Wt && y < a.Ht) {
    const size_t p = (size_t)y * a.Wt + x, kt = (size_t)k * a.nt;
    gmem(a.out_rgb)[3 * kt + p] = c0;
    gmem(a.out_rgb)[3 * kt + a.nt + p] = c1;
    gmem(a.out_rgb)[3 * kt + 2 * (size_t)a.nt + p] = c2;
    gmem(a.out_alpha)[kt + p] = 1.0f - T;
    gmem(a.out_depth)[kt + p] = T < 1.0f ? zs / (1.0f - T) : 0.0f;
  }
}

uint32_t ewa_tiles_per_splat(float r_max) {
  // candidate window <= 2 (r_max + 1/16) + 1 pixels wide, below 2 ceil(r_max) + 3
  const int w = 2 * (int)ceilf(r_max) + 3;
  const int per = (w - 1) / kEwaTile + 2;
  return (uint32_t)(per * per);
}

int launch_splat_ewa(const EwaArgs &a, hipStream_t s) {
  const uint32_t n = (uint32_t)a.K * a.ntiles;
  const dim3 gsrc(splat_bin_blocks((uint32_t)a.Ws, (uint32_t)a.Hs), a.K);
  {
    KernelTimer t("ewa_zero", s);
    hipLaunchKernelGGL(ewa_zero_kernel, dim3(min((n + 256) / 256, 1024u)), dim3(256), 0, s,
                       a.tile_count, n + 1);
    if (int rc = check_hip(hipGetLastError(), "ewa_zero_kernel")) return rc;
  }
  {
    KernelTimer t("ewa_count", s);
    hipLaunchKernelGGL(ewa_bin_kernel<false>, gsrc, dim3(256), 0, s, a);
    if (int rc = check_hip(hipGetLastError(), "ewa_bin_kernel<count>")) return rc;
  }
  {
    KernelTimer t("ewa_alloc", s);
    hipLaunchKernelGGL(ewa_alloc_kernel, dim3((n + 255) / 256), dim3(256), 0, s, a.tile_count,
                       a.tile_offset, a.tile_cursor, n);
    if (int rc = check_hip(hipGetLastError(), "ewa_alloc_kernel")) return rc;
  }
  {
    KernelTimer t("ewa_fill", s);
    hipLaunchKernelGGL(ewa_bin_kernel<true>, gsrc, dim3(256), 0, s, a);
    if (int rc = check_hip(hipGetLastError(), "ewa_bin_kernel<fill>")) return rc;
  }
  KernelTimer t("ewa_raster", s);
  hipLaunchKernelGGL(ewa_raster_kernel, dim3(a.ntiles, a.K), dim3(64), 0, s, a);
  return check_hip(hipGetLastError(), "ewa_raster_kernel");
}

}  // namespace gg
