// Frustum-volume TSDF for gfx950: fusion weight map, depth bins, fused
// integrate + extraction, standalone extraction, adjoints.
//
// Paper passages: Suppl. A.1 (projection, signed distance, truncation,
// noise-aware weight, occlusion rule, sign change along the ray), Suppl. A.2
// (temporal weight), §3.2 (image-based TSDF guiding the target depth).
//
// Arithmetic is FP32 in a fixed operation order (no contraction; fused
// multiply-adds are explicit fmaf; divide and square root are correctly
// rounded) so that the volume and the extracted bins are bitwise
// reproducible and equal to the plain definition.
#include "tsdf_device.h"

namespace gg {

// ---------------------------------------------------------------------------
// depth bins: z_d = 1 / (1/z_near - d du), tau_d = trunc du z_d^2 (in bins)

__global__ void bins_kernel(int32_t D, float z_near, float z_far, float trunc, int32_t in_bins,
                            float2 *out) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= D) return;
  const float un = 1.0f / z_near;
  const float uf = 1.0f / z_far;
  const float du = (un - uf) / (float)(D - 1);
  const float z = bin_depth(d, D, z_near, z_far);
  out[d] = make_float2(z, in_bins ? (trunc * du) * (z * z) : trunc);
}

int launch_bins(const gg_tsdf_params &p, float2 *bins, hipStream_t s) {
  KernelTimer t("bins", s);
  hipLaunchKernelGGL(bins_kernel, dim3((p.num_bins + 255) / 256), dim3(256), 0, s, p.num_bins,
                     p.z_near, p.z_far, p.trunc, p.trunc_in_bins, bins);
  return check_hip(hipGetLastError(), "bins_kernel");
}

// ---------------------------------------------------------------------------
// fusion weight (Suppl. A.1): one workgroup per 32 x 8 pixels of one view,
// the tile plus its halo staged in LDS by coalesced row loads.  Output: the
// view table (usable depth, or -inf for a hole so that the occlusion test
// drops it; omega), one 8-byte record per pixel, gathered by the fusion.

__global__ __launch_bounds__(256) void conf_kernel(ConfArgs a) {
  __shared__ float tile[kConfLH * kConfLW];
  conf_tile(a, blockIdx.z, blockIdx.x, blockIdx.y, tile);
}

int launch_conf(const ConfArgs &a, hipStream_t s) {
  KernelTimer t("conf", s);
  dim3 grid((a.Ws + kConfTX - 1) / kConfTX, (a.Hs + kConfTY - 1) / kConfTY, a.K);
  hipLaunchKernelGGL(conf_kernel, grid, dim3(kConfTX * kConfTY), 0, s, a);
  return check_hip(hipGetLastError(), "conf_kernel");
}

template <int V, int KC, bool kExact, bool kStage, int kCarry, bool kRows = false>
__global__ __launch_bounds__(1024) void integrate_kernel(IntegrateArgs a) {
  extern __shared__ float smem[];
  integrate_tile<V, KC, kExact, kStage, kCarry, kRows>(
      a, band_tile(a, xcd_tile(blockIdx.x, a.nblocks)), smem);
}

template <int V, int KC, bool kStage, int kCarry>
static void launch_integrate_vk(const IntegrateArgs &a, uint32_t threads, size_t shm,
                                hipStream_t s) {
  // structured view-table loads: only in the staged, carried forms with up to four views
  // (the host sets a.rows where they pay; elsewhere the specialisation does not exist)
  if constexpr (kStage && kCarry == 1 && KC >= 1 && KC <= 4) {
    if (a.rows && !a.exact_only) {
      hipLaunchKernelGGL((integrate_kernel<V, KC, false, kStage, kCarry, true>), dim3(a.nblocks),
                         dim3(threads), shm, s, a);
      return;
    }
  }
  if (a.exact_only)
    hipLaunchKernelGGL((integrate_kernel<V, KC, true, kStage, kCarry>), dim3(a.nblocks),
                       dim3(threads), shm, s, a);
  else
    hipLaunchKernelGGL((integrate_kernel<V, KC, false, kStage, kCarry>), dim3(a.nblocks),
                       dim3(threads), shm, s, a);
}

template <int V, bool kStage, int kCarry>
static void launch_integrate_v(const IntegrateArgs &a, uint32_t threads, size_t shm,
                               hipStream_t s) {
  switch (a.K) {
    case 1: launch_integrate_vk<V, 1, kStage, kCarry>(a, threads, shm, s); break;
    case 2: launch_integrate_vk<V, 2, kStage, kCarry>(a, threads, shm, s); break;
    case 3: launch_integrate_vk<V, 3, kStage, kCarry>(a, threads, shm, s); break;
    case 4: launch_integrate_vk<V, 4, kStage, kCarry>(a, threads, shm, s); break;
    case 6: launch_integrate_vk<V, 6, kStage, kCarry>(a, threads, shm, s); break;
    case 8: launch_integrate_vk<V, 8, kStage, kCarry>(a, threads, shm, s); break;
    default: launch_integrate_vk<V, 0, kStage, kCarry>(a, threads, shm, s); break;
  }
}

template <int V>
static void launch_integrate_staged(const IntegrateArgs &a, uint32_t threads, hipStream_t s) {
  const size_t shm = integrate_lds_bytes<V>(threads, a.ppb, a.D, true);
  if (a.carry)
    launch_integrate_v<V, true, 1>(a, threads, shm, s);
  else
    launch_integrate_v<V, true, 0>(a, threads, shm, s);
}

// The volume stream goes through LDS (integrate_tile's kStage) where the
// launch shape allows it: 4 or 8 bins per thread, 16 pixels per wavefront
// row, whole groups of 4 chunks per wavefront, and the LDS within 64 KB.
template <int V>
static bool stage_fits(const IntegrateArgs &a, uint32_t threads) {
  return a.pw_shift == 4 && a.cpp % 4 == 0 && threads % 64 == 0 &&
         integrate_lds_bytes<V>(threads, a.ppb, a.D, true) <= 65536;
}

int launch_integrate(const IntegrateArgs &a, int V, uint32_t threads, hipStream_t s) {
  KernelTimer t("integrate", s);
  if (V == 8 && stage_fits<8>(a, threads))
    launch_integrate_staged<8>(a, threads, s);
  else if (V == 4 && stage_fits<4>(a, threads))
    launch_integrate_staged<4>(a, threads, s);
  else {
    const size_t shm = integrate_lds_head(threads, a.ppb);
    if (V == 8)
      launch_integrate_v<8, false, -1>(a, threads, shm, s);
    else if (V == 4)
      launch_integrate_v<4, false, -1>(a, threads, shm, s);
    else if (V == 2)
      launch_integrate_v<2, false, -1>(a, threads, shm, s);
    else
      launch_integrate_v<1, false, -1>(a, threads, shm, s);
  }
  return check_hip(hipGetLastError(), "integrate_kernel");
}

// ---------------------------------------------------------------------------
// standalone extraction: same thread layout, reads F and W.

template <int V>
__global__ __launch_bounds__(1024) void extract_kernel(ExtractArgs a) {
  extern __shared__ float smem[];
  float *sF = smem;
  float *sW = smem + blockDim.x;
  int *sBest = reinterpret_cast<int *>(smem + 2 * blockDim.x);
  const uint32_t t = threadIdx.x;
  const uint32_t lp = fdiv(t, a.cpp_div);
  const uint32_t chunk = t - lp * a.cpp;
  const uint32_t tile = xcd_tile(blockIdx.x, a.nblocks);
  const uint32_t pix = tile * a.ppb + lp;
  const bool active = pix < a.npix;
  const int d0 = (int)chunk * V;
  float F[V], W[V];  // launched with exactly ppb * cpp threads: every lane used
  if (active) {
    loadv<V>(a.F + (size_t)pix * a.D + d0, F);
    loadv<V>(a.W + (size_t)pix * a.D + d0, W);
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) F[v] = W[v] = 0.0f;
  }
  const int D = a.D;
  const float zn = a.z_near, zf = a.z_far;
  extract_block<V>(F, W, true, active, pix, lp, chunk, a.cpp, 1u, d0, D, sF, sW, sBest, a.out_depth,
                   a.out_bin, [D, zn, zf](int d) { return bin_depth(d, D, zn, zf); });
}

int launch_extract(const ExtractArgs &a, int V, uint32_t threads, hipStream_t s) {
  KernelTimer t("extract", s);
  const size_t shm = sizeof(float) * 2 * threads + sizeof(int) * a.ppb;
  if (V == 8)
    hipLaunchKernelGGL(extract_kernel<8>, dim3(a.nblocks), dim3(threads), shm, s, a);
  else if (V == 4)
    hipLaunchKernelGGL(extract_kernel<4>, dim3(a.nblocks), dim3(threads), shm, s, a);
  else if (V == 2)
    hipLaunchKernelGGL(extract_kernel<2>, dim3(a.nblocks), dim3(threads), shm, s, a);
  else
    hipLaunchKernelGGL(extract_kernel<1>, dim3(a.nblocks), dim3(threads), shm, s, a);
  return check_hip(hipGetLastError(), "extract_kernel");
}

// Adjoint of the interpolation z* = z_d + (z_{d+1} - z_d) F_d / (F_d - F_{d+1}).
__global__ void extract_backward_kernel(ExtractArgs a) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.npix) return;
  const int d = a.bin[p];
  float2 out = make_float2(0.0f, 0.0f);
  if (d >= 0 && d < a.D - 1) {
    const float f0 = a.F[(size_t)p * a.D + d], f1 = a.F[(size_t)p * a.D + d + 1];
    const float za = bin_depth(d, a.D, a.z_near, a.z_far);
    const float zb = bin_depth(d + 1, a.D, a.z_near, a.z_far);
    const float dz = zb - za, delta = f0 - f1, g = a.g_depth[p];
    out.x = g * ((-dz * f1) / (delta * delta));
    out.y = g * ((dz * f0) / (delta * delta));
  }
  reinterpret_cast<float2 *>(a.g_F2)[p] = out;
}

int launch_extract_backward(const ExtractArgs &a, hipStream_t s) {
  KernelTimer t("extract_backward", s);
  hipLaunchKernelGGL(extract_backward_kernel, dim3((a.npix + 255) / 256), dim3(256), 0, s, a);
  return check_hip(hipGetLastError(), "extract_backward_kernel");
}

// ---------------------------------------------------------------------------
// adjoint of the fusion.  (1) per pixel with a crossing, bound |contribution|
// of its two voxels' per-view terms from the voxels alone; (2) recompute the
// terms and scatter them into per-source-pixel 64-bit fixed-point
// accumulators scaled by that bound (integer addition is associative: the
// result does not depend on arrival order); (3) chain the weight gradient
// through nu of its window; (4) gather the window terms.

__global__ void zero_u64_kernel(unsigned long long *p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// Calls f(k, q, dD, dw) for each view sample of voxel (pix, d) whose
// contribution is live, with dD = dL/dD_k[q] through the clamp and
// dw = dL/domega_k[q].
template <typename Fn>
__device__ __forceinline__ void voxel_adjoint(const TsdfBackArgs &a, uint32_t pix, int d, float gF,
                                              Fn f) {
  const uint32_t y = fdiv(pix, a.wt_div), x = pix - y * a.wt_div.d;
  const float px = (float)x + 0.5f, py = (float)y + 0.5f;
  const float2 b = a.bins[d];
  const float z = b.x, tau = b.y;
  const size_t o = (size_t)pix * a.D + d;
  const float Wn = a.W[o], Fv = a.F[o];
  const float fWs = (float)a.Ws, fHs = (float)a.Hs;
  for (int k = 0; k < a.K; ++k) {
    const Proj &P = a.views[k];
    float h0, h1, h2;
    ray_of(P, px, py, h0, h1, h2);
    const float X0 = fmaf(z, h0, P.c[0]), X1 = fmaf(z, h1, P.c[1]), Z = fmaf(z, h2, P.c[2]);
    if (!(Z > 0.0f)) continue;
    const float inv = 1.0f / Z;
    const float u = X0 * inv, w = X1 * inv;
    if (!(u >= 0.0f && u < fWs && w >= 0.0f && w < fHs)) continue;
    const uint32_t q = (uint32_t)w * (uint32_t)a.Ws + (uint32_t)u;
    const float2 e = a.table[(size_t)k * table_view_records(a.Ws, a.Hs) +
                             (size_t)(uint32_t)w * table_pitch(a.Ws) + (uint32_t)u];
    const float s = e.x - Z;
    if (s < -tau) continue;
    const float c = fminf(s, tau);
    const float dD = (s < tau) ? (gF * e.y) / Wn : 0.0f;
    const float dw = (gF * (c - Fv)) / Wn;
    f(k, q, dD, dw);
  }
}

// An upper bound on |dD| and |dw| over every view sample of the pixel's two
// voxels, from the voxel alone: the table weight is at most 1 and the clamp
// keeps |c| <= tau, so |dD| <= |gF| / W and |dw| <= |gF| (tau + |F|) / W.
// Rounding is monotone, so the bound evaluated in FP32 also bounds the
// FP32 terms voxel_adjoint computes.
__device__ __forceinline__ float voxel_bound(const TsdfBackArgs &a, uint32_t pix, int d,
                                             float gF) {
  const size_t o = (size_t)pix * a.D + d;
  const float Wn = gmem(a.W)[o], Fv = gmem(a.F)[o];
  const float tau = gload2(a.bins + d).y, ag = fabsf(gF);
  return fmaxf(ag / Wn, (ag * (tau + fabsf(Fv))) / Wn);
}

__global__ __launch_bounds__(256) void tsdf_bwd_max_kernel(TsdfBackArgs a) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  float m = 0.0f;
  if (p < a.npix) {
    const int d = gmem(a.bin)[p];
    if (d >= 0) {
      const float2 g = reinterpret_cast<const float2 *>(a.g_F2)[p];
      m = fmaxf(voxel_bound(a, p, d, g.x), voxel_bound(a, p, d + 1, g.y));
    }
  }
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  __shared__ float red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    float r = red[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = fmaxf(r, red[i]);
    atomicMax(a.maxbits, __float_as_uint(r));  // non-negative floats order as integers
  }
}

// Fixed-point exponent: every accumulated sum stays below 2^61 in magnitude.
__device__ __forceinline__ int fixed_exponent(const TsdfBackArgs &a) {
  const float m = __uint_as_float(*a.maxbits);
  if (!(m > 0.0f)) return INT_MIN;
  int e;
  frexp((double)m * 2.0 * (double)a.npix, &e);
  return 61 - e;
}

__device__ __forceinline__ unsigned long long to_fixed(float v, int E) {
  return (unsigned long long)(long long)llrint(ldexp((double)v, E));
}

__global__ __launch_bounds__(256) void tsdf_bwd_scatter_kernel(TsdfBackArgs a) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.npix) return;
  const int d = a.bin[p];
  if (d < 0) return;
  const int E = fixed_exponent(a);
  if (E == INT_MIN) return;
  const float2 g = reinterpret_cast<const float2 *>(a.g_F2)[p];
  auto sc = [&](int k, uint32_t q, float dD, float dw) {
    const size_t i = (size_t)k * a.ns + q;
    if (dD != 0.0f) atomicAdd(&a.acc_D[i], to_fixed(dD, E));
    if (dw != 0.0f) atomicAdd(&a.acc_w[i], to_fixed(dw, E));
  };
  voxel_adjoint(a, p, d, g.x, sc);
  voxel_adjoint(a, p, d + 1, g.y, sc);
}

__device__ __forceinline__ float from_fixed(unsigned long long v, int E) {
  return (float)ldexp((double)(long long)v, -E);
}

// The window parameters of the backward as the confidence kernel's record,
// so both share the tile staging and the window statistic.
__device__ __forceinline__ ConfArgs conf_of(const TsdfBackArgs &a) {
  ConfArgs c{};
  c.depth = a.depth;
  c.Ws = a.Ws;
  c.Hs = a.Hs;
  c.K = a.K;
  c.radius = a.radius;
  c.tw2 = a.tw2;
  c.n2 = a.n2;
  c.scale = a.scale;
  return c;
}

// dL/dnu at each source pixel: dL/domega * domega/dnu where the min(., 1)
// of the weight is inactive and nu > 0.  nu is the confidence kernel's
// window statistic (same tile staging, same terms in the same order); one
// 32 x 8 tile of view blockIdx.z per workgroup.
__global__ __launch_bounds__(256) void tsdf_bwd_nu_kernel(TsdfBackArgs a) {
  __shared__ float tile[kConfLH * kConfLW];
  const ConfArgs c = conf_of(a);
  const int k = blockIdx.z, i0 = blockIdx.x * kConfTX, j0 = blockIdx.y * kConfTY;
  stage_tile(tile, a.depth + (size_t)k * a.ns, i0, j0, c);
  __syncthreads();
  const int lx = threadIdx.x & (kConfTX - 1), ly = threadIdx.x / kConfTX;
  const int i = i0 + lx, j = j0 + ly;
  const bool interior = i0 >= a.radius && j0 >= a.radius && i0 + kConfTX + a.radius <= a.Ws &&
                        j0 + kConfTY + a.radius <= a.Hs;
  if (ly >= kConfTY || i >= a.Ws || j >= a.Hs) return;
  const size_t o = (size_t)k * a.ns + (size_t)j * a.Ws + i;
  const int E = fixed_exponent(a);
  float out = 0.0f;
  const float gw = (E == INT_MIN) ? 0.0f : from_fixed(a.acc_w[o], E);
  const int li = lx + kMaxR, lj = ly + kMaxR;
  const float dq = tile[lj * kConfLW + li];  // NaN for a hole
  if (gw != 0.0f && depth_ok(dq)) {
    const float nu = interior ? window_nu_fast(tile, li, lj, dq, c)
                              : window_nu(tile, li, lj, i, j, dq, c);
    if (nu > 0.0f) {
      const float raw = a.scale / sqrtf(nu / a.n2);
      if (raw < 1.0f) out = gw * ((-0.5f * raw) / nu);
    }
  }
  gmem(a.gnu)[o] = out;
}

// The window terms of g_depth_in for a pixel r with a usable depth dr, in
// row-major order over the window without its centre: r as the centre
// (gr = gnu_r) and r as a neighbour of each n (gq = gnu_n).  Bounds-checked
// form; holes in `tile` are NaN and fail depth_ok.
__device__ __forceinline__ float finish_window(const float *tile, const float *gtile, int li,
                                               int lj, int i, int j, float dr, float gr, float g,
                                               const TsdfBackArgs &a) {
  for (int dy = -a.radius; dy <= a.radius; ++dy) {
    const int jj = j + dy;
    if (jj < 0 || jj >= a.Hs) continue;
    for (int dx = -a.radius; dx <= a.radius; ++dx) {
      const int ii = i + dx;
      if (ii < 0 || ii >= a.Ws || (dx == 0 && dy == 0)) continue;
      const int l = (lj + dy) * kConfLW + (li + dx);
      const float dn = tile[l];
      if (!depth_ok(dn)) continue;
      const float dd = dr - dn;
      if (dd * dd < a.tw2) {
        if (gr != 0.0f) g += gr * 2.0f * dd;
        const float gq = gtile[l];
        if (gq != 0.0f) g -= gq * 2.0f * (dn - dr);
      }
    }
  }
  return g;
}

// The same for a pixel whose window lies inside the image: a hole's NaN
// makes dd NaN and fails dd^2 < tau^2, exactly as the hole test skips it.
template <int R>
__device__ __forceinline__ float finish_window_interior(const float *tile, const float *gtile,
                                                        int li, int lj, float dr, float gr,
                                                        float g, float tw2) {
#pragma unroll
  for (int dy = -R; dy <= R; ++dy)
#pragma unroll
    for (int dx = -R; dx <= R; ++dx) {
      if (dx == 0 && dy == 0) continue;
      const int l = (lj + dy) * kConfLW + (li + dx);
      const float dn = tile[l];
      const float dd = dr - dn;
      if (dd * dd < tw2) {
        if (gr != 0.0f) g += gr * 2.0f * dd;
        const float gq = gtile[l];
        if (gq != 0.0f) g -= gq * 2.0f * (dn - dr);
      }
    }
  return g;
}

__device__ __forceinline__ float finish_window_fast(const float *tile, const float *gtile, int li,
                                                    int lj, float dr, float gr, float g,
                                                    const TsdfBackArgs &a) {
  switch (a.radius) {
    case 0: return finish_window_interior<0>(tile, gtile, li, lj, dr, gr, g, a.tw2);
    case 1: return finish_window_interior<1>(tile, gtile, li, lj, dr, gr, g, a.tw2);
    case 2: return finish_window_interior<2>(tile, gtile, li, lj, dr, gr, g, a.tw2);
    case 3: return finish_window_interior<3>(tile, gtile, li, lj, dr, gr, g, a.tw2);
    case 4: return finish_window_interior<4>(tile, gtile, li, lj, dr, gr, g, a.tw2);
    case 5: return finish_window_interior<5>(tile, gtile, li, lj, dr, gr, g, a.tw2);
    case 6: return finish_window_interior<6>(tile, gtile, li, lj, dr, gr, g, a.tw2);
    default: return finish_window_interior<kMaxR>(tile, gtile, li, lj, dr, gr, g, a.tw2);
  }
}

// g_depth_in[r] = direct (fixed point) + window terms of r as a centre and
// as a neighbour of each q in its window; one 32 x 8 tile of view
// blockIdx.z per workgroup, depths and gnu staged in LDS with the halo.
__global__ __launch_bounds__(256) void tsdf_bwd_finish_kernel(TsdfBackArgs a) {
  __shared__ float tile[kConfLH * kConfLW];
  __shared__ float gtile[kConfLH * kConfLW];
  const ConfArgs c = conf_of(a);
  const int k = blockIdx.z, i0 = blockIdx.x * kConfTX, j0 = blockIdx.y * kConfTY;
  stage_tile(tile, a.depth + (size_t)k * a.ns, i0, j0, c);
  stage_rows<false>(gtile, a.gnu + (size_t)k * a.ns, i0, j0, c);
  __syncthreads();
  const int lx = threadIdx.x & (kConfTX - 1), ly = threadIdx.x / kConfTX;
  const int i = i0 + lx, j = j0 + ly;
  const bool interior = i0 >= a.radius && j0 >= a.radius && i0 + kConfTX + a.radius <= a.Ws &&
                        j0 + kConfTY + a.radius <= a.Hs;
  if (ly >= kConfTY || i >= a.Ws || j >= a.Hs) return;
  const size_t o = (size_t)k * a.ns + (size_t)j * a.Ws + i;
  const int E = fixed_exponent(a);
  float g = (E == INT_MIN) ? 0.0f : from_fixed(a.acc_D[o], E);
  const int li = lx + kMaxR, lj = ly + kMaxR;
  const float dr = tile[lj * kConfLW + li];
  if (depth_ok(dr)) {
    const float gr = gtile[lj * kConfLW + li];
    g = interior ? finish_window_fast(tile, gtile, li, lj, dr, gr, g, a)
                 : finish_window(tile, gtile, li, lj, i, j, dr, gr, g, a);
  }
  gmem(a.g_depth_in)[o] = g;
}

int launch_tsdf_backward(const TsdfBackArgs &a, hipStream_t s) {
  {
    KernelTimer t("tsdf_bwd_zero", s);
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1024), dim3(256), 0, s, a.acc_D,
                       (size_t)a.K * a.ns * 2 + 1);
    if (int rc = check_hip(hipGetLastError(), "zero_u64_kernel")) return rc;
  }
  const dim3 gp((a.npix + 255) / 256);
  {
    KernelTimer t("tsdf_bwd_max", s);
    hipLaunchKernelGGL(tsdf_bwd_max_kernel, gp, dim3(256), 0, s, a);
    if (int rc = check_hip(hipGetLastError(), "tsdf_bwd_max_kernel")) return rc;
  }
  {
    KernelTimer t("tsdf_bwd_scatter", s);
    hipLaunchKernelGGL(tsdf_bwd_scatter_kernel, gp, dim3(256), 0, s, a);
    if (int rc = check_hip(hipGetLastError(), "tsdf_bwd_scatter_kernel")) return rc;
  }
  const dim3 gt((a.Ws + kConfTX - 1) / kConfTX, (a.Hs + kConfTY - 1) / kConfTY, a.K);
  {
    KernelTimer t("tsdf_bwd_nu", s);
    hipLaunchKernelGGL(tsdf_bwd_nu_kernel, gt, dim3(kConfTX * kConfTY), 0, s, a);
    if (int rc = check_hip(hipGetLastError(), "tsdf_bwd_nu_kernel")) return rc;
  }
  KernelTimer t("tsdf_bwd_finish", s);
  hipLaunchKernelGGL(tsdf_bwd_finish_kernel, gt, dim3(kConfTX * kConfTY), 0, s, a);
  return check_hip(hipGetLastError(), "tsdf_bwd_finish_kernel");
}

// ---------------------------------------------------------------------------
// self-check of the fast reciprocal against IEEE division (test hook)

__global__ void recip_selftest_kernel(uint32_t e_lo, uint32_t n_exp,
                                      unsigned long long *mismatches) {
  const uint64_t n = (uint64_t)n_exp << 23;
  unsigned long long bad = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t bits = ((e_lo + (uint32_t)(i >> 23)) << 23) | (uint32_t)(i & 0x7fffffu);
    const float z = __uint_as_float(bits);
    const float a = recip_rn(z);
    const float b = 1.0f / z;
    bad += (__float_as_uint(a) != __float_as_uint(b)) ? 1ull : 0ull;
  }
  for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off);
  if ((threadIdx.x & 63) == 0 && bad) atomicAdd(mismatches, bad);
}

__global__ void fast_recip_kernel(const float *in, float *out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = recip_pos(in[i]);
}

int launch_recip_selftest(uint32_t e_lo, uint32_t n_exp, unsigned long long *mismatches,
                          hipStream_t s) {
  hipLaunchKernelGGL(recip_selftest_kernel, dim3(2048), dim3(256), 0, s, e_lo, n_exp, mismatches);
  return check_hip(hipGetLastError(), "recip_selftest_kernel");
}

int launch_fast_recip(const float *in, float *out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fast_recip_kernel, dim3(1024), dim3(256), 0, s, in, out, n);
  return check_hip(hipGetLastError(), "fast_recip_kernel");
}

}  // namespace gg
