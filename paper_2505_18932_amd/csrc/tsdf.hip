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
#include <climits>

#include "ggeom_internal.h"

namespace gg {

// ---------------------------------------------------------------------------
// depth bins: z_d = 1 / (1/z_near - d du), tau_d = trunc du z_d^2 (in bins)

__device__ __forceinline__ float bin_depth(int d, int D, float z_near, float z_far) {
  const float un = 1.0f / z_near;
  const float uf = 1.0f / z_far;
  const float du = (un - uf) / (float)(D - 1);
  const float u = un - (float)d * du;
  return 1.0f / u;
}

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

__device__ __forceinline__ void stage_tile(float *tile, const float *dk, int i0, int j0,
                                           const ConfArgs &a) {
  const int r = a.radius;
  const int tw = kConfTX + 2 * r, th = kConfTY + 2 * r;
  for (int e = threadIdx.x; e < tw * th; e += blockDim.x) {
    const int ly = e / tw, lx = e - ly * tw;
    const int gi = i0 - r + lx, gj = j0 - r + ly;
    float v = 0.0f;
    if (gi >= 0 && gi < a.Ws && gj >= 0 && gj < a.Hs) v = dk[(size_t)gj * a.Ws + gi];
    // stored at (ly + kMaxR - r, lx + kMaxR - r) so that window offsets are
    // relative to the fixed centre origin
    tile[(ly + kMaxR - r) * kConfLW + (lx + kMaxR - r)] = v;
  }
}

__global__ __launch_bounds__(256) void conf_kernel(ConfArgs a) {
  __shared__ float tile[kConfLH * kConfLW];
  const int k = blockIdx.z;
  const int i0 = blockIdx.x * kConfTX, j0 = blockIdx.y * kConfTY;
  const float *dk = a.depth + (size_t)k * a.Ws * a.Hs;
  stage_tile(tile, dk, i0, j0, a);
  __syncthreads();
  const int lx = threadIdx.x & (kConfTX - 1), ly = threadIdx.x / kConfTX;
  const int i = i0 + lx, j = j0 + ly;
  if (i >= a.Ws || j >= a.Hs) return;
  const int li = lx + kMaxR, lj = ly + kMaxR;
  const float dq = tile[lj * kConfLW + li];
  float2 rec = make_float2(-INFINITY, 0.0f);
  if (depth_ok(dq)) {
    const float nu = window_nu(tile, li, lj, i, j, dq, a);
    const float om = (nu == 0.0f) ? 1.0f : fminf(a.scale / sqrtf(nu / a.n2), 1.0f);
    rec = make_float2(dq, om);
  }
  a.table[(size_t)k * a.Ws * a.Hs + (size_t)j * a.Ws + i] = rec;
}

int launch_conf(const ConfArgs &a, hipStream_t s) {
  KernelTimer t("conf", s);
  dim3 grid((a.Ws + kConfTX - 1) / kConfTX, (a.Hs + kConfTY - 1) / kConfTY, a.K);
  hipLaunchKernelGGL(conf_kernel, grid, dim3(kConfTX * kConfTY), 0, s, a);
  return check_hip(hipGetLastError(), "conf_kernel");
}

// ---------------------------------------------------------------------------
// vector access of V consecutive floats (V = 4, 2, 1)

template <int V>
__device__ __forceinline__ void loadv(const float *p, float (&o)[V]) {
  if constexpr (V == 4) {
    const float4 v = *reinterpret_cast<const float4 *>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  } else if constexpr (V == 2) {
    const float2 v = *reinterpret_cast<const float2 *>(p);
    o[0] = v.x; o[1] = v.y;
  } else {
    o[0] = *p;
  }
}

template <int V>
__device__ __forceinline__ void storev(float *p, const float (&o)[V]) {
  if constexpr (V == 4) {
    *reinterpret_cast<float4 *>(p) = make_float4(o[0], o[1], o[2], o[3]);
  } else if constexpr (V == 2) {
    *reinterpret_cast<float2 *>(p) = make_float2(o[0], o[1]);
  } else {
    *p = o[0];
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
                                              bool active, uint32_t pix, uint32_t lp,
                                              uint32_t chunk, uint32_t cpp, int d0, int D,
                                              float *sF, float *sW, int *sBest,
                                              float *out_depth, int32_t *out_bin, ZF zf) {
  const uint32_t t = threadIdx.x;
  sF[t] = F[0];
  sW[t] = W[0];
  if (chunk == 0) sBest[lp] = INT_MAX;
  __syncthreads();
  const bool has_next = chunk + 1 < cpp;
  const float nF = has_next ? sF[t + 1] : 0.0f;
  const float nW = has_next ? sW[t + 1] : 0.0f;
  if (active) {
    const int cand = local_crossing<V>(F, W, nF, nW, d0, D);
    if (cand != INT_MAX) atomicMin(&sBest[lp], cand);
  }
  __syncthreads();
  if (!active) return;
  const int best = sBest[lp];
  if (best == INT_MAX) {
    if (chunk == 0) {
      out_depth[pix] = 0.0f;
      out_bin[pix] = -1;
    }
    return;
  }
#pragma unroll
  for (int v = 0; v < V; ++v) {
    if (best == d0 + v) {
      const float f0 = F[v];
      const float f1 = (v + 1 < V) ? F[(v + 1) % V] : nF;
      const float za = zf(best), zb = zf(best + 1);
      const float frac = f0 / (f0 - f1);
      out_depth[pix] = za + (zb - za) * frac;
      out_bin[pix] = best;
    }
  }
}

// ---------------------------------------------------------------------------
// fused integrate + extraction.  Workgroup = ppb whole pixels; thread = V
// consecutive bins of one pixel (the volume is D-innermost, so a wavefront
// reads and writes one contiguous span of F and W: fully coalesced).

template <int V>
__global__ __launch_bounds__(1024) void integrate_kernel(IntegrateArgs a) {
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

  float z[V], tau[V], S[V], Wo[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const float2 b = a.bins[d0 + v];
    z[v] = b.x;
    tau[v] = b.y;
    S[v] = 0.0f;
    Wo[v] = 0.0f;
  }
  float Fn[V], Wn[V];
  if (active) {
    const uint32_t y = fdiv(pix, a.wt_div);
    const uint32_t x = pix - y * a.wt_div.d;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const float fWs = (float)a.Ws, fHs = (float)a.Hs;
    for (int k = 0; k < a.K; ++k) {
      const Proj &P = a.views[k];
      float h0, h1, h2;
      ray_of(P, px, py, h0, h1, h2);
      const float2 *tab = a.table + (size_t)k * a.ns;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const float X0 = fmaf(z[v], h0, P.c[0]);
        const float X1 = fmaf(z[v], h1, P.c[1]);
        const float Z = fmaf(z[v], h2, P.c[2]);
        if (Z > 0.0f) {
          const float inv = 1.0f / Z;
          const float u = X0 * inv, w = X1 * inv;
          if (u >= 0.0f && u < fWs && w >= 0.0f && w < fHs) {
            const float2 e = tab[(uint32_t)w * (uint32_t)a.Ws + (uint32_t)u];
            const float s = e.x - Z;  // -inf for a hole: dropped below
            if (!(s < -tau[v])) {
              const float c = fminf(s, tau[v]);
              S[v] = fmaf(e.y, c, S[v]);
              Wo[v] = Wo[v] + e.y;
            }
          }
        }
      }
    }
    const size_t base = (size_t)pix * a.D + d0;
    float Fp[V], Wp[V];
    if (a.carry) {
      loadv<V>(a.F_prev + base, Fp);
      loadv<V>(a.W_prev + base, Wp);
    }
    const float m = a.mask ? fmaxf(1.0f - a.mask[pix], 0.0f) : 1.0f;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const float wp = a.carry ? fminf((a.decay * Wp[v]) * m, a.cap) : 0.0f;
      const float Fpv = a.carry ? Fp[v] : 0.0f;
      const float wn = wp + Wo[v];
      Fn[v] = (wn > 0.0f) ? fmaf(wp, Fpv, S[v]) / wn : 0.0f;
      Wn[v] = wn;
    }
    storev<V>(a.F + base, Fn);
    storev<V>(a.W + base, Wn);
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) Fn[v] = Wn[v] = 0.0f;
  }
  if (a.out_depth) {
    const float2 *bins = a.bins;
    extract_block<V>(Fn, Wn, active, pix, lp, chunk, a.cpp, d0, a.D, sF, sW, sBest, a.out_depth,
                     a.out_bin, [bins](int d) { return bins[d].x; });
  }
}

int launch_integrate(const IntegrateArgs &a, int V, uint32_t threads, hipStream_t s) {
  KernelTimer t("integrate", s);
  const size_t shm = sizeof(float) * 2 * threads + sizeof(int) * a.ppb;
  if (V == 4)
    hipLaunchKernelGGL(integrate_kernel<4>, dim3(a.nblocks), dim3(threads), shm, s, a);
  else if (V == 2)
    hipLaunchKernelGGL(integrate_kernel<2>, dim3(a.nblocks), dim3(threads), shm, s, a);
  else
    hipLaunchKernelGGL(integrate_kernel<1>, dim3(a.nblocks), dim3(threads), shm, s, a);
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
  float F[V], W[V];
  if (active) {
    loadv<V>(a.F + (size_t)pix * a.D + d0, F);
    loadv<V>(a.W + (size_t)pix * a.D + d0, W);
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) F[v] = W[v] = 0.0f;
  }
  const int D = a.D;
  const float zn = a.z_near, zf = a.z_far;
  extract_block<V>(F, W, active, pix, lp, chunk, a.cpp, d0, D, sF, sW, sBest, a.out_depth,
                   a.out_bin, [D, zn, zf](int d) { return bin_depth(d, D, zn, zf); });
}

int launch_extract(const ExtractArgs &a, int V, uint32_t threads, hipStream_t s) {
  KernelTimer t("extract", s);
  const size_t shm = sizeof(float) * 2 * threads + sizeof(int) * a.ppb;
  if (V == 4)
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
// adjoint of the fusion.  (1) per pixel with a crossing, recompute the two
// voxels' per-view terms and find max |contribution|; (2) scatter them into
// per-source-pixel 64-bit fixed-point accumulators (integer addition is
// associative: the result does not depend on arrival order); (3) chain the
// weight gradient through nu of its window; (4) gather the window terms.

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
    const float2 e = a.table[(size_t)k * a.ns + q];
    const float s = e.x - Z;
    if (s < -tau) continue;
    const float c = fminf(s, tau);
    const float dD = (s < tau) ? (gF * e.y) / Wn : 0.0f;
    const float dw = (gF * (c - Fv)) / Wn;
    f(k, q, dD, dw);
  }
}

__global__ __launch_bounds__(256) void tsdf_bwd_max_kernel(TsdfBackArgs a) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  float m = 0.0f;
  if (p < a.npix) {
    const int d = a.bin[p];
    if (d >= 0) {
      const float2 g = reinterpret_cast<const float2 *>(a.g_F2)[p];
      voxel_adjoint(a, p, d, g.x, [&](int, uint32_t, float dD, float dw) {
        m = fmaxf(m, fmaxf(fabsf(dD), fabsf(dw)));
      });
      voxel_adjoint(a, p, d + 1, g.y, [&](int, uint32_t, float dD, float dw) {
        m = fmaxf(m, fmaxf(fabsf(dD), fabsf(dw)));
      });
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

// dL/dnu at each source pixel: dL/domega * domega/dnu where the min(., 1)
// of the weight is inactive and nu > 0.
__global__ __launch_bounds__(256) void tsdf_bwd_nu_kernel(TsdfBackArgs a) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i >= a.ns) return;
  const size_t o = (size_t)k * a.ns + i;
  const int E = fixed_exponent(a);
  float out = 0.0f;
  const float gw = (E == INT_MIN) ? 0.0f : from_fixed(a.acc_w[o], E);
  const float *dk = a.depth + (size_t)k * a.ns;
  const float dq = dk[i];
  if (gw != 0.0f && depth_ok(dq)) {
    const int qy = (int)(i / (uint32_t)a.Ws), qx = (int)(i - (uint32_t)qy * a.Ws);
    float nu = 0.0f;
    for (int dy = -a.radius; dy <= a.radius; ++dy) {
      const int jj = qy + dy;
      if (jj < 0 || jj >= a.Hs) continue;
      for (int dx = -a.radius; dx <= a.radius; ++dx) {
        const int ii = qx + dx;
        if (ii < 0 || ii >= a.Ws) continue;
        const float dn = dk[(size_t)jj * a.Ws + ii];
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
    if (nu > 0.0f) {
      const float raw = a.scale / sqrtf(nu / a.n2);
      if (raw < 1.0f) out = gw * ((-0.5f * raw) / nu);
    }
  }
  a.gnu[o] = out;
}

// g_depth_in[r] = direct (fixed point) + window terms of r as a centre and
// as a neighbour of each q in its window.
__global__ __launch_bounds__(256) void tsdf_bwd_finish_kernel(TsdfBackArgs a) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i >= a.ns) return;
  const size_t o = (size_t)k * a.ns + i;
  const int E = fixed_exponent(a);
  float g = (E == INT_MIN) ? 0.0f : from_fixed(a.acc_D[o], E);
  const float *dk = a.depth + (size_t)k * a.ns;
  const float *gn = a.gnu + (size_t)k * a.ns;
  const float dr = dk[i];
  if (depth_ok(dr)) {
    const int ry = (int)(i / (uint32_t)a.Ws), rx = (int)(i - (uint32_t)ry * a.Ws);
    const float gr = gn[i];
    for (int dy = -a.radius; dy <= a.radius; ++dy) {
      const int jj = ry + dy;
      if (jj < 0 || jj >= a.Hs) continue;
      for (int dx = -a.radius; dx <= a.radius; ++dx) {
        const int ii = rx + dx;
        if (ii < 0 || ii >= a.Ws || (dx == 0 && dy == 0)) continue;
        const size_t n = (size_t)jj * a.Ws + ii;
        const float dn = dk[n];
        if (!depth_ok(dn)) continue;
        const float dd = dr - dn;  // r as the centre
        if (dd * dd < a.tw2) {
          if (gr != 0.0f) g += gr * 2.0f * dd;
          const float gq = gn[n];  // r as a neighbour of n: d(nu_n)/dD_r = -2 (D_n - D_r)
          if (gq != 0.0f) g -= gq * 2.0f * (dn - dr);
        }
      }
    }
  }
  a.g_depth_in[o] = g;
}

int launch_tsdf_backward(const TsdfBackArgs &a, hipStream_t s) {
  {
    KernelTimer t("tsdf_bwd_zero", s);
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1024), dim3(256), 0, s, a.acc_D,
                       (size_t)a.K * a.ns * 2 + 1);
    if (int rc = check_hip(hipGetLastError(), "zero_u64_kernel")) return rc;
  }
  const dim3 gp((a.npix + 255) / 256), gs((a.ns + 255) / 256, a.K);
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
  {
    KernelTimer t("tsdf_bwd_nu", s);
    hipLaunchKernelGGL(tsdf_bwd_nu_kernel, gs, dim3(256), 0, s, a);
    if (int rc = check_hip(hipGetLastError(), "tsdf_bwd_nu_kernel")) return rc;
  }
  KernelTimer t("tsdf_bwd_finish", s);
  hipLaunchKernelGGL(tsdf_bwd_finish_kernel, gs, dim3(256), 0, s, a);
  return check_hip(hipGetLastError(), "tsdf_bwd_finish_kernel");
}

}  // namespace gg
