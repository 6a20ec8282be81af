// Inputs of the blending network (§3.3; the supplement's list of network
// inputs) and the blend of Eq. 4-5 for given weights.  One thread per target
// pixel; every plane is written coalesced (plane-major, pixel-minor).  The
// per-pixel geometry follows the FP32 operation order stated in the header.
#include "ggeom_internal.h"

namespace gg {

__device__ __forceinline__ float dot3(const float a[3], const float b[3]) {
  return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

__device__ __forceinline__ void surface_point(const NetArgs &a, int i, int j, float D, float X[3]) {
  float h0, h1, h2;
  ray_of(a.M, (float)i + 0.5f, (float)j + 0.5f, h0, h1, h2);
  X[0] = fmaf(D, h0, a.M.c[0]);
  X[1] = fmaf(D, h1, a.M.c[1]);
  X[2] = fmaf(D, h2, a.M.c[2]);
}

__global__ __launch_bounds__(256) void netinputs_kernel(NetArgs a) {
  const size_t n = (size_t)a.W * a.H;
  const int K = a.K;
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(p / (size_t)a.W), i = (int)(p - (size_t)j * a.W);
    GG_GLOBAL float *out = gmem(a.out);
    // copies: rendered images, depths, alphas, TSDF depth
    for (int c = 0; c < 3 * K; ++c) out[(size_t)c * n + p] = gmem(a.rgb)[(size_t)c * n + p];
    for (int k = 0; k < K; ++k) {
      out[(size_t)(3 * K + k) * n + p] = gmem(a.depth)[(size_t)k * n + p];
      out[(size_t)(4 * K + k) * n + p] = gmem(a.alpha)[(size_t)k * n + p];
    }
    const GG_GLOBAL float *td = gmem(a.tsdf_depth);
    const float D = td[p];
    out[(size_t)(5 * K) * n + p] = D;
    const bool ok = D > 0.0f;
    float X[3] = {0.0f, 0.0f, 0.0f}, nrm[3] = {0.0f, 0.0f, 0.0f};
    bool has_n = false;
    if (ok) {
      surface_point(a, i, j, D, X);
      const int ni[4] = {i - 1, i + 1, i, i}, nj[4] = {j, j, j - 1, j + 1};
      float P[4][3];
      bool v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        v[e] = ni[e] >= 0 && ni[e] < a.W && nj[e] >= 0 && nj[e] < a.H &&
               td[(size_t)nj[e] * a.W + ni[e]] > 0.0f;
        P[e][0] = P[e][1] = P[e][2] = 0.0f;
        if (v[e]) surface_point(a, ni[e], nj[e], td[(size_t)nj[e] * a.W + ni[e]], P[e]);
      }
      float tx[3], ty[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        tx[r] = v[0] && v[1] ? P[1][r] - P[0][r]
                             : (v[1] ? P[1][r] - X[r] : (v[0] ? X[r] - P[0][r] : 0.0f));
        ty[r] = v[2] && v[3] ? P[3][r] - P[2][r]
                             : (v[3] ? P[3][r] - X[r] : (v[2] ? X[r] - P[2][r] : 0.0f));
      }
      if ((v[0] || v[1]) && (v[2] || v[3])) {
        const float c3[3] = {tx[1] * ty[2] - tx[2] * ty[1], tx[2] * ty[0] - tx[0] * ty[2],
                             tx[0] * ty[1] - tx[1] * ty[0]};
        const float len = sqrtf(dot3(c3, c3));
        if (len > 0.0f) {
#pragma unroll
          for (int r = 0; r < 3; ++r) nrm[r] = c3[r] / len;
          const float tc[3] = {a.M.c[0] - X[0], a.M.c[1] - X[1], a.M.c[2] - X[2]};
          if (dot3(nrm, tc) < 0.0f) {
#pragma unroll
            for (int r = 0; r < 3; ++r) nrm[r] = -nrm[r];
          }
          has_n = true;
        }
      }
    }
    float h[3];
    ray_of(a.M, (float)i + 0.5f, (float)j + 0.5f, h[0], h[1], h[2]);
    const float hl = sqrtf(dot3(h, h));
    const float dt[3] = {h[0] / hl, h[1] / hl, h[2] / hl};
    for (int k = 0; k < K; ++k) {
      float dn = 0.0f, dd = 0.0f;
      if (ok) {
        float r3[3] = {X[0] - a.Cs[k][0], X[1] - a.Cs[k][1], X[2] - a.Cs[k][2]};
        const float rl = sqrtf(dot3(r3, r3));
        if (rl > 0.0f) {
#pragma unroll
          for (int r = 0; r < 3; ++r) r3[r] = r3[r] / rl;
          if (has_n) dn = dot3(r3, nrm);
          dd = dot3(r3, dt);
        }
      }
      out[(size_t)(5 * K + 1 + k) * n + p] = dn;
      out[(size_t)(6 * K + 1 + k) * n + p] = dd;
      out[(size_t)(7 * K + 1 + k) * n + p] = a.dist[k];
      out[(size_t)(8 * K + 1 + k) * n + p] = a.axd[k];
    }
  }
}

__global__ __launch_bounds__(256) void blend_kernel(BlendArgs a) {
  const size_t n = (size_t)a.W * a.H;
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x) {
    float num0 = 0.0f, num1 = 0.0f, num2 = 0.0f, numd = 0.0f, den = 0.0f;
    for (int k = 0; k < a.K; ++k) {
      const float aw = gmem(a.alpha)[(size_t)k * n + p] * gmem(a.w)[(size_t)k * n + p];
      num0 = fmaf(gmem(a.rgb)[(size_t)(3 * k + 0) * n + p], aw, num0);
      num1 = fmaf(gmem(a.rgb)[(size_t)(3 * k + 1) * n + p], aw, num1);
      num2 = fmaf(gmem(a.rgb)[(size_t)(3 * k + 2) * n + p], aw, num2);
      numd = fmaf(gmem(a.depth)[(size_t)k * n + p], aw, numd);
      den = den + aw;
    }
    const float wb = gmem(a.w_bg)[p];
    const float num[3] = {num0, num1, num2};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float fg = den > 0.0f ? num[c] / den : 0.0f;
      gmem(a.out_rgb)[(size_t)c * n + p] = fmaf(wb, gmem(a.rgb_bg)[(size_t)c * n + p],
                                               (1.0f - wb) * fg);
    }
    gmem(a.out_depth)[p] = den > 0.0f ? numd / den : 0.0f;
  }
}

static unsigned pixel_grid(size_t n) {
  const size_t b = (n + 255) / 256;
  return (unsigned)(b < 65536 ? (b ? b : 1) : 65536);
}

int launch_network_inputs(const NetArgs &a, hipStream_t s) {
  KernelTimer t("network_inputs", s);
  hipLaunchKernelGGL(netinputs_kernel, dim3(pixel_grid((size_t)a.W * a.H)), dim3(256), 0, s, a);
  return check_hip(hipGetLastError(), "netinputs_kernel");
}

int launch_blend(const BlendArgs &a, hipStream_t s) {
  KernelTimer t("blend", s);
  hipLaunchKernelGGL(blend_kernel, dim3(pixel_grid((size_t)a.W * a.H)), dim3(256), 0, s, a);
  return check_hip(hipGetLastError(), "blend_kernel");
}

}  // namespace gg
