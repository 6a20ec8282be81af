// Z-buffered forward splatting of per-pixel Gaussians for gfx950 (paper §3.1
// and Suppl. A.3: each input pixel is an isotropic, fully opaque Gaussian at
// its back-projected point, coloured by the pixel and scaled so that its
// source-image footprint is one pixel; each view is rendered separately into
// the target, giving colour, accumulated opacity and depth).
//
// Pipeline per call (all views at once):
//   count  - every source pixel computes its target footprint and counts the
//            16x16 target tiles its candidate window touches (wavefront-
//            aggregated atomics: lanes hitting the same tile elect a leader);
//   scan   - exclusive scan of the tile counts (one workgroup);
//   fill   - the same walk writes each source index into its tiles' lists;
//   raster - one workgroup per (view, tile): z-test as an LDS 64-bit atomic
//            minimum of (bits(z) << 32 | source index), then the band blend
//            accumulated in LDS 64-bit fixed point.  Both are integer
//            reductions, so the result does not depend on the order in which
//            list entries arrive: winners are bitwise reproducible and the
//            colour is deterministic.
#include "splat_device.h"

namespace gg {

template <bool kFill>
__global__ __launch_bounds__(256) void splat_bin_kernel(SplatArgs a) {
  splat_bin_block<kFill>(a, blockIdx.y, blockIdx.x);
}

__global__ __launch_bounds__(1024) void tile_scan_kernel(const uint32_t *cnt, uint32_t *off,
                                                         uint32_t *cursor, uint32_t n) {
  __shared__ ScanLds lds;
  tile_scan_block(cnt, off, cursor, n, lds);
}

__global__ void zero_u32_kernel(uint32_t *p, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ __launch_bounds__(256) void splat_raster_kernel(SplatArgs a) {
  __shared__ RasterLds L;
  raster_tile<true>(a, blockIdx.y, blockIdx.x, L);
}

uint32_t splat_tiles_per_splat(float r_max) {
  // candidate window width <= 2 ceil(r) + 3 pixels -> tiles per dimension
  const int w = 2 * (int)ceilf(r_max) + 3;
  const int per = (w - 1) / kTile + 2;
  return (uint32_t)(per * per);
}

int launch_splat_forward(SplatArgs &a, hipStream_t s) {
  const uint32_t n = (uint32_t)a.K * a.ntiles;
  const dim3 gsrc(splat_bin_blocks((uint32_t)a.Ws, (uint32_t)a.Hs), a.K);
  {
    KernelTimer t("splat_zero", s);
    hipLaunchKernelGGL(zero_u32_kernel, dim3(min((n + 255) / 256, 1024u)), dim3(256), 0, s,
                       a.tile_count, n);
    if (int rc = check_hip(hipGetLastError(), "zero_u32_kernel")) return rc;
  }
  {
    KernelTimer t("splat_count", s);
    hipLaunchKernelGGL(splat_bin_kernel<false>, gsrc, dim3(256), 0, s, a);
    if (int rc = check_hip(hipGetLastError(), "splat_bin_kernel<count>")) return rc;
  }
  {
    KernelTimer t("splat_scan", s);
    hipLaunchKernelGGL(tile_scan_kernel, dim3(1), dim3(1024), 0, s, a.tile_count, a.tile_offset,
                       a.tile_cursor, n);
    if (int rc = check_hip(hipGetLastError(), "tile_scan_kernel")) return rc;
  }
  {
    KernelTimer t("splat_fill", s);
    hipLaunchKernelGGL(splat_bin_kernel<true>, gsrc, dim3(256), 0, s, a);
    if (int rc = check_hip(hipGetLastError(), "splat_bin_kernel<fill>")) return rc;
  }
  if (a.out_mask_max) {
    KernelTimer t("splat_zero", s);
    hipLaunchKernelGGL(zero_u32_kernel, dim3(min((a.nt + 255) / 256, 1024u)), dim3(256), 0, s,
                       reinterpret_cast<uint32_t *>(a.out_mask_max), a.nt);
    if (int rc = check_hip(hipGetLastError(), "zero_u32_kernel")) return rc;
  }
  KernelTimer t("splat_raster", s);
  hipLaunchKernelGGL(splat_raster_kernel, dim3(a.ntiles, a.K), dim3(kTile * kTile), 0, s, a);
  return check_hip(hipGetLastError(), "splat_raster_kernel");
}

// ---------------------------------------------------------------------------
// adjoint: one thread per source pixel gathers over the target pixels its
// footprint covers (no atomics).  L = <g_rgb, rgb> + <g_depth, depth> +
// <g_alpha, alpha>; with n = sum G over the band:
//   dL/dc_q  = sum_p g_rgb(p) G_qp / n(p)
//   dL/dG_qp = sum_c g_rgb_c(p) (c_q,c - rgb_c(p)) / n(p)
//              + g_alpha(p) prod_{j in band(p), j != q} (1 - G_jp)
//   dL/dD_q  = sum_p dL/dG_qp dG_qp/dD_q + [q wins p] g_depth(p) dz/dD
// The product over the other band members comes from the tape:
// exp(sum log(1 - G) - log(1 - G_q)) when no member has G == 1.

__global__ __launch_bounds__(256) void splat_backward_kernel(SplatArgs a) {
  const int k = blockIdx.y;
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.ns) return;
  const uint32_t j = fdiv(q, a.ws_div), i = q - j * (uint32_t)a.Ws;
  const SplatView &V = a.views[k];
  const float D = a.depth[(size_t)k * a.ns + q];
  const SplatGeom g = splat_geom(V, D, i, j, a);
  float gD = 0.0f, gc0 = 0.0f, gc1 = 0.0f, gc2 = 0.0f;
  if (g.ok) {
    float h0, h1, h2;
    ray_of(V.P, (float)i + 0.5f, (float)j + 0.5f, h0, h1, h2);
    const float X0 = fmaf(D, h0, V.P.c[0]), X1 = fmaf(D, h1, V.P.c[1]);
    const float Z = g.z, Z2 = Z * Z;
    const float dxdD = (h0 * Z - X0 * h2) / Z2;
    const float dydD = (h1 * Z - X1 * h2) / Z2;
    const float sig = V.sscale * (D / Z);
    const float dsdD = V.sscale * V.P.c[2] / Z2;
    // per source pixel: the Gaussian's footprint terms of dG/dD as products
    const float inv_s2 = 1.0f / g.s2, ks = dsdD / (sig * g.s2);
    const uint8_t *cq = a.rgb + ((size_t)k * a.ns + q) * 3;
    const float c[3] = {unorm8(cq[0]), unorm8(cq[1]), unorm8(cq[2])};
    const size_t kt = (size_t)k * a.nt;
    const float *grgb = a.g_rgb ? a.g_rgb + 3 * kt : nullptr;
    const float *frgb = a.fw_rgb + 3 * kt;
    const float *tape = a.fw_tape + 3 * kt;
    for (int b = g.b0; b <= g.b1; ++b)
      for (int aa = g.a0; aa <= g.a1; ++aa) {
        const float d2 = cover_d2(g, aa, b);
        if (!(d2 <= g.R2)) continue;
        const size_t p = (size_t)b * a.Wt + aa;
        const int32_t win = a.fw_win[kt + p];
        if (win < 0) continue;
        if (!(g.z <= a.fw_depth[kt + p] * a.band)) continue;
        // G exactly as the forward evaluates it: its equality with 1 selects the
        // opacity term below, as it selected the tape's count in the forward
        const float G = expf((-0.5f * d2) / g.s2);
        const float inv_n = 1.0f / tape[p];
        float dLdG = 0.0f;
        if (grgb) {
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) {
            const float gr = grgb[ch * a.nt + p];
            const float contrib = (gr * G) * inv_n;
            if (ch == 0) gc0 += contrib;
            if (ch == 1) gc1 += contrib;
            if (ch == 2) gc2 += contrib;
            dLdG += (gr * (c[ch] - frgb[ch * a.nt + p])) * inv_n;
          }
        }
        if (a.g_alpha) {
          const float L = tape[a.nt + p], ones = tape[2 * a.nt + p];
          float others = 0.0f;
          if (ones == 0.0f)
            others = expf(L - logf(1.0f - G));
          else if (G == 1.0f && ones == 1.0f)
            others = expf(L);
          dLdG += a.g_alpha[kt + p] * others;
        }
        const float dx = ((float)aa + 0.5f) - g.x, dy = ((float)b + 0.5f) - g.y;
        const float dGdD = G * ((dx * dxdD + dy * dydD) * inv_s2 + d2 * ks);
        gD += dLdG * dGdD;
        if (a.g_depth && (uint32_t)win == q) gD += a.g_depth[kt + p] * h2;
      }
  }
  const size_t o = (size_t)k * a.ns + q;
  a.g_depth_in[o] = gD;
  a.g_rgb_in[3 * o + 0] = gc0;
  a.g_rgb_in[3 * o + 1] = gc1;
  a.g_rgb_in[3 * o + 2] = gc2;
}

int launch_splat_backward(const SplatArgs &a, hipStream_t s) {
  KernelTimer t("splat_backward", s);
  hipLaunchKernelGGL(splat_backward_kernel, dim3((a.ns + 255) / 256, a.K), dim3(256), 0, s, a);
  return check_hip(hipGetLastError(), "splat_backward_kernel");
}

}  // namespace gg
