// Colour-difference masks between consecutive frames (Eq. 1, §3.2) and the
// temporally filtered depth (Eq. 2).  Three streaming passes per call:
//   1. one thread per low-resolution pixel: the factor x factor box sums of
//      both frames (exact integers), the channel mean of |I - I'| and the
//      clamped mask;
//   2. one thread per low-resolution pixel: the 3 x 3 maximum;
//   3. one thread per full-resolution pixel: bilinear upsampling, and the
//      depth filter fused in (one read of D and of the previous filtered
//      depth, one write of each output).
// The low-resolution planes (1/16 of a frame) stay in L2 between passes.
// Every step follows the FP32 operation order stated in the header, so the
// outputs are bitwise those of that definition.
#include "ggeom_internal.h"

namespace gg {

__global__ __launch_bounds__(256) void mask_low_kernel(MaskArgs a) {
  const size_t nq = (size_t)a.Wq * a.Hq, n = nq * a.K;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
       t += (size_t)gridDim.x * blockDim.x) {
    const uint32_t k = (uint32_t)(t / nq), r = (uint32_t)(t - (size_t)k * nq);
    const uint32_t b = r / (uint32_t)a.Wq, aa = r - b * (uint32_t)a.Wq;
    const int j0 = (int)b * a.factor, i0 = (int)aa * a.factor;
    const int j1 = min(j0 + a.factor, a.H), i1 = min(i0 + a.factor, a.W);
    const GG_GLOBAL uint8_t *f0 = gmem(a.rgb) + (size_t)k * a.W * a.H * 3;
    const GG_GLOBAL uint8_t *f1 = gmem(a.rgb_prev) + (size_t)k * a.W * a.H * 3;
    int st[3] = {0, 0, 0}, sp[3] = {0, 0, 0};
    for (int j = j0; j < j1; ++j) {
      const size_t row = ((size_t)j * a.W) * 3;
      for (int i = i0 * 3; i < i1 * 3; i += 3) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          st[ch] += f0[row + i + ch];
          sp[ch] += f1[row + i + ch];
        }
      }
    }
    const int cnt = (j1 - j0) * (i1 - i0);
    const int d = abs(st[0] - sp[0]) + abs(st[1] - sp[1]) + abs(st[2] - sp[2]);
    const float dI = (float)d / (float)(765 * cnt);
    const float tq = dI / a.lambda_t;
    gmem(a.low)[t] = fminf(tq + a.beta, 1.0f);
  }
}

__global__ __launch_bounds__(256) void mask_pool_kernel(MaskArgs a) {
  const size_t nq = (size_t)a.Wq * a.Hq, n = nq * a.K;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
       t += (size_t)gridDim.x * blockDim.x) {
    const uint32_t k = (uint32_t)(t / nq), r = (uint32_t)(t - (size_t)k * nq);
    const int b = (int)(r / (uint32_t)a.Wq), aa = (int)(r - (uint32_t)b * (uint32_t)a.Wq);
    const GG_GLOBAL float *low = gmem(a.low) + (size_t)k * nq;
    float m = low[r];
    for (int bb = max(b - 1, 0); bb <= min(b + 1, a.Hq - 1); ++bb)
      for (int x = max(aa - 1, 0); x <= min(aa + 1, a.Wq - 1); ++x)
        m = fmaxf(m, low[(size_t)bb * a.Wq + x]);
    gmem(a.pool)[t] = m;
  }
}

__global__ __launch_bounds__(256) void mask_up_kernel(MaskArgs a) {
  const size_t np = (size_t)a.W * a.H, nq = (size_t)a.Wq * a.Hq, n = np * a.K;
  const float fac = (float)a.factor, xmax = (float)(a.Wq - 1), ymax = (float)(a.Hq - 1);
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
       t += (size_t)gridDim.x * blockDim.x) {
    const uint32_t k = (uint32_t)(t / np), r = (uint32_t)(t - (size_t)k * np);
    const uint32_t j = r / (uint32_t)a.W, i = r - j * (uint32_t)a.W;
    float x = ((float)i + 0.5f) / fac - 0.5f;
    float y = ((float)j + 0.5f) / fac - 0.5f;
    x = x < 0.0f ? 0.0f : (x > xmax ? xmax : x);
    y = y < 0.0f ? 0.0f : (y > ymax ? ymax : y);
    const int x0 = (int)floorf(x), y0 = (int)floorf(y);
    const int x1 = min(x0 + 1, a.Wq - 1), y1 = min(y0 + 1, a.Hq - 1);
    const float fx = x - (float)x0, fy = y - (float)y0;
    const GG_GLOBAL float *pool = gmem(a.pool) + (size_t)k * nq;
    const float m00 = pool[(size_t)y0 * a.Wq + x0], m10 = pool[(size_t)y0 * a.Wq + x1];
    const float m01 = pool[(size_t)y1 * a.Wq + x0], m11 = pool[(size_t)y1 * a.Wq + x1];
    const float top = m00 + fx * (m10 - m00);
    const float bot = m01 + fx * (m11 - m01);
    const float M = top + fy * (bot - top);
    gmem(a.mask)[t] = M;
    if (a.depth) {
      const float D = gmem(a.depth)[t];
      float out;
      if (!depth_ok(D)) {
        out = 0.0f;
      } else {
        const float pv = a.prev ? gmem(a.prev)[t] : 0.0f;
        out = (pv > 0.0f && pv < INFINITY) ? fmaf(M, D, (1.0f - M) * pv) : D;
      }
      gmem(a.filtered)[t] = out;
    }
  }
}

static unsigned grid_for(size_t n) {
  const size_t b = (n + 255) / 256;
  return (unsigned)(b < 65536 ? (b ? b : 1) : 65536);
}

int launch_difference_masks(const MaskArgs &a, hipStream_t s) {
  KernelTimer t("difference_masks", s);
  const size_t nq = (size_t)a.Wq * a.Hq * a.K, np = (size_t)a.W * a.H * a.K;
  hipLaunchKernelGGL(mask_low_kernel, dim3(grid_for(nq)), dim3(256), 0, s, a);
  if (int rc = check_hip(hipGetLastError(), "mask_low_kernel")) return rc;
  hipLaunchKernelGGL(mask_pool_kernel, dim3(grid_for(nq)), dim3(256), 0, s, a);
  if (int rc = check_hip(hipGetLastError(), "mask_pool_kernel")) return rc;
  hipLaunchKernelGGL(mask_up_kernel, dim3(grid_for(np)), dim3(256), 0, s, a);
  return check_hip(hipGetLastError(), "mask_up_kernel");
}

}  // namespace gg
