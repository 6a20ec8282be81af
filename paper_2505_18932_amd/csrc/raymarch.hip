// Volume-free TSDF raymarch (Suppl. A.1: advance along the target ray by
// 0.8 s until s changes sign, then three bisection steps; Suppl. A.2: the
// previous output depth as one more input with the temporal weight).
//
// One thread per target pixel.  Each evaluation of the fused signed distance
// at a depth z issues the K view-table gathers together (compile-time K) and
// accumulates them in view order with the volume fusion's rules, so a
// sample's contribution is bitwise the same as in a voxel at that depth.
// There is no volume: per pixel the kernel reads the view tables and writes
// one depth (and the accumulated weight for the next frame).
#include "tsdf_device.h"

namespace gg {

struct Fused {
  float S, Wo, Wt;
};

// One view's sample at depth z: its depth Z in the view and its record.
template <bool kExact>
__device__ __forceinline__ float2 march_sample(const RaymarchArgs &a, int k, float px, float py,
                                               float z, float &Z) {
  const Proj &P = a.views[k];
  float h0, h1, h2;
  ray_of(P, px, py, h0, h1, h2);
  const float X0 = fmaf(z, h0, P.c[0]);
  const float X1 = fmaf(z, h1, P.c[1]);
  Z = fmaf(z, h2, P.c[2]);
  const float fWs = (float)a.Ws, fHs = (float)a.Hs;
  uint32_t off;
  // recip_rn unless a lane's depth lies in (0, 2^-100] (wave-uniform choice)
  const uint32_t pitch = table_pitch(a.Ws);
  if (kExact || __any(Z > 0.0f && !(Z > kRecipLo)))
    off = sample_offset<kDivide>(X0, X1, Z, (uint32_t)a.Ws, (uint32_t)a.Hs, pitch, fWs, fHs);
  else
    off = sample_offset<kChecked>(X0, X1, Z, (uint32_t)a.Ws, (uint32_t)a.Hs, pitch, fWs, fHs);
  const size_t rec = table_view_records(a.Ws, a.Hs);
  return bload2(buffer_of(a.table + (size_t)k * rec, (uint32_t)(rec * 8u)), off);
}

__device__ __forceinline__ void march_accumulate(float Z, float2 e, float tau, float &S,
                                                 float &Wo) {
  const float s = e.x - Z;
  const float c = __builtin_amdgcn_fmed3f(s, -tau, tau);  // min(s, tau) where kept
  const float w = (s < -tau) ? 0.0f : e.y;
  S = fmaf(w, c, S);
  Wo = Wo + w;
}

template <int KC, bool kExact>
__device__ __forceinline__ Fused march_eval(const RaymarchArgs &a, float px, float py, float z,
                                            float tau, float wtmp, float Dp) {
  float S = 0.0f, Wo = 0.0f;
  if constexpr (KC > 0) {
    float Z[KC];
    float2 e[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) e[k] = march_sample<kExact>(a, k, px, py, z, Z[k]);
#pragma unroll
    for (int k = 0; k < KC; ++k) march_accumulate(Z[k], e[k], tau, S, Wo);
  } else {
    for (int k = 0; k < a.K; ++k) {
      float Z;
      const float2 e = march_sample<kExact>(a, k, px, py, z, Z);
      march_accumulate(Z, e, tau, S, Wo);
    }
  }
  float Wt = Wo;
  if (wtmp > 0.0f && Dp > 0.0f) {
    const float s = Dp - z;
    if (!(s < -tau)) {
      S = fmaf(wtmp, fminf(s, tau), S);
      Wt = Wt + wtmp;
    }
  }
  return Fused{S, Wo, Wt};
}

__device__ __forceinline__ float march_tau(const RaymarchArgs &a, float z) {
  return a.trunc_in_bins ? (a.trunc * a.du) * (z * z) : a.trunc;
}

template <int KC, bool kExact>
__global__ __launch_bounds__(256) void raymarch_kernel(RaymarchArgs a) {
  const uint32_t pix = blockIdx.x * blockDim.x + threadIdx.x;
  if (pix >= a.npix) return;
  const uint32_t y = fdiv(pix, a.wt_div), x = pix - y * a.wt_div.d;
  const float px = (float)x + 0.5f, py = (float)y + 0.5f;
  float wtmp = 0.0f, Dp = 0.0f;
  if (a.dprev) {
    const float m = a.mask ? fmaxf(1.0f - gmem(a.mask)[pix], 0.0f) : 1.0f;
    wtmp = fminf((a.decay * gmem(a.acc)[pix]) * m, a.cap);
    Dp = gmem(a.dprev)[pix];
  }
  float z = a.z_near, zprev = 0.0f;
  bool prev_pos = false, found = false;
  int steps = 0;
  while (z <= a.z_far && steps < a.max_samples) {
    const float tau = march_tau(a, z);
    const Fused f = march_eval<KC, kExact>(a, px, py, z, tau, wtmp, Dp);
    ++steps;
    const float smin = (a.du * z) * z;
    if (f.Wt > 0.0f) {
      const float s = f.S / f.Wt;
      if (s > 0.0f) {
        zprev = z;
        prev_pos = true;
        z = z + fmaxf(0.8f * s, smin);
      } else if (prev_pos) {
        found = true;
        break;
      } else {
        z = z + smin;
      }
    } else {
      prev_pos = false;
      z = z + 0.8f * tau;
    }
  }
  float dep = 0.0f, an = 0.0f;
  if (found) {
    float lo = zprev, hi = z;
    for (int it = 0; it < 3; ++it) {
      const float mid = lo + (hi - lo) * 0.5f;
      const Fused f = march_eval<KC, kExact>(a, px, py, mid, march_tau(a, mid), wtmp, Dp);
      if (f.Wt > 0.0f && f.S / f.Wt > 0.0f)
        lo = mid;
      else
        hi = mid;
    }
    dep = lo + (hi - lo) * 0.5f;
    const Fused f = march_eval<KC, kExact>(a, px, py, dep, march_tau(a, dep), wtmp, Dp);
    an = wtmp + f.Wo;
  }
  gmem(a.out_depth)[pix] = dep;
  if (a.out_acc) gmem(a.out_acc)[pix] = an;
  if (a.out_steps) gmem(a.out_steps)[pix] = steps;
}

template <int KC>
static void launch_raymarch_k(const RaymarchArgs &a, hipStream_t s) {
  const dim3 grid((a.npix + 255) / 256);
  if (a.exact_only)
    hipLaunchKernelGGL((raymarch_kernel<KC, true>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((raymarch_kernel<KC, false>), grid, dim3(256), 0, s, a);
}

int launch_raymarch(const RaymarchArgs &a, hipStream_t s) {
  KernelTimer t("raymarch", s);
  switch (a.K) {
    case 1: launch_raymarch_k<1>(a, s); break;
    case 2: launch_raymarch_k<2>(a, s); break;
    case 3: launch_raymarch_k<3>(a, s); break;
    case 4: launch_raymarch_k<4>(a, s); break;
    case 6: launch_raymarch_k<6>(a, s); break;
    case 8: launch_raymarch_k<8>(a, s); break;
    default: launch_raymarch_k<0>(a, s); break;
  }
  return check_hip(hipGetLastError(), "raymarch_kernel");
}

}  // namespace gg
