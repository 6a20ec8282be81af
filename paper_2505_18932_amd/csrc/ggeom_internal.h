// Internal declarations of the gfx950 geometry-stage library: kernel argument
// records (passed by value as kernel arguments, so launches need no host to
// device copies and are capture-safe), device helpers, launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "ggeom.h"

namespace gg {

// ---------------------------------------------------------------------------
// host side: errors and launch timing

int fail(int code, const char *fmt, ...);
int check_hip(hipError_t e, const char *what);

// Brackets one kernel launch with HIP events when timing is enabled.
struct KernelTimer {
  KernelTimer(const char *name, hipStream_t s);
  ~KernelTimer();
  const char *name_;
  hipStream_t stream_;
  int slot_;
};

// Magic-number division by a runtime constant d (1 <= d < 2^31):
// q = umulhi(n, m) >> s, corrected once.
struct FastDiv {
  uint32_t d, m, s;
};
FastDiv make_fastdiv(uint32_t d);

__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f) {
  uint32_t q = __umulhi(n, f.m) >> f.s;
  if (n - q * f.d >= f.d) ++q;
  return q;
}

// The relative projection of a pixel ray into another camera, FP32:
// (x, y, z) = zeta * H (px, py, 1)^T + c.
struct Proj {
  float H[9];
  float c[3];
};
void relproj(const gg_camera &a, const gg_camera &b, Proj &out);

__device__ __forceinline__ bool depth_ok(float d) { return d > 0.0f && d < INFINITY; }

// Global-memory view of a pointer.  Pointers read from memory (the batched
// path's device-resident descriptors) carry no address space, and accesses
// through them would compile to flat instead of global instructions.
#define GG_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GG_GLOBAL T *gmem(T *p) {
  return (GG_GLOBAL T *)p;
}

// Vector loads and stores through global-memory views (HIP's float2/float4
// classes cannot bind to address-space-qualified storage; these builtin
// vectors can).
typedef float gg_v2f __attribute__((ext_vector_type(2)));
typedef float gg_v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float2 gload2(const float2 *p) {
  const gg_v2f v = *(const GG_GLOBAL gg_v2f *)p;
  return make_float2(v.x, v.y);
}

__device__ __forceinline__ void gstore2(float2 *p, float2 v) {
  *(GG_GLOBAL gg_v2f *)p = (gg_v2f){v.x, v.y};
}

// Range-checked loads through a buffer resource (raw addressing, stride 0):
// a load at a byte offset at or beyond the resource's size returns zeros
// and touches no memory.  kOutOfRange is beyond every resource made here
// (sizes are at most 2^31 bytes).
constexpr uint32_t kOutOfRange = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void *p, uint32_t bytes) {
  // last word: 32-bit data format, no swizzle, no index addressing
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                           0x00020000);
}

__device__ __forceinline__ float2 bload2(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  const gg_v2f v = __builtin_bit_cast(gg_v2f, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  return make_float2(v.x, v.y);
}

// The view table: per view Hs rows of Ws + 1 records, the last record of each
// row (0, 0) -- no usable depth, no weight -- so that a sample whose column
// falls outside the image may read that record instead of being tested.
__host__ __device__ constexpr uint32_t table_pitch(int32_t Ws) { return (uint32_t)Ws + 1u; }
__host__ __device__ constexpr size_t table_view_records(int32_t Ws, int32_t Hs) {
  return (size_t)Hs * table_pitch(Ws);
}
// A structured buffer resource holds its stride (the row pitch, bytes) in a
// 14-bit field: rows of at most 2047 records.
__host__ __device__ constexpr bool table_rows_ok(int32_t Ws) { return table_pitch(Ws) * 8u <= 16383u; }

// Structured buffer load (row index and byte offset within the row; the
// hardware multiplies the index by the stride).  A row index at or past the
// resource's row count reads zeros and touches no memory; the offset is not
// checked against the stride, so the caller keeps it inside the row.
extern "C" __device__ gg_v2f gg_struct_buffer_load_v2f32(__amdgpu_buffer_rsrc_t rsrc,
                                                          int32_t vindex, int32_t voffset,
                                                          int32_t soffset, int32_t aux)
    __asm("llvm.amdgcn.struct.ptr.buffer.load.v2f32");

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rows_of(const void *p, uint32_t pitch_bytes,
                                                          uint32_t rows) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)pitch_bytes, (int)rows,
                                           0x00020000);
}

__device__ __forceinline__ float2 rload2(__amdgpu_buffer_rsrc_t r, uint32_t row, uint32_t off) {
  const gg_v2f v = gg_struct_buffer_load_v2f32(r, (int32_t)row, (int32_t)off, 0, 0);
  return make_float2(v.x, v.y);
}

__device__ __forceinline__ uint32_t gatomic_add(uint32_t *p, uint32_t v) {
  return __hip_atomic_fetch_add(gmem(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Range in which recip_rn() is the correctly rounded reciprocal.
constexpr float kRecipLo = 0x1p-100f, kRecipHi = 0x1p100f;

// Correctly rounded 1/z for kRecipLo < z < kRecipHi: the hardware
// approximation (v_rcp_f32, about 1 ulp) refined by one Newton-Raphson step
// with fused multiply-adds, e = 1 - z y, y' = y + y e (Markstein's
// correction).  The test suite compares it bitwise with IEEE division for
// every FP32 significand over that exponent range.
__device__ __forceinline__ float recip_rn(float z) {
  const float y = __builtin_amdgcn_rcpf(z);
  const float e = fmaf(-z, y, 1.0f);
  return fmaf(y, e, y);
}

// 1/z, correctly rounded for every z > 0: the fast path above, else the
// compiler's IEEE division (rare: depths below 2^-100 or above 2^100).
__device__ __forceinline__ float recip_pos(float z) {
  if (__builtin_expect(z > kRecipLo && z < kRecipHi, 1)) return recip_rn(z);
  return 1.0f / z;
}

// A colour channel c = u / 255, correctly rounded, for u = 0..255, in three
// FP32 operations instead of an IEEE division: q = u r with r = RN(1/255),
// then one correction with the remainder u - 255 q, which the fused
// multiply-add forms exactly (Markstein's step).  The result equals the
// IEEE quotient for every u (tests/test_unorm8_cpu.py checks all 256 in
// exact rational arithmetic).
__device__ __forceinline__ float unorm8(uint32_t u) {
  constexpr float r = 1.0f / 255.0f;
  const float x = (float)u;
  const float q = x * r;
  return fmaf(fmaf(-q, 255.0f, x), r, q);
}

// floor(x) converted to int32 in one instruction (saturating; x finite).
__device__ __forceinline__ int32_t floor_i32(float x) {
  int32_t r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// h = H (px, py, 1)^T, one fused multiply-add chain per row.
__device__ __forceinline__ void ray_of(const Proj &P, float px, float py, float &h0, float &h1,
                                       float &h2) {
  h0 = fmaf(P.H[0], px, fmaf(P.H[1], py, P.H[2]));
  h1 = fmaf(P.H[3], px, fmaf(P.H[4], py, P.H[5]));
  h2 = fmaf(P.H[6], px, fmaf(P.H[7], py, P.H[8]));
}

// Workgroup id -> logical tile id such that each of the 8 XCDs (which
// receive workgroups round-robin) works on one contiguous range of tiles,
// keeping its gathers in its own L2.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t wg, uint32_t n) {
  const uint32_t x = wg & 7u, m = wg >> 3;
  const uint32_t q = n >> 3, r = n & 7u;
  return x * q + (x < r ? x : r) + m;
}

// ---------------------------------------------------------------------------
// fusion (tsdf.hip)

struct ConfArgs {
  const float *depth;  // K x Hs x Ws
  float2 *table;       // K x Hs x (Ws + 1): (usable depth or +inf, omega), rows closed by (0, 0)
  int32_t Ws, Hs, K;
  int32_t radius;      // (w - 1) / 2
  float tw2;           // conf_tau^2
  float n2;            // w * w
  float scale;         // conf_scale
};

struct IntegrateArgs {
  Proj views[GG_MAX_VIEWS];  // target -> view k
  const float2 *table;       // K x Hs x (Ws + 1) view table (table_pitch)
  const float2 *bins;        // D x (z_d, tau_d)
  const float *mask;         // Ht x Wt or null
  const float *F_prev;       // may alias F
  const float *W_prev;
  float *F;
  float *W;
  float *out_depth;  // null: no fused extraction
  int32_t *out_bin;
  int32_t K, Ws, Hs, D;
  uint32_t npix;     // Ht * Wt
  uint32_t ns;       // Hs * Ws
  FastDiv wt_div;    // by Wt
  FastDiv cpp_div;   // by chunks per pixel (D / V)
  uint32_t cpp, ppb; // chunks per pixel, pixels per workgroup
  uint32_t pw_shift; // 2^pw_shift neighbouring pixels share each wavefront row
  uint32_t nblocks;
  // tile order: band_T tiles per target row, visited in vertical bands of
  // band_B tiles across and band_H rows (band_T = 0: row-major)
  uint32_t band_T, band_B, band_H;
  float decay, cap;
  int32_t carry;
  int32_t exact_only;  // 1: every sample takes IEEE division (extreme depths)
  int32_t rows;        // 1: the launch reads the view tables with structured loads
};

struct ExtractArgs {
  const float *F;
  const float *W;
  float *out_depth;
  int32_t *out_bin;
  const float *g_depth;  // backward only
  float *g_F2;           // backward only
  const int32_t *bin;    // backward only
  uint32_t npix;
  int32_t D;
  FastDiv cpp_div;
  uint32_t cpp, ppb, nblocks;
  float z_near, z_far;
};

struct TsdfBackArgs {
  Proj views[GG_MAX_VIEWS];
  const float2 *table;   // recomputed view table, K x Hs x (Ws + 1)
  const float2 *bins;
  const float *depth;
  const float *F;
  const float *W;
  const int32_t *bin;
  const float *g_F2;
  unsigned long long *acc_D;  // K x Ns fixed point
  unsigned long long *acc_w;  // K x Ns fixed point
  float *gnu;                 // K x Ns
  uint32_t *maxbits;          // [0]: max |contribution| as float bits
  float *g_depth_in;
  int32_t K, Ws, Hs, D;
  uint32_t npix, ns;
  FastDiv wt_div;
  int32_t radius;
  float tw2, n2, scale;
};

// Volume-free raymarch (raymarch.hip).
struct RaymarchArgs {
  Proj views[GG_MAX_VIEWS];  // target -> view k
  const float2 *table;       // K x Hs x (Ws + 1) view table (table_pitch)
  int32_t K, Ws, Hs;
  uint32_t ns, npix;
  FastDiv wt_div;            // by Wt
  float z_near, z_far, du, trunc;
  int32_t trunc_in_bins;
  float decay, cap;
  int32_t max_samples;
  const float *dprev, *acc, *mask;  // Ht x Wt or null (dprev and acc together)
  float *out_depth, *out_acc;
  int32_t *out_steps;
  int32_t exact_only;
};

int launch_raymarch(const RaymarchArgs &a, hipStream_t s);

// Blending-network inputs and the blend (netinputs.hip).
struct NetArgs {
  Proj M;                  // H: R_t^T K_t^-1 (pixel -> world ray), c: the target's centre
  float Cs[GG_MAX_VIEWS][3];   // centres of the input cameras
  float dist[GG_MAX_VIEWS];    // |C_k - C_t|
  float axd[GG_MAX_VIEWS];     // optical-axis dot products
  int32_t K, W, H;
  const float *tsdf_depth;     // H x W
  const float *rgb;            // K x 3 x H x W
  const float *depth, *alpha;  // K x H x W
  float *out;                  // (9K + 1) x H x W
};

struct BlendArgs {
  int32_t K, W, H;
  const float *rgb, *depth, *alpha, *w;  // K x 3 x H x W, K x H x W (x3)
  const float *w_bg, *rgb_bg;            // H x W, 3 x H x W
  float *out_rgb, *out_depth;            // 3 x H x W, H x W
};

int launch_network_inputs(const NetArgs &a, hipStream_t s);
int launch_blend(const BlendArgs &a, hipStream_t s);

int launch_bins(const gg_tsdf_params &p, float2 *bins, hipStream_t s);
int launch_conf(const ConfArgs &a, hipStream_t s);
int launch_integrate(const IntegrateArgs &a, int V, uint32_t threads, hipStream_t s);
int launch_extract(const ExtractArgs &a, int V, uint32_t threads, hipStream_t s);
int launch_extract_backward(const ExtractArgs &a, hipStream_t s);
int launch_tsdf_backward(const TsdfBackArgs &a, hipStream_t s);
int launch_recip_selftest(uint32_t e_lo, uint32_t n_exp, unsigned long long *mismatches,
                          hipStream_t s);
int launch_fast_recip(const float *in, float *out, int64_t n, hipStream_t s);

// ---------------------------------------------------------------------------
// splatting (splat.hip)

constexpr int kTile = 16;  // target tiles are kTile x kTile pixels

struct SplatView {
  Proj P;        // view k -> target
  float sscale;  // sigma_px * fx_T / fx_k
};

struct SplatArgs {
  SplatView views[GG_MAX_VIEWS];
  const float *depth;   // K x Ns
  const uint8_t *rgb;   // K x Ns x 3
  int32_t K, Ws, Hs, Wt, Ht;
  uint32_t ns, nt;
  FastDiv ws_div;       // by Ws
  int32_t ntx, nty;     // target tiles per row / column
  uint32_t ntiles;      // per view
  float zmin, rmax2, band;
  uint32_t *tile_count;   // K x ntiles (+1 for the total)
  uint32_t *tile_offset;  // K x ntiles + 1
  uint32_t *tile_cursor;  // K x ntiles
  uint32_t *list;         // entries: source index
  uint32_t list_cap;
  int32_t *win_idx;
  float *out_depth, *out_rgb, *out_alpha, *out_tape;
  // difference-mask channel (nullable)
  const float *mask_in;   // K x Ns
  float *out_mask;        // K x Nt
  float *out_mask_max;    // Nt, zeroed by the launcher, maximum over views as float bits
  // backward
  const float *g_rgb, *g_depth, *g_alpha, *fw_rgb, *fw_depth, *fw_tape;
  const int32_t *fw_win;
  float *g_depth_in, *g_rgb_in;
};

uint32_t splat_tiles_per_splat(float r_max);

// ---------------------------------------------------------------------------
// difference masks and filtered depth (temporal.hip)

struct MaskArgs {
  const uint8_t *rgb, *rgb_prev;  // K x H x W x 3
  float *low, *pool;              // K x Hq x Wq (workspace)
  float *mask;                    // K x H x W
  const float *depth, *prev;      // K x H x W; depth null: no filter; prev null: first frame
  float *filtered;
  int32_t K, W, H, Wq, Hq, factor;
  float beta, lambda_t;
};

int launch_difference_masks(const MaskArgs &a, hipStream_t s);
int launch_splat_forward(SplatArgs &a, hipStream_t s);
int launch_splat_backward(const SplatArgs &a, hipStream_t s);

}  // namespace gg
