// Internal declarations of the EWA front-to-back compositing path (ewa.hip):
// the per-pixel Gaussians projected with the local affine (EWA) map and
// composited in depth order per target pixel, as the 3D Gaussian splatting
// rasteriser that §3.1 renders them with.
#pragma once

#include "ggeom_internal.h"

namespace gg {

constexpr int kEwaTile = 8;             // target tiles of 8 x 8 pixels, one wavefront each
constexpr uint32_t kEwaSortCap = 512;  // the longest tile list sorted in LDS in one piece

struct EwaArgs {
  SplatView views[GG_MAX_VIEWS];  // view k -> target, sigma_px fx_T / fx_k
  const float *depth;             // K x Ns
  const uint8_t *rgb;             // K x Ns x 3
  int32_t K, Ws, Hs, Wt, Ht;
  uint32_t ns, nt;
  FastDiv ws_div;                 // by Ws
  int32_t ntx, nty;               // tiles per row / column
  uint32_t ntiles;                // per view
  float fx, fy, cx, cy;           // target intrinsics
  float ry, ry2;                  // fy / fx and its square, rounded once from FP64
  float lowpass, zmin, rmax;
  uint32_t *tile_count;           // K x ntiles, then the list allocator
  uint32_t *tile_offset;          // K x ntiles: start of each tile's list segment
  uint32_t *tile_cursor;          // K x ntiles
  unsigned long long *keys;       // list entries: bits(z) << 32 | source index
  unsigned long long *keys_alt;   // merge scratch, same layout
  uint32_t cap;                   // entries either key buffer holds
  float4 *rec;                    // K x Ns x 2: (u, v, Ah, Bn), (Ch, r, g, b)
  uint32_t sort_limit;            // lists longer than this are merge-sorted in global memory
  float *out_rgb;                 // K x 3 x Nt
  float *out_alpha, *out_depth;   // K x Nt
};

// Upper bound on the tiles one Gaussian's candidate window touches.
uint32_t ewa_tiles_per_splat(float r_max);
int launch_splat_ewa(const EwaArgs &a, hipStream_t s);

}  // namespace gg
