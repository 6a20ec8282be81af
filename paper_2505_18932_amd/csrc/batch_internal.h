// Batched path: device-resident item descriptors, work lists and the plan.
#pragma once

#include <vector>

#include "splat_device.h"
#include "tsdf_device.h"

namespace gg {

constexpr int kConfTileFloats = kConfLH * kConfLW;

// Fusion work is split into classes that each run one specialisation of the
// plain kernel's device function: bins per thread (8, 4, 2, 1) times view
// count (1, 2, 3, 4, 6, 8 compile-time, other counts at run time, or every
// sample by IEEE division) times the volume stream's form (direct with the
// carry decided at run time; through LDS without or with a carry, for 8 or
// 4 bins per thread).
constexpr int kVecClasses = 4, kViewClasses = 8, kModeClasses = 3;
constexpr int kIntegClasses = kVecClasses * kViewClasses * kModeClasses;
constexpr int kLightCounters = 2;  // persistent phases: bin count, bin fill
constexpr int kXcds = 8;           // each phase keeps one counter per XCD
constexpr int kBatchCounters = kLightCounters * kXcds;

__host__ __device__ constexpr int vec_of_class(int c) {
  return 8 >> ((c / kModeClasses) / kViewClasses);
}
__host__ __device__ constexpr int views_of_class(int c) {
  return ((c / kModeClasses) % kViewClasses) < 4
             ? ((c / kModeClasses) % kViewClasses) + 1
             : (((c / kModeClasses) % kViewClasses) == 4
                    ? 6
                    : (((c / kModeClasses) % kViewClasses) == 5 ? 8 : 0));
}
__host__ __device__ constexpr bool exact_class(int c) {
  return (c / kModeClasses) % kViewClasses == 7;
}
// 0: direct volume stream, carry at run time; 1: through LDS, no carry; 2:
// through LDS, carried
__host__ __device__ constexpr int mode_of_class(int c) { return c % kModeClasses; }

inline int integ_class(int V, int K, bool exact_only, int mode) {
  const int vi = V == 8 ? 0 : (V == 4 ? 1 : (V == 2 ? 2 : 3));
  int kc = 6;  // runtime view count
  if (exact_only)
    kc = 7;
  else if (K >= 1 && K <= 4)
    kc = K - 1;
  else if (K == 6)
    kc = 4;
  else if (K == 8)
    kc = 5;
  return (vi * kViewClasses + kc) * kModeClasses + mode;
}

// Everything one item's phases need, in device memory (read with scalar
// loads: the descriptor address is uniform per work entry).
struct BatchItem {
  IntegrateArgs integ;
  ConfArgs conf;
  SplatArgs splat;
  float2 *bins;
  int32_t D;
  float z_near, z_far, trunc;
  int32_t trunc_in_bins;
};

// One unit of work of one phase: item, view, and a tile / block coordinate.
struct WorkItem {
  uint16_t item, k;
  uint16_t x, y;  // conf: tile (x, y); splat bin: source block x; raster / fusion: tile x
};

// Entry e of a work list, read once and made uniform: the item index then
// addresses its descriptor through the scalar unit (SGPRs), instead of a
// vector register pair held for the whole tile.
__device__ __forceinline__ WorkItem uniform_entry(const WorkItem *work, uint32_t e) {
  static_assert(sizeof(WorkItem) == 8, "WorkItem is two dwords");
  const uint2 raw = reinterpret_cast<const uint2 *>(work)[e];
  const uint32_t lo = __builtin_amdgcn_readfirstlane(raw.x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane(raw.y);
  WorkItem w;
  w.item = (uint16_t)(lo & 0xffffu);
  w.k = (uint16_t)(lo >> 16);
  w.x = (uint16_t)(hi & 0xffffu);
  w.y = (uint16_t)(hi >> 16);
  return w;
}

// The fusion and raster phases address tiles beyond 65535: they use x as
// the low 16 bits and y as the high 16 bits of a 32-bit tile index.
__device__ __forceinline__ uint32_t work_tile(const WorkItem &w) {
  return (uint32_t)w.x | ((uint32_t)w.y << 16);
}

// One fusion launch of the batch: the tiles of every item in one
// specialisation (class) and workgroup size.
struct IntegGroup {
  int cls = 0;
  uint32_t threads = 0;
  size_t shm = 0;              // dynamic LDS (its items' largest)
  WorkItem *list = nullptr;    // device
  uint32_t n = 0;
};

struct BatchPlan {
  int32_t n_items = 0;
  int cus = 256, blocks_per_cu = 0;  // 0: the binning phases fill each CU
  int branches = 2;                  // 2: splat phases beside the fusion; 1: one sequence
  int occ_bin = 1;  // resident workgroups per CU of the binning phases
  // device memory owned by the plan
  void *dev = nullptr;
  size_t dev_bytes = 0;
  BatchItem *d_items = nullptr;
  WorkItem *d_conf = nullptr, *d_bin = nullptr, *d_raster = nullptr;
  uint32_t n_conf = 0, n_bin = 0, n_raster = 0;
  std::vector<IntegGroup> integ;
  uint32_t *d_splat_items = nullptr;
  uint32_t n_splat_items = 0;
  uint32_t *zero_ptr = nullptr;  // tile counts of every item, then the counters
  size_t zero_words = 0;
  uint32_t *d_ctr = nullptr;     // kBatchCounters work counters of the binning phases
                                 // (zeroed per launch): kXcds per phase
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// Record every phase on s (captured into the plan's graph); with a side
// stream and the two events the splat phases become a parallel branch.
int batch_record(BatchPlan &P, hipStream_t s, hipStream_t side, hipEvent_t fork,
                 hipEvent_t join);
int batch_occupancy(BatchPlan &P);

}  // namespace gg
