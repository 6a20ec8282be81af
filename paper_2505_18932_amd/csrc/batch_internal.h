// Batched path: device-resident item descriptors, work lists and the plan.
#pragma once

#include "splat_device.h"
#include "tsdf_device.h"

namespace gg {

constexpr int kConfTileFloats = kConfLH * kConfLW;
constexpr int kBatchCounters = 8;

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

// The fusion and raster phases address tiles beyond 65535: they use x as
// the low 16 bits and y as the high 16 bits of a 32-bit tile index.
__device__ __forceinline__ uint32_t work_tile(const WorkItem &w) {
  return (uint32_t)w.x | ((uint32_t)w.y << 16);
}

struct BatchPlan {
  int32_t n_items = 0;
  int cus = 256, blocks_per_cu = 4;
  uint32_t integ_threads = 256;
  // device memory owned by the plan
  void *dev = nullptr;
  size_t dev_bytes = 0;
  BatchItem *d_items = nullptr;
  WorkItem *d_conf = nullptr, *d_bin = nullptr, *d_raster = nullptr, *d_integ[3] = {};
  uint32_t n_conf = 0, n_bin = 0, n_raster = 0, n_integ[3] = {};
  uint32_t *d_splat_items = nullptr;
  uint32_t n_splat_items = 0;
  uint32_t *zero_ptr = nullptr;  // tile counts of every item, then the counters
  size_t zero_words = 0;
  uint32_t *d_ctr = nullptr;     // kBatchCounters work counters (zeroed per launch)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

int batch_record(BatchPlan &P, hipStream_t s);

}  // namespace gg
