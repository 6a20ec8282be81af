// Batched path: many target views of uneven resolution, view count and bin
// count fused by kernels over per-phase work lists, the whole batch captured
// once into a hipGraph and replayed with one launch.
//
// Each work item runs the same device function as the plain entry points
// (conf_tile, splat_bin_block, tile_scan_block, raster_tile,
// integrate_tile), so every output is bitwise identical to the
// corresponding plain call.  Work lists are grouped by item; the splat
// binning phases run persistent workgroups that take chunks of their lists,
// the others one workgroup per entry; either way each XCD walks a
// contiguous part of a list.
#include <algorithm>
#include <cstring>
#include <vector>

#include "batch_internal.h"

namespace gg {

// ---------------------------------------------------------------------------
// device phases

__global__ void batch_zero_kernel(uint32_t *p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void batch_bins_kernel(const BatchItem *__restrict__ items) {
  const BatchItem &it = items[blockIdx.x];
  for (int d = threadIdx.x; d < it.D; d += blockDim.x) {
    const float un = 1.0f / it.z_near;
    const float uf = 1.0f / it.z_far;
    const float du = (un - uf) / (float)(it.D - 1);
    const float u = un - (float)d * du;
    const float z = 1.0f / u;
    gstore2(it.bins + d, make_float2(z, it.trunc_in_bins ? (it.trunc * du) * (z * z) : it.trunc));
  }
}

// Dynamic work distribution in chunks, XCD-aware.  Entries differ in cost by
// orders of magnitude (items differ in size, view count and bins), so a
// static split leaves long tails; one atomic per entry, on the other hand,
// serialises on the counter, so workgroups take chunks of `chunk`
// consecutive entries (the host sizes them to about eight per workgroup).
// Workgroups are dispatched round-robin over the 8 XCDs (blockIdx & 7 is
// the XCD, as in xcd_tile), and consecutive entries of a list are
// neighbouring tiles of one item that share source lines: each XCD first
// drains its own contiguous eighth of the list, through its own counter,
// so those lines stay in its L2, then helps the other XCDs.  Which
// workgroup runs an entry never changes its result.
struct WorkCursor {
  uint32_t part;  // the part (of kXcds) being drained
  uint32_t left;  // parts not yet found empty
};

__device__ __forceinline__ uint32_t part_lo(uint32_t n, uint32_t p) {
  return (uint32_t)(((uint64_t)n * p) / kXcds);
}

// First entry of the next chunk this workgroup takes, and its end; false
// when every part is drained.  The counters (kXcds per phase) start at 0.
__device__ __forceinline__ bool next_chunk(uint32_t *ctr, uint32_t n, uint32_t chunk,
                                           WorkCursor &c, uint32_t *slot, uint32_t &w0,
                                           uint32_t &w1) {
  while (c.left) {
    const uint32_t lo = part_lo(n, c.part), hi = part_lo(n, c.part + 1);
    __syncthreads();  // the previous chunk is done with the slot
    if (threadIdx.x == 0) *slot = gatomic_add(&ctr[c.part], chunk);
    __syncthreads();
    // uniform across the workgroup: the entries' descriptors then load
    // through the scalar unit into SGPRs instead of once per lane
    const uint32_t got = __builtin_amdgcn_readfirstlane(*slot);
    if (got < hi - lo) {
      w0 = lo + got;
      w1 = hi - w0 < chunk ? hi : w0 + chunk;
      return true;
    }
    c.part = (c.part + 1) % kXcds;
    --c.left;
  }
  return false;
}

// Runs body(w) for every entry w < n this workgroup takes.
template <typename Body>
__device__ __forceinline__ void for_each_entry(uint32_t n, uint32_t chunk, uint32_t *ctr,
                                               Body &&body) {
  __shared__ uint32_t slot;
  WorkCursor c{blockIdx.x % kXcds, kXcds};
  uint32_t w0, w1;
  while (next_chunk(ctr, n, chunk, c, &slot, w0, w1))
    for (uint32_t w = w0; w < w1; ++w) body(w);
}

// The confidence, raster and fusion phases run one workgroup per entry, as
// their plain launches run one per tile: their lists hold far more entries
// than the device holds workgroups, so the dispatcher balances them as well
// as a work queue would, without a counter and barriers per grab.  Entries
// go to the XCDs in contiguous parts (xcd_tile), so the tiles in flight on
// an XCD are neighbours in the list and share the lines in its L2.
__global__ __launch_bounds__(256) void batch_conf_kernel(const BatchItem *__restrict__ items,
                                                         const WorkItem *__restrict__ work,
                                                         uint32_t n) {
  __shared__ float tile[kConfTileFloats];
  const WorkItem wi = uniform_entry(work, xcd_tile(blockIdx.x, n));
  conf_tile(items[wi.item].conf, wi.k, wi.x, wi.y, tile);
}

template <bool kFill>
__global__ __launch_bounds__(256) void batch_bin_kernel(const BatchItem *__restrict__ items,
                                                        const WorkItem *__restrict__ work,
                                                        uint32_t n, uint32_t chunk,
                                                        uint32_t *ctr) {
  for_each_entry(n, chunk, ctr, [&](uint32_t w) {
    const WorkItem wi = work[w];
    splat_bin_block<kFill>(items[wi.item].splat, wi.k, work_tile(wi));
  });
}

__global__ __launch_bounds__(1024) void batch_scan_kernel(const BatchItem *__restrict__ items,
                                                          const uint32_t *__restrict__ list) {
  __shared__ ScanLds lds;
  const SplatArgs &a = items[list[blockIdx.x]].splat;
  tile_scan_block(a.tile_count, a.tile_offset, a.tile_cursor, (uint32_t)a.K * a.ntiles, lds);
}

__global__ __launch_bounds__(256) void batch_raster_kernel(const BatchItem *__restrict__ items,
                                                           const WorkItem *__restrict__ work,
                                                           uint32_t n) {
  __shared__ RasterLds lds;
  const WorkItem wi = uniform_entry(work, xcd_tile(blockIdx.x, n));
  raster_tile<false>(items[wi.item].splat, wi.k, work_tile(wi), lds);
}

// Fusion: one workgroup tile of one item per work entry, every entry of a
// launch in the same specialisation as the plain kernel (so the same code);
// each item's tiles are listed in the plain launch's band order.
template <int V, int KC, bool kExact, int kMode>
__global__ __launch_bounds__(1024) void batch_integrate_kernel(const BatchItem *__restrict__ items,
                                                               const WorkItem *__restrict__ work,
                                                               uint32_t n) {
  extern __shared__ float smem[];
  const WorkItem wi = uniform_entry(work, xcd_tile(blockIdx.x, n));
  if constexpr (kMode == 0)
    integrate_tile<V, KC, kExact>(items[wi.item].integ, work_tile(wi), smem);
  else
    integrate_tile<V, KC, kExact, true, kMode == 2 ? 1 : 0>(items[wi.item].integ, work_tile(wi),
                                                             smem);
}

template <int C>
static void launch_integ_class(const BatchPlan &P, const IntegGroup &g, hipStream_t s) {
  // the LDS form exists for 8 and 4 bins per thread only (the host assigns
  // no items to the other combinations)
  if constexpr (mode_of_class(C) == 0 || vec_of_class(C) >= 4)
    hipLaunchKernelGGL((batch_integrate_kernel<vec_of_class(C), views_of_class(C), exact_class(C),
                                               mode_of_class(C)>),
                       dim3(g.n), dim3(g.threads), g.shm, s, P.d_items, g.list, g.n);
}

template <int C>
static void dispatch_integ_class(const BatchPlan &P, const IntegGroup &g, hipStream_t s) {
  if constexpr (C < kIntegClasses) {
    if (g.cls == C)
      launch_integ_class<C>(P, g, s);
    else
      dispatch_integ_class<C + 1>(P, g, s);
  }
}

// ---------------------------------------------------------------------------
// plan

static int persistent_grid(uint32_t n, int per_cu, int cus) {
  const uint64_t g = (uint64_t)cus * (uint64_t)(per_cu > 0 ? per_cu : 1);
  return (int)(n < g ? (n ? n : 1) : g);
}

// Entries per counter grab: about eight grabs per workgroup.
static uint32_t chunk_of(uint32_t n, int grid) {
  const uint64_t c = (uint64_t)n / ((uint64_t)grid * 8u);
  return c ? (uint32_t)c : 1u;
}

// Resident workgroups per CU of the persistent binning phases: their grids
// fill the device exactly, or hold at most blocks_per_cu workgroups per CU
// (leaving the rest of each CU to the other branch).
int batch_occupancy(BatchPlan &P) {
  int b = 0;
  if (int rc = check_hip(hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &b, batch_bin_kernel<true>, 256, 0), "batch occupancy"))
    return rc;
  const int cap = P.blocks_per_cu > 0 ? P.blocks_per_cu : 1 << 20;
  P.occ_bin = std::max(1, std::min(b, cap));
  return GG_OK;
}

int batch_record(BatchPlan &P, hipStream_t s, hipStream_t side, hipEvent_t fork,
                 hipEvent_t join) {
  const int cus = P.cus;
  // tile counts of every item and the phases' work counters
  hipLaunchKernelGGL(batch_zero_kernel, dim3(1024), dim3(256), 0, s, P.zero_ptr, P.zero_words);
  // The splat phases depend on the depth maps and the zeroed counts only: with a side stream
  // they form a second branch of the graph, beside the bins, weights and fusion of the main
  // branch, and the two overlap; the branches join before the graph ends.
  const bool branch = side && P.n_bin && P.branches != 1;
  if (branch) {
    if (int rc = check_hip(hipEventRecord(fork, s), "batch fork")) return rc;
    if (int rc = check_hip(hipStreamWaitEvent(side, fork, 0), "batch fork")) return rc;
  }
  const hipStream_t ss = branch ? side : s;
  if (P.n_bin) {
    const int gb = persistent_grid(P.n_bin, P.occ_bin, cus);
    hipLaunchKernelGGL(batch_bin_kernel<false>, dim3(gb), dim3(256), 0, ss, P.d_items, P.d_bin,
                       P.n_bin, chunk_of(P.n_bin, gb), P.d_ctr + 0 * kXcds);
    hipLaunchKernelGGL(batch_scan_kernel, dim3(P.n_splat_items), dim3(1024), 0, ss, P.d_items,
                       P.d_splat_items);
    hipLaunchKernelGGL(batch_bin_kernel<true>, dim3(gb), dim3(256), 0, ss, P.d_items, P.d_bin,
                       P.n_bin, chunk_of(P.n_bin, gb), P.d_ctr + 1 * kXcds);
    if (P.n_raster)
      hipLaunchKernelGGL(batch_raster_kernel, dim3(P.n_raster), dim3(256), 0, ss, P.d_items,
                         P.d_raster, P.n_raster);
  }
  if (branch)
    if (int rc = check_hip(hipEventRecord(join, side), "batch join")) return rc;
  hipLaunchKernelGGL(batch_bins_kernel, dim3(P.n_items), dim3(256), 0, s, P.d_items);
  if (P.n_conf)
    hipLaunchKernelGGL(batch_conf_kernel, dim3(P.n_conf), dim3(256), 0, s, P.d_items, P.d_conf,
                       P.n_conf);
  for (const IntegGroup &g : P.integ)
    if (g.n) dispatch_integ_class<0>(P, g, s);
  if (branch)
    if (int rc = check_hip(hipStreamWaitEvent(s, join, 0), "batch join")) return rc;
  return check_hip(hipGetLastError(), "batch phases");
}

}  // namespace gg
