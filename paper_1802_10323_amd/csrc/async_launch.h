// async_launch.h - entry into the asynchronous-staging transform kernels
// (r2r_fast.h).  They are compiled in translation units of their own: the
// register allocator treats a kernel differently depending on what else is
// in its unit, and the FP64 length-512 DFT / DCT-IV kernels (which may use
// up to 256 VGPRs) only avoid spills in a unit without the others
// (r2r_async_wide.hip); the rest are in r2r_async.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "r2r_fast.h"
#include "tri_fast.h"

namespace poisson_dev {

// Launch the staging transform for complex length M (128 or 256), tile
// shape `shape` (AsyncVar<M, shape>: 0 or 1, and 2 for FP32 length 512),
// transform type `kind` and direction `inverse`, arguments as for
// r2r_fast_kernel with that tile shape.  hipErrorInvalidValue if (M, shape,
// kind) has no instantiation.
hipError_t async_transform_launch(const R2RFastArgs<double>& a, int M, int shape, int kind,
                                  int inverse, hipStream_t stream);
hipError_t async_transform_launch(const R2RFastArgs<float>& a, int M, int shape, int kind,
                                  int inverse, hipStream_t stream);

// The staging elimination (tri_async.hip) for lines of n points, with the
// chunking of variant 0 (tri_fast.h).  hipErrorInvalidValue if n has none.
hipError_t async_elimination_launch(const TriFastArgs<double>& a, int n, hipStream_t stream);
hipError_t async_elimination_launch(const TriFastArgs<float>& a, int n, hipStream_t stream);

// The register-staged transform (FP64, length 512, strided axes, 32 lines
// per tile; r2r_async_wide.hip), arguments as for r2r_fast_kernel with
// RegStageCfg; `hinted` selects the form with nontemporal accesses.
// hipErrorInvalidValue for a contiguous axis.
hipError_t regstage_launch(const R2RFastArgs<double>& a, int kind, int inverse, bool hinted,
                           hipStream_t stream);

// The direct elimination of contiguous lines (tri_async.hip), with the
// chunking of variant 0 (tri_fast.h).  hipErrorInvalidValue if n has none
// or its chunks are not whole 16-byte pieces.
hipError_t direct_elimination_launch(const TriFastArgs<double>& a, int n, hipStream_t stream);
hipError_t direct_elimination_launch(const TriFastArgs<float>& a, int n, hipStream_t stream);

// The kernels of AsyncBudget<double, FastVar<256, 0>, kind>::WIDE
// (r2r_async_wide.hip).
hipError_t async_wide_launch(const R2RFastArgs<double>& a, int kind, int inverse,
                             hipStream_t stream);

// Upper bound on the blocks of the persistent launch being made on this
// thread (0: none): the grid cap of the plan whose stage is launched.  A
// testing switch (environment variable POISSON_GRID_CAP, read by
// plan_create) that makes small fields loop over many tiles per block, as
// the largest fields do.
int grid_cap_blocks();

// Blocks of a persistent launch of `fn` (512 threads, static LDS only): as
// many as are resident at once, at most one per tile.
inline int async_resident_blocks(const void* fn, long long ntiles) {
  static std::mutex mu;
  static std::vector<std::pair<std::pair<const void*, int>, int>> cache;   // (fn, device) -> blocks
  int dev = 0;
  (void)hipGetDevice(&dev);
  int blocks = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    for (auto& e : cache)
      if (e.first.first == fn && e.first.second == dev) blocks = e.second;
  }
  if (!blocks) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 512, 0) != hipSuccess) per_cu = 1;
    blocks = cus * std::max(per_cu, 1);
    std::lock_guard<std::mutex> lk(mu);
    cache.push_back({{fn, dev}, blocks});
  }
  const int cap = grid_cap_blocks();
  if (cap > 0) blocks = std::min(blocks, cap);
  return (int)std::min<long long>(ntiles, blocks);
}

// Blocks of a persistent launch of `fn` with 256 threads and static LDS
// only: as many as are resident at once (occupancy API), at most `work`.
inline int direct_blocks(const void* fn, long long work) {
  static std::mutex mu;
  static std::vector<std::pair<std::pair<const void*, int>, int>> cache;   // (fn, device) -> blocks
  int dev = 0;
  (void)hipGetDevice(&dev);
  int blocks = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    for (auto& e : cache)
      if (e.first.first == fn && e.first.second == dev) blocks = e.second;
  }
  if (!blocks) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0) != hipSuccess) per_cu = 1;
    blocks = cus * std::max(per_cu, 1);
    std::lock_guard<std::mutex> lk(mu);
    cache.push_back({{fn, dev}, blocks});
  }
  const int cap = grid_cap_blocks();
  if (cap > 0) blocks = std::min(blocks, cap);
  return (int)std::max<long long>(1, std::min<long long>(work, blocks));
}

}  // namespace poisson_dev
