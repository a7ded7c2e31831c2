// batch_kernels.h - one persistent launch per solver stage over many
// independent instances of different sizes.
//
// A batched stage is a list of jobs, one per instance: the launch arguments
// that instance's own kernel for the stage would get, the size-specialised
// kernel body it needs, and the index of its first work item.  The work
// items of the stage are the tiles of all jobs, numbered job after job; the
// blocks of the persistent grid take contiguous runs of items (one run per
// XCD, interleaved over that XCD's blocks), find the job of each item by a
// binary search over the jobs' first items (block-uniform, scalar loads),
// and run the same tile function as the single-instance kernel, so a
// batched solve is bitwise identical to solving the instances one by one.
//
// LDS tables that depend on the job (transform twiddles: on the length and
// the type class; elimination coefficients: on the instance) are reloaded
// only when the job of the next item needs other ones.
#pragma once
#include "r2r_fast.h"
#include "tri_fast.h"

namespace poisson_dev {

template <typename T>
struct BatchR2RJob {
  R2RFastArgs<T> a;
  int M;        // complex FFT length (n = 2M)
  int first;    // items of the jobs before this one
};

template <typename T>
struct BatchTriJob {
  TriFastArgs<T> a;
  int shape;    // rows per chunk * 100 + chunks per line
  int first;
};

// Job holding item `it`: jobs are sorted by `first`, jobs[0].first = 0.
template <typename J>
__device__ __forceinline__ int batch_job_of(const J* __restrict__ jobs, int njobs, int it) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].first <= it) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename T, int M>
__device__ __forceinline__ void batch_r2r_item(unsigned char* smem, const R2RFastArgs<T>& A,
                                               int tile, int& loaded, int tid) {
  static_assert(fast_nt<M>() == 512, "the batched transform kernel runs 512-thread blocks");
  const FastLds<T, M> S = fast_lds<T, M>(smem);
  const int key = 2 * M + (A.kind >= K_ND ? 1 : 0);
  if (loaded != key) {
    fast_twiddles<T, M>(S, A, tid);
    loaded = key;
  }
  fast_tile<T, M>(S, A, tile, tid);
}

template <typename T>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
void batch_r2r_kernel(const BatchR2RJob<T>* __restrict__ jobs, int njobs, int items) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int tid = threadIdx.x;
  int loaded = -1;
  const TileRange tr = xcd_tiles(items);
  for (int it = tr.first; it < tr.end; it += tr.step) {
    const BatchR2RJob<T>& J = jobs[batch_job_of(jobs, njobs, it)];
    const int tile = it - J.first;
    switch (J.M) {
      case 16: batch_r2r_item<T, 16>(smem_raw, J.a, tile, loaded, tid); break;
      case 32: batch_r2r_item<T, 32>(smem_raw, J.a, tile, loaded, tid); break;
      case 48: batch_r2r_item<T, 48>(smem_raw, J.a, tile, loaded, tid); break;
      case 64: batch_r2r_item<T, 64>(smem_raw, J.a, tile, loaded, tid); break;
      case 96: batch_r2r_item<T, 96>(smem_raw, J.a, tile, loaded, tid); break;
      case 128: batch_r2r_item<T, 128>(smem_raw, J.a, tile, loaded, tid); break;
      case 192: batch_r2r_item<T, 192>(smem_raw, J.a, tile, loaded, tid); break;
      case 256: batch_r2r_item<T, 256>(smem_raw, J.a, tile, loaded, tid); break;
      default: break;   // the host only builds jobs of the lengths above
    }
  }
}

template <typename T, int RPC, int P>
__device__ __noinline__ void batch_tri_item(unsigned char* smem, const TriFastArgs<T>& A,
                                               int job, int tile, int& loaded, int tid) {
  using L = TriFastLayout<T, RPC, P>;
  static_assert(L::NT == 512, "the batched elimination kernel runs 512-thread blocks");
  const lptr<T> lds = as_lds(reinterpret_cast<T*>(smem));
  const lptr<T> coef = lds + L::TILE;
  if (loaded != job) {
    tri_fast_coefs<T, RPC, P>(coef, A, tid);
    loaded = job;
  }
  tri_fast_tile<T, RPC, P>(lds, coef, A, tile, tid);
}

template <typename T>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
void batch_tri_kernel(const BatchTriJob<T>* __restrict__ jobs, int njobs, int items) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int tid = threadIdx.x;
  int loaded = -1;
  const TileRange tr = xcd_tiles(items);
  for (int it = tr.first; it < tr.end; it += tr.step) {
    const int j = batch_job_of(jobs, njobs, it);
    const BatchTriJob<T>& J = jobs[j];
    const int tile = it - J.first;
    switch (J.shape) {
      case 416: batch_tri_item<T, 4, 16>(smem_raw, J.a, j, tile, loaded, tid); break;
      case 616: batch_tri_item<T, 6, 16>(smem_raw, J.a, j, tile, loaded, tid); break;
      case 816: batch_tri_item<T, 8, 16>(smem_raw, J.a, j, tile, loaded, tid); break;
      case 1216: batch_tri_item<T, 12, 16>(smem_raw, J.a, j, tile, loaded, tid); break;
      case 832: batch_tri_item<T, 8, 32>(smem_raw, J.a, j, tile, loaded, tid); break;
      case 664: batch_tri_item<T, 6, 64>(smem_raw, J.a, j, tile, loaded, tid); break;
      case 864: batch_tri_item<T, 8, 64>(smem_raw, J.a, j, tile, loaded, tid); break;
      default: break;   // the host only builds jobs of the shapes above
    }
  }
}

}  // namespace poisson_dev
