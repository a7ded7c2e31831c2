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
  int V;        // variant (tile shape, radix order)
  int first;    // items of the jobs before this one
};

template <typename T>
struct BatchTriJob {
  TriFastArgs<T> a;
  int key;      // 2 * line length + variant (chunking)
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

// One item of a transform job; not inlined, so that each of the many
// configurations keeps its own register allocation.
template <typename T, typename C>
__device__ __noinline__ void batch_r2r_item(unsigned char* smem, const R2RFastArgs<T>& A,
                                            int tile, int& loaded, int tid) {
  const FastLds<T, C> S = fast_lds<T, C>(smem);
  // twiddle values depend on the length and the type class, their LDS place
  // on the tile size
  const int key = (C::M * 1024 + C::NL) * 2 + (A.kind >= K_ND ? 1 : 0);
  if (loaded != key) {
    fast_twiddles<T, C>(S, A, tid);
    loaded = key;
  }
  fast_tile<T, C>(S, A, tile, tid);
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
    if (J.a.skip && J.a.skip[0] != 0.0) continue;   // instance done (refinement converged)
    const int tile = it - J.first;
    switch (J.M * 4 + J.V) {
#define POISSON_BV(M_, V_) \
  case M_ * 4 + V_: batch_r2r_item<T, FastVar<M_, V_>>(smem_raw, J.a, tile, loaded, tid); break;
#define POISSON_BM(M_) POISSON_BV(M_, 0) POISSON_BV(M_, 1) POISSON_BV(M_, 2) POISSON_BV(M_, 3)
      POISSON_BM(16) POISSON_BM(32) POISSON_BM(48) POISSON_BM(64)
      POISSON_BM(96) POISSON_BM(128) POISSON_BM(192) POISSON_BM(256)
#undef POISSON_BM
#undef POISSON_BV
      default: break;   // the host only builds jobs of the configurations above
    }
  }
}

template <typename T, int RPC, int P>
__device__ __noinline__ void batch_tri_item(unsigned char* smem, const TriFastArgs<T>& A,
                                               int job, int tile, int& loaded, int tid) {
  using L = TriFastLayout<T, RPC, P>;
  static_assert(L::NT == 512, "the batched elimination kernel runs 512-thread blocks");
  const lptr<T> lds = as_lds(reinterpret_cast<T*>(smem));
  const lptr<double> coef =
      as_lds(reinterpret_cast<double*>(smem + tri_fast_coef_offset<T, RPC, P>()));
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
    if (J.a.skip && J.a.skip[0] != 0.0) continue;   // instance done (refinement converged)
    const int tile = it - J.first;
    switch (J.key) {
#define POISSON_BT(N_, V_, R_, P_) \
  case N_ * 2 + V_: batch_tri_item<T, R_, P_>(smem_raw, J.a, j, tile, loaded, tid); break;
      POISSON_BT(64, 0, 4, 16) POISSON_BT(64, 1, 2, 32)
      POISSON_BT(96, 0, 6, 16) POISSON_BT(96, 1, 3, 32)
      POISSON_BT(128, 0, 8, 16) POISSON_BT(128, 1, 4, 32)
      POISSON_BT(192, 0, 12, 16) POISSON_BT(192, 1, 6, 32)
      POISSON_BT(256, 0, 8, 32) POISSON_BT(256, 1, 16, 16)
      POISSON_BT(384, 0, 6, 64) POISSON_BT(384, 1, 12, 32)
      POISSON_BT(512, 0, 8, 64) POISSON_BT(512, 1, 16, 32)
#undef POISSON_BT
      default: break;   // the host only builds jobs of the configurations above
    }
  }
}

}  // namespace poisson_dev
