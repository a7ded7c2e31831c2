// refine_kernels.h - FP64 kernels around the FP32 solve for iterative
// refinement: seven-point residual (Eq. (poi), finite-volume rows on the
// non-uniform axis), solution update, width-weighted means, and the norms
// that decide when to stop.  All reductions are fixed-order (per-block
// partial sums, then one block adding the partials in index order), so a
// result does not depend on scheduling.
//
// Device status block (doubles):
//   [0] skip flag (1 once refinement has converged: later sweeps return)
//   [1] scratch scalar (weighted mean)
//   [2] converged flag
//   [3] relative update of the previous sweep
//   [4 + 2s], [5 + 2s]: ||e_s||^2 and ||Phi_s||^2 of sweep s (-1 if not run)
//   [REFINE_PARTIALS ...]: per-block partial sums (2 per block)
#pragma once
#include <algorithm>

#include "device_common.h"

namespace poisson_dev {

static constexpr int REFINE_MAX_SWEEPS = 64;
static constexpr int REFINE_BLOCKS = 1024;
static constexpr int REFINE_NT = 256;
static constexpr int REFINE_PARTIALS = 4 + 2 * REFINE_MAX_SWEEPS + 8;
static constexpr int REFINE_STAT_SLOTS = REFINE_PARTIALS + 2 * REFINE_BLOCKS;

struct OpAxis {            // one axis of the operator: rows a, b, c and widths h
  const double* a;
  const double* b;
  const double* c;
  const double* h;
  int n;
};

struct RefineGeom {
  OpAxis ax[3];            // x, y, z
  long long npts;
  double* stats;
};

__device__ __forceinline__ bool refine_skip(const double* stats) { return stats[0] != 0.0; }

template <int NT>
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = a;
  sh[NT + tid] = b;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) {
      sh[tid] += sh[tid + s];
      sh[NT + tid] += sh[NT + tid + s];
    }
    __syncthreads();
  }
  a = sh[0];
  b = sh[NT];
}

// Grid position (i, j, k) of point idx, advanced by a fixed step without
// 64-bit divisions in the loop (only the set-up divides).
struct GridWalk {
  int i, j, k, di, dj, dk, nx, ny;
  __device__ GridWalk(long long idx, long long step, int nx_, int ny_) : nx(nx_), ny(ny_) {
    const long long plane = (long long)nx * ny;
    k = (int)(idx / plane);
    const int r = (int)(idx - k * plane);
    j = r / nx;
    i = r - j * nx;
    dk = (int)(step / plane);
    const int rs = (int)(step - dk * plane);
    dj = rs / nx;
    di = rs - dj * nx;
  }
  __device__ void advance() {
    i += di;
    int cj = 0;
    if (i >= nx) { i -= nx; cj = 1; }
    j += dj + cj;
    int ck = 0;
    if (j >= ny) { j -= ny; ck = 1; }
    k += dk + ck;
  }
};

// Each kernel below is a device body over a block range, called by a
// kernel for one plan (blockIdx / gridDim) and by a batched kernel that
// runs the same body for every instance of a batch, each on its own block
// range (same blocks, same reduction order: bitwise the same result).

// reset the status block (a fill kernel rather than a memset, so the
// sequence can be captured in a graph)
__device__ __forceinline__ void refine_init_body(double* stats) {
  for (int i = threadIdx.x; i < REFINE_PARTIALS; i += blockDim.x) stats[i] = i >= 4 ? -1.0 : 0.0;
}

// partial sums of w*x (slot 0) and w (slot 1), w = hx_i hy_j hz_k
__device__ __forceinline__ void refine_wsum_body(const double* __restrict__ x, const RefineGeom& G,
                                                 int block, int nblocks, double* sh) {
  double sx = 0.0, sw = 0.0;
  const long long step = (long long)nblocks * REFINE_NT;
  const long long first = block * (long long)REFINE_NT + threadIdx.x;
  GridWalk at(first, step, G.ax[0].n, G.ax[1].n);
  for (long long idx = first; idx < G.npts; idx += step, at.advance()) {
    const double w = G.ax[0].h[at.i] * G.ax[1].h[at.j] * G.ax[2].h[at.k];
    sx += w * x[idx];
    sw += w;
  }
  block_sum2<REFINE_NT>(sx, sw, sh);
  if (threadIdx.x == 0) {
    G.stats[REFINE_PARTIALS + 2 * block] = sx;
    G.stats[REFINE_PARTIALS + 2 * block + 1] = sw;
  }
}

// stats[1] = (sum of slot 0) / (sum of slot 1)   (weighted mean)
__device__ __forceinline__ void refine_mean_body(double* stats, int nblocks, double* sh) {
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += REFINE_NT) {
    a += stats[REFINE_PARTIALS + 2 * i];
    b += stats[REFINE_PARTIALS + 2 * i + 1];
  }
  block_sum2<REFINE_NT>(a, b, sh);
  if (threadIdx.x == 0) stats[1] = b > 0.0 ? a / b : 0.0;
}

// A load or store with the nontemporal hint (NT) or a plain one.  The
// single-plan kernels take the hint on fields of 512 MiB and more: on the
// 512^3 cube the refined solve went 4.51-4.52 -> 4.44-4.46 ms with it;
// the batched kernels (many small instances) keep plain accesses.
template <bool NT, typename T>
__device__ __forceinline__ T refine_ld(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void refine_st(T v, T* p) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// f64 = rhs - mean (mean = stats[1] if `project`), e32 = (float) f64
template <bool NT>
__device__ __forceinline__ void refine_prep_body(const double* __restrict__ rhs,
                                                 double* __restrict__ f64, float* __restrict__ e32,
                                                 const double* stats, int project, long long npts,
                                                 int block, int nblocks) {
  const double mean = project ? stats[1] : 0.0;
  for (long long idx = block * (long long)REFINE_NT + threadIdx.x; idx < npts;
       idx += (long long)nblocks * REFINE_NT) {
    const double f = refine_ld<NT>(&rhs[idx]) - mean;
    refine_st<NT>(f, &f64[idx]);
    refine_st<NT>((float)f, &e32[idx]);
  }
}

// x -= stats[1]
__device__ __forceinline__ void refine_shift_body(double* __restrict__ x, const double* stats,
                                                  long long npts, int block, int nblocks) {
  const double mean = stats[1];
  for (long long idx = block * (long long)REFINE_NT + threadIdx.x; idx < npts;
       idx += (long long)nblocks * REFINE_NT)
    x[idx] -= mean;
}

// phi += e; per-block partial ||e||^2 and ||phi||^2
template <bool NT>
__device__ __forceinline__ void refine_update_body(double* __restrict__ phi,
                                                   const float* __restrict__ e32,
                                                   const RefineGeom& G, int block, int nblocks,
                                                   double* sh) {
  if (refine_skip(G.stats)) return;
  double se = 0.0, sp = 0.0;
  for (long long idx = block * (long long)REFINE_NT + threadIdx.x; idx < G.npts;
       idx += (long long)nblocks * REFINE_NT) {
    const double e = (double)refine_ld<NT>(&e32[idx]);
    const double x = refine_ld<NT>(&phi[idx]) + e;
    refine_st<NT>(x, &phi[idx]);
    se += e * e;
    sp += x * x;
  }
  block_sum2<REFINE_NT>(se, sp, sh);
  if (threadIdx.x == 0) {
    G.stats[REFINE_PARTIALS + 2 * block] = se;
    G.stats[REFINE_PARTIALS + 2 * block + 1] = sp;
  }
}

// Record sweep `sweep`: rel = ||e|| / ||phi||; the error left after the
// update is estimated from the contraction rho = rel / rel_prev as
// rel * rho / (1 - rho) (rel_prev = 1 at the first sweep, whose correction
// measures the first FP32 solve's error); once that is <= tol / 10 the
// remaining sweeps are skipped.  The margin covers a contraction that
// differs between sweeps: the residual's spectrum is not f's, so the FP32
// solve of a correction can be several times less accurate than the first.
__device__ __forceinline__ void refine_status_body(double* stats, int nblocks, int sweep,
                                                   double tol, double* sh) {
  if (refine_skip(stats)) return;
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += REFINE_NT) {
    a += stats[REFINE_PARTIALS + 2 * i];
    b += stats[REFINE_PARTIALS + 2 * i + 1];
  }
  block_sum2<REFINE_NT>(a, b, sh);
  if (threadIdx.x == 0) {
    stats[4 + 2 * sweep] = a;
    stats[5 + 2 * sweep] = b;
    const double rel = b > 0.0 ? sqrt(a / b) : 0.0;
    const double prev = stats[3] > 0.0 ? stats[3] : 1.0;
    const double rho = rel / prev;
    const double est = rho < 1.0 ? rel * rho / (1.0 - rho) : rel;
    stats[3] = rel;
    if (est <= 0.1 * tol) {
      stats[2] = 1.0;
      stats[0] = 1.0;
    }
  }
}

// Launch shape of refine_residual_kernel: blocks of REFINE_NT points of an
// xy plane, each marching through `kz` consecutive planes; `blocks` is the
// block count rounded up to a multiple of 8 (see refine_residual_kernel).
struct ResidualGrid {
  int plane_blocks, kz, z_chunks, blocks;
};

inline ResidualGrid residual_grid(int nx, int ny, int nz) {
  ResidualGrid r;
  r.plane_blocks = (int)(((long long)nx * ny + REFINE_NT - 1) / REFINE_NT);
  // about 2048 blocks in all, at least 4 planes each
  r.kz = (int)std::max<long long>(4, ((long long)nz * r.plane_blocks + 2047) / 2048);
  r.kz = std::min(r.kz, nz);
  r.z_chunks = (nz + r.kz - 1) / r.kz;
  r.blocks = (r.plane_blocks * r.z_chunks + 7) / 8 * 8;
  return r;
}

// e32 = (float)(f64 - A phi), FP64 arithmetic.  One thread per point of an
// xy plane, marching through kz planes with phi of the planes below, at and
// above in registers (each phi value is read from HBM about once; its x and
// y neighbours come from the caches).  The 8 XCDs receive consecutive
// blocks round-robin: block b works on chunk (b mod 8) * (blocks / 8) +
// b / 8, so each XCD sweeps a contiguous run of rows, whose y neighbours its
// own L2 holds.
template <bool NT>
__device__ __forceinline__ void refine_residual_body(const double* __restrict__ phi,
                                                     const double* __restrict__ f64,
                                                     float* __restrict__ e32, const RefineGeom& G,
                                                     const ResidualGrid& rg, int block) {
  if (refine_skip(G.stats)) return;
  const int chunk = (block % 8) * (rg.blocks / 8) + block / 8;
  if (chunk >= rg.plane_blocks * rg.z_chunks) return;
  const int nx = G.ax[0].n, ny = G.ax[1].n, nz = G.ax[2].n;
  const int p = (chunk % rg.plane_blocks) * REFINE_NT + (int)threadIdx.x;
  if (p >= nx * ny) return;
  const int k0 = (chunk / rg.plane_blocks) * rg.kz;
  const int k1 = min(k0 + rg.kz, nz);
  const int i = p % nx, j = p / nx;
  const OpAxis& X = G.ax[0];
  const OpAxis& Y = G.ax[1];
  const OpAxis& Z = G.ax[2];
  // a_q phi_{q-1} + b_q phi_q + c_q phi_{q+1} per axis; a_0 / c_{n-1} are
  // the periodic wrap couplings (zero at a wall, where the ghost rule is in b)
  const double ax = X.a[i], bx = X.b[i], cx = X.c[i];
  const double ay = Y.a[j], by = Y.b[j], cy = Y.c[j];
  const int xl = (i > 0 ? i - 1 : nx - 1) - i, xh = (i < nx - 1 ? i + 1 : 0) - i;
  const int yl = ((j > 0 ? j - 1 : ny - 1) - j) * nx, yh = ((j < ny - 1 ? j + 1 : 0) - j) * nx;
  const long long plane = (long long)nx * ny;
  double below = phi[(k0 > 0 ? k0 - 1 : nz - 1) * plane + p];
  double at = phi[k0 * plane + p];
  for (int k = k0; k < k1; ++k) {
    const long long o = k * plane + p;
    const double above = phi[(k < nz - 1 ? o + plane : (long long)p)];
    const double opx = ax * phi[o + xl] + bx * at + cx * phi[o + xh];
    const double opy = ay * phi[o + yl] + by * at + cy * phi[o + yh];
    const double opz = Z.a[k] * below + Z.b[k] * at + Z.c[k] * above;
    refine_st<NT>((float)(refine_ld<NT>(&f64[o]) - ((opx + opy) + opz)), &e32[o]);
    below = at;
    at = above;
  }
}

// ---- kernels for one plan

__global__ void refine_init_kernel(double* stats) { refine_init_body(stats); }

__global__ __launch_bounds__(REFINE_NT) void refine_wsum_kernel(const double* __restrict__ x,
                                                                 RefineGeom G) {
  __shared__ double sh[2 * REFINE_NT];
  refine_wsum_body(x, G, blockIdx.x, gridDim.x, sh);
}

__global__ __launch_bounds__(REFINE_NT) void refine_mean_kernel(double* stats, int nblocks) {
  __shared__ double sh[2 * REFINE_NT];
  refine_mean_body(stats, nblocks, sh);
}

template <bool NT>
__global__ __launch_bounds__(REFINE_NT) void refine_prep_kernel(const double* __restrict__ rhs,
                                                                 double* __restrict__ f64,
                                                                 float* __restrict__ e32,
                                                                 const double* stats, int project,
                                                                 long long npts) {
  refine_prep_body<NT>(rhs, f64, e32, stats, project, npts, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(REFINE_NT) void refine_shift_kernel(double* __restrict__ x,
                                                                  const double* stats,
                                                                  long long npts) {
  refine_shift_body(x, stats, npts, blockIdx.x, gridDim.x);
}

// e32 = (float)(f64 - A phi), FP64 arithmetic (see refine_residual_body)
template <bool NT>
__global__ __launch_bounds__(REFINE_NT) void refine_residual_kernel(const double* __restrict__ phi,
                                                                     const double* __restrict__ f64,
                                                                     float* __restrict__ e32,
                                                                     RefineGeom G, ResidualGrid rg) {
  refine_residual_body<NT>(phi, f64, e32, G, rg, blockIdx.x);
}

template <bool NT>
__global__ __launch_bounds__(REFINE_NT) void refine_update_kernel(double* __restrict__ phi,
                                                                   const float* __restrict__ e32,
                                                                   RefineGeom G) {
  __shared__ double sh[2 * REFINE_NT];
  refine_update_body<NT>(phi, e32, G, blockIdx.x, gridDim.x, sh);
}

__global__ __launch_bounds__(REFINE_NT) void refine_status_kernel(double* stats, int nblocks,
                                                                   int sweep, double tol) {
  __shared__ double sh[2 * REFINE_NT];
  refine_status_body(stats, nblocks, sweep, tol, sh);
}

// ---- kernels for a batch: job j owns blocks [first, first + count) of a
// launch (element-wise kernels: nb blocks; residual: rg.blocks, a multiple
// of 8 starting at a multiple of 8, so its XCD order is kept); reductions
// and per-instance steps take one block per job.

struct RefineJob {
  RefineGeom G;
  double* phi;          // the caller's field (Phi, and f on entry)
  double* f64;
  float* e32;
  int singular;
  int nb;               // blocks of the element-wise kernels
  ResidualGrid rg;
  int first_e;          // first block in the element-wise launches
  int first_r;          // first block in the residual launch
  int max_iters;
  double tol;
};

// job of block `b` (jobs sorted by first block, the first one at 0)
template <bool RESIDUAL>
__device__ __forceinline__ int refine_job_of(const RefineJob* __restrict__ jobs, int njobs, int b) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((RESIDUAL ? jobs[mid].first_r : jobs[mid].first_e) <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void refine_batch_init(const RefineJob* __restrict__ jobs) {
  refine_init_body(jobs[blockIdx.x].G.stats);
}

// the projection of f and the gauge of Phi touch singular instances only
__global__ __launch_bounds__(REFINE_NT) void refine_batch_wsum(const RefineJob* __restrict__ jobs,
                                                                int njobs) {
  __shared__ double sh[2 * REFINE_NT];
  const RefineJob& J = jobs[refine_job_of<false>(jobs, njobs, blockIdx.x)];
  if (!J.singular) return;
  refine_wsum_body(J.phi, J.G, blockIdx.x - J.first_e, J.nb, sh);
}

__global__ __launch_bounds__(REFINE_NT) void refine_batch_mean(const RefineJob* __restrict__ jobs) {
  __shared__ double sh[2 * REFINE_NT];
  const RefineJob& J = jobs[blockIdx.x];
  if (!J.singular) return;
  refine_mean_body(J.G.stats, J.nb, sh);
}

__global__ __launch_bounds__(REFINE_NT) void refine_batch_prep(const RefineJob* __restrict__ jobs,
                                                                int njobs) {
  const RefineJob& J = jobs[refine_job_of<false>(jobs, njobs, blockIdx.x)];
  refine_prep_body<false>(J.phi, J.f64, J.e32, J.G.stats, J.singular, J.G.npts, blockIdx.x - J.first_e,
                   J.nb);
}

// sweep `sweep`: the residual, or the stop of an instance at its limit
__global__ __launch_bounds__(REFINE_NT) void refine_batch_residual(const RefineJob* __restrict__ jobs,
                                                                    int njobs, int sweep) {
  const RefineJob& J = jobs[refine_job_of<true>(jobs, njobs, blockIdx.x)];
  const int block = blockIdx.x - J.first_r;
  if (sweep >= J.max_iters) {
    if (block == 0 && threadIdx.x == 0) J.G.stats[0] = 1.0;
    return;
  }
  refine_residual_body<false>(J.phi, J.f64, J.e32, J.G, J.rg, block);
}

__global__ __launch_bounds__(REFINE_NT) void refine_batch_update(const RefineJob* __restrict__ jobs,
                                                                  int njobs) {
  __shared__ double sh[2 * REFINE_NT];
  const RefineJob& J = jobs[refine_job_of<false>(jobs, njobs, blockIdx.x)];
  refine_update_body<false>(J.phi, J.e32, J.G, blockIdx.x - J.first_e, J.nb, sh);
}

__global__ __launch_bounds__(REFINE_NT) void refine_batch_status(const RefineJob* __restrict__ jobs,
                                                                  int sweep) {
  __shared__ double sh[2 * REFINE_NT];
  const RefineJob& J = jobs[blockIdx.x];
  refine_status_body(J.G.stats, J.nb, sweep, J.tol, sh);
}

__global__ __launch_bounds__(REFINE_NT) void refine_batch_shift(const RefineJob* __restrict__ jobs,
                                                                 int njobs) {
  const RefineJob& J = jobs[refine_job_of<false>(jobs, njobs, blockIdx.x)];
  if (!J.singular) return;
  refine_shift_body(J.phi, J.G.stats, J.G.npts, blockIdx.x - J.first_e, J.nb);
}

}  // namespace poisson_dev
