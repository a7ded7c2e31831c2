// plane_kernels.h - both transforms of a small grid in one sweep (Sec. 2.1,
// steps 1 and 3, Table 2), for plans whose transformed axes are x and y
// with at most PLANE_NMAX points each.
//
// A solve of a 32^3 grid moves 0.5 MB per stage and is bound by the fixed
// cost of each launch and of each tile's chain of passes, not by HBM; the
// two transforms of a direction then take one launch instead of two.  A
// block holds one x-y plane (contiguous: z is the elimination axis) in LDS
// and applies each axis's transform as a dense matrix: the plan builds the
// matrices once by running its own transform kernels on unit vectors, so
// the result is the same linear map as the FFT path (up to rounding), for
// every boundary pair.  Matrix storage: row j is the transform of unit
// vector j (M[j * n + p] is output p of input j), so the threads of an
// output row read consecutive entries.
#pragma once
#include "device_common.h"

namespace poisson_dev {

static constexpr int PLANE_NT = 1024;   // one output per thread per pass up to 32 x 32
static constexpr int PLANE_NMAX = 48;

// Forward (INV false): along x, then along y; backward: along y, then x.
// mx / my: the matrices of this direction.  out64: if set, the result is
// written there widened to FP64 (the first FP32 solve of a refinement).
// skip: a refinement's stop flag (nothing to do once it is set).
template <typename T, bool INV>
__global__ __launch_bounds__(PLANE_NT) void plane_transform_kernel(T* __restrict__ data,
                                                                   double* __restrict__ out64,
                                                                   const T* __restrict__ mx,
                                                                   const T* __restrict__ my,
                                                                   int nx, int ny,
                                                                   const double* skip) {
  if (skip && skip[0] != 0.0) return;
  extern __shared__ __align__(16) unsigned char plane_smem[];
  T* X = reinterpret_cast<T*>(plane_smem);   // the plane, ny rows of nx
  T* Y = X + nx * ny;                        // after the first axis
  T* Mx = Y + nx * ny;
  T* My = Mx + nx * nx;
  const int np = nx * ny;
  const long long base = (long long)blockIdx.x * np;
  for (int e = threadIdx.x; e < np; e += PLANE_NT) X[e] = data[base + e];
  for (int e = threadIdx.x; e < nx * nx; e += PLANE_NT) Mx[e] = mx[e];
  for (int e = threadIdx.x; e < ny * ny; e += PLANE_NT) My[e] = my[e];
  __syncthreads();
  auto along_x = [&](const T* in, T* out) {
    for (int e = threadIdx.x; e < np; e += PLANE_NT) {
      const int y = e / nx, p = e - y * nx;
      T acc = 0;
      for (int j = 0; j < nx; ++j) acc += Mx[j * nx + p] * in[y * nx + j];
      out[e] = acc;
    }
  };
  auto along_y = [&](const T* in, T* out) {
    for (int e = threadIdx.x; e < np; e += PLANE_NT) {
      const int p = e / nx, x = e - p * nx;
      T acc = 0;
      for (int j = 0; j < ny; ++j) acc += My[j * ny + p] * in[j * nx + x];
      out[e] = acc;
    }
  };
  if (!INV) along_x(X, Y);
  else along_y(X, Y);
  __syncthreads();
  if (!INV) along_y(Y, X);
  else along_x(Y, X);
  __syncthreads();
  if (out64) {
    for (int e = threadIdx.x; e < np; e += PLANE_NT) out64[base + e] = (double)X[e];
  } else {
    for (int e = threadIdx.x; e < np; e += PLANE_NT) data[base + e] = X[e];
  }
}

}  // namespace poisson_dev
