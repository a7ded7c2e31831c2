// device_common.h - types shared by the gfx950 kernels of the Poisson solver.
//
// Every kernel works on "lines": the n values of the field along the axis the
// kernel processes (a transformed axis or the elimination axis).  A workgroup
// stages a tile of `nl` lines in LDS, laid out point-major / line-minor:
//   element (line l, point p) at lds[p * nlp + l]      (nlp >= nl: row pitch)
// so that lanes with consecutive l touch consecutive LDS words.
//
// Two tile shapes exist, chosen by the axis stride:
//  * strided  - the processed axis is y or z; lines run along the contiguous
//               x axis, so a tile holds `txw` consecutive x positions times
//               `nbt` consecutive positions of the third ("batch") axis, and
//               every global access of a row of the tile is contiguous in x.
//  * contiguous - the processed axis is x itself; a tile holds `nl`
//               consecutive lines, each n contiguous values.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace poisson_dev {

template <typename T>
struct cplx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return {a.re, -a.im}; }
// multiply by -i (forward) or +i (backward)
template <typename T, bool FWD>
__device__ __forceinline__ cplx<T> mul_mi(cplx<T> a) {
  return FWD ? cplx<T>{a.im, -a.re} : cplx<T>{-a.im, a.re};
}

// Where the lines of a launch live in the field.
struct LineGeom {
  int n;            // points per line
  int layout;       // 0 = strided, 1 = contiguous
  long long sp;     // element stride between consecutive points of a line
  // strided layout
  int nx;           // extent of the lane (x) axis
  int nb;           // extent of the batch axis
  long long sb;     // element stride of the batch axis
  int txw;          // x positions per tile
  int nbt;          // batch positions per tile
  int tiles_x;      // ceil(nx / txw)
  // contiguous layout
  long long nlines; // number of lines (each n contiguous values, stride n)
  // both
  int nl;           // lines per tile
  long long ntiles; // tiles in the launch
};

// Global element offset of the first point of line l of tile `tile`, or -1
// if that line lies outside the field (ragged last tile).
__device__ __forceinline__ long long line_base(const LineGeom& g, long long tile, int l) {
  if (g.layout == 0) {
    const long long tx = tile % g.tiles_x;
    const long long tb = tile / g.tiles_x;
    const long long x = tx * g.txw + (l % g.txw);
    const long long b = tb * g.nbt + (l / g.txw);
    if (l >= g.nl || x >= g.nx || b >= g.nb) return -1;
    return x + b * g.sb;
  }
  const long long L = tile * g.nl + l;
  if (l >= g.nl || L >= g.nlines) return -1;
  return L * g.n;
}

// Spectral coordinates (u, v) of line l of a tile: the indices along the two
// other axes, u along the lane / first line axis, v along the second.
__device__ __forceinline__ void line_coords(const LineGeom& g, long long tile, int l, int nu,
                                            int& u, int& v) {
  if (g.layout == 0) {
    const long long tx = tile % g.tiles_x;
    const long long tb = tile / g.tiles_x;
    u = (int)(tx * g.txw + (l % g.txw));
    v = (int)(tb * g.nbt + (l / g.txw));
  } else {
    const long long L = tile * g.nl + l;
    u = (int)(L % nu);
    v = (int)(L / nu);
  }
}

}  // namespace poisson_dev
