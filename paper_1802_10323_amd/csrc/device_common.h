// device_common.h - types shared by the gfx950 kernels of the Poisson solver.
//
// Every kernel works on "lines": the n values of the field along the axis the
// kernel processes (a transformed axis or the elimination axis).  A workgroup
// stages a tile of nl = 2^lognl lines in LDS, laid out point-major /
// line-minor:
//   element (line l, point p) at lds[p * nlp + l]      (nlp >= nl: row pitch)
// so that lanes with consecutive l touch consecutive LDS words.
//
// Two tile shapes exist, chosen by the axis stride:
//  * strided  - the processed axis is y or z; lines run along the contiguous
//               x axis, so a tile holds txw = 2^logtxw consecutive x positions
//               times nbt = 2^lognbt consecutive positions of the third
//               ("batch") axis, and every global access of a row of the tile
//               is contiguous in x;
//  * contiguous - the processed axis is x itself; a tile holds nl consecutive
//               lines, each n contiguous values, read by 2^logtpl lanes per
//               line.
// All index arithmetic is 32-bit shifts and masks except the final element
// offset (64-bit).
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
  int logtxw;       // x positions per tile = 2^logtxw
  int lognbt;       // batch positions per tile = 2^lognbt
  int tiles_x;      // ceil(nx / txw)
  // contiguous layout
  int nlines;       // number of lines (each n contiguous values, stride n)
  int logtpl;       // lanes per line in the contiguous loaders = 2^logtpl
  // both
  int lognl;        // lines per tile = 2^lognl
  int ntiles;       // tiles in the launch
};

// First line of a tile: x0/b0 (strided) or line index L0 (contiguous).
struct TileOrigin {
  int x0, b0, L0;
};

__device__ __forceinline__ TileOrigin tile_origin(const LineGeom& g, int tile) {
  TileOrigin o{0, 0, 0};
  if (g.layout == 0) {
    const int tb = tile / g.tiles_x;
    o.x0 = (tile - tb * g.tiles_x) << g.logtxw;
    o.b0 = tb << g.lognbt;
  } else {
    o.L0 = tile << g.lognl;
  }
  return o;
}

// Element offset of point 0 of line l of the tile, or -1 if the line lies
// outside the field (ragged last tile).
__device__ __forceinline__ long long line_base(const LineGeom& g, const TileOrigin& o, int l) {
  if (g.layout == 0) {
    const int x = o.x0 + (l & ((1 << g.logtxw) - 1));
    const int b = o.b0 + (l >> g.logtxw);
    if (x >= g.nx || b >= g.nb) return -1;
    return x + (long long)b * g.sb;
  }
  const int L = o.L0 + l;
  if (L >= g.nlines) return -1;
  return (long long)L * g.n;
}

// Coordinates (u, v) of line l along the two axes other than the processed
// one: u along the lower-numbered axis, v along the higher.
__device__ __forceinline__ void line_coords(const LineGeom& g, const TileOrigin& o, int l, int nu,
                                            int& u, int& v) {
  if (g.layout == 0) {
    u = o.x0 + (l & ((1 << g.logtxw) - 1));
    v = o.b0 + (l >> g.logtxw);
  } else {
    const int L = o.L0 + l;
    v = L / nu;
    u = L - v * nu;
  }
}

// Visit every (line, point) of a tile once, with coalesced global order:
// f(l, p, base) with base = line_base(l) (negative for a line outside the field).
template <int NT, typename F>
__device__ __forceinline__ void for_tile(const LineGeom& g, const TileOrigin& o, int tid, F&& f) {
  if (g.layout == 0) {
    const int l = tid & ((1 << g.lognl) - 1);
    const long long base = line_base(g, o, l);
    const int step = NT >> g.lognl;
    for (int p = tid >> g.lognl; p < g.n; p += step) f(l, p, base);
  } else {
    const int tpl = 1 << g.logtpl;
    const int nl = 1 << g.lognl;
    for (int l = tid >> g.logtpl; l < nl; l += NT >> g.logtpl) {
      const long long base = line_base(g, o, l);
      for (int p = tid & (tpl - 1); p < g.n; p += tpl) f(l, p, base);
    }
  }
}

// floor(j / d) for j, d < 2^16 with magic = ceil(2^32 / d), d > 1.
__device__ __forceinline__ int fast_div(int j, unsigned magic) {
  return (int)__umulhi((unsigned)j, magic);
}

}  // namespace poisson_dev
