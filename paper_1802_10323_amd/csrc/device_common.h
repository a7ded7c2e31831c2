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

// LineGeom as separate scalar parameters of a non-inlined device function
// (a struct passed by value would go through scratch memory).
#define GEOM_PARAMS                                                                      \
  int g_n, int g_layout, long long g_sp, int g_nx, int g_nb, long long g_sb, int g_logtxw, \
      int g_lognbt, int g_tiles_x, int g_nlines, int g_logtpl, int g_lognl, int g_ntiles
#define GEOM_ARGS(g)                                                                      \
  (g).n, (g).layout, (g).sp, (g).nx, (g).nb, (g).sb, (g).logtxw, (g).lognbt, (g).tiles_x, \
      (g).nlines, (g).logtpl, (g).lognl, (g).ntiles
#define GEOM_REBUILD                                                                     \
  LineGeom { g_n, g_layout, g_sp, g_nx, g_nb, g_sb, g_logtxw, g_lognbt, g_tiles_x,       \
             g_nlines, g_logtpl, g_lognl, g_ntiles }

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

// Tiles of this block in a persistent launch.  The 8 XCDs of the chip
// receive consecutive blocks round-robin (block b runs on XCD b mod 8), and
// each XCD has its own L2: every XCD gets one contiguous eighth of the tiles,
// so the blocks running together on an XCD work on neighbouring tiles.
struct TileRange {
  int first, end, step;
};
__device__ __forceinline__ TileRange xcd_tiles(int ntiles) {
  const int G = gridDim.x, b = blockIdx.x;
  if (G < 8 || (G & 7)) return {b, ntiles, G};
  const int chunk = (ntiles + 7) >> 3;
  const int x = b & 7;
  const int end = min(ntiles, (x + 1) * chunk);
  return {x * chunk + (b >> 3), end, G >> 3};
}

// Field pointers seen as global-address-space pointers, so that loads and
// stores compile to global_* (not flat_*) instructions inside non-inlined
// device functions.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(T* p) {
  return (gptr<T>)p;
}
// element i of a read-only complex table in global memory
template <typename T>
__device__ __forceinline__ cplx<T> ldg(const cplx<T>* p, int i) {
  const gptr<const T> q = (gptr<const T>)p;
  return {q[2 * i], q[2 * i + 1]};
}
// ... and LDS pointers as local-address-space pointers (ds_* instructions).
template <typename T>
using lptr = __attribute__((address_space(3))) T*;
template <typename T>
__device__ __forceinline__ lptr<T> as_lds(T* p) {
  return (lptr<T>)p;
}

// Barrier for hand-offs through LDS between the waves of a block.  Unlike
// __syncthreads() it orders LDS accesses only: the wave waits for its own LDS
// operations, not for its global loads and stores, so a tile's stores (and
// reads of a next tile already issued) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Wait until at most N vector-memory operations of this wave are still
// outstanding.  The counter retires in issue order, so when at least N
// operations were issued after a group of reads, this waits for those reads
// and lets the last N (a tile's stores) stay in flight.
template <int N>
__device__ __forceinline__ void vm_wait_keep() {
  static_assert(N >= 0 && N < 64, "vector-memory counter range");
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// floor(j / d) for j, d < 2^16 with magic = ceil(2^32 / d), d > 1.
__device__ __forceinline__ int fast_div(int j, unsigned magic) {
  return (int)__umulhi((unsigned)j, magic);
}

// Element i (0 <= i < EPT) of thread tid in a tile of NT threads: line l,
// point p, and its global offset (-1 if outside the tile or the field).
//  strided: thread tid keeps line tid mod nl, points step by NT/nl;
//  contiguous: the tile's lines are one contiguous run of nl*n values, so
//  element e = tid + i*NT sits at offset L0*n + e (l, p = divmod(e, n)).
// `sbase` is line_base() of the thread's line (strided layout only).
template <int NT>
__device__ __forceinline__ long long tile_elem(const LineGeom& g, const TileOrigin& o,
                                               long long sbase, unsigned n_magic, int tid, int i,
                                               int& l, int& p) {
  if (g.layout == 0) {
    l = tid & ((1 << g.lognl) - 1);
    p = (tid >> g.lognl) + i * (NT >> g.lognl);
    return (p < g.n && sbase >= 0) ? sbase + p * g.sp : -1;
  }
  const int e = tid + i * NT;
  l = g.n > 1 ? fast_div(e, n_magic) : e;
  p = e - l * g.n;
  return (l < (1 << g.lognl) && o.L0 + l < g.nlines) ? (long long)o.L0 * g.n + e : -1;
}

}  // namespace poisson_dev
