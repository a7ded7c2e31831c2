// tri_fast.h - size-specialised elimination of the reduced systems of
// Eq. (poi_reduced) for lines whose length n is a multiple of the chunk
// count: n = RPC * P, RPC rows per chunk, P chunks (lanes) per line.
//
// Same algorithm as tridiag_kernel.h (chunked Thomas, interface system by
// parallel cyclic reduction, back substitution), with every loop bound a
// compile-time constant, so that
//  * the coefficients of the axis are copied to LDS once per block, laid out
//    [row in chunk][chunk] so that the P lanes of a line read consecutive
//    words, instead of being fetched from global memory row by row;
//  * the whole chunk (values, pivots, spike vector) lives in registers from
//    the first read to the final write;
//  * the reciprocal of every pivot is the hardware estimate refined by
//    Newton steps (relative error at the rounding level of the type)
//    instead of a correctly rounded division sequence;
//  * the interface system is reduced in normalised form (unit diagonal:
//    three values move between lanes per step instead of four, one
//    reciprocal instead of two), and a line of 16 chunks occupies one
//    16-lane row of the wavefront, so its exchanges are DPP row rotations
//    (VALU) instead of LDS permutes.
#pragma once
#include <type_traits>
#include "tridiag_kernel.h"
#include "stage_dma.h"

namespace poisson_dev {

template <typename T>
struct TriFastArgs {
  T* data;
  LineGeom g;
  int periodic;
  int singular;
  int nu;             // extent of u (contiguous layout: line index = u + nu v)
  int nv;             // extent of v
  // coefficient tables in FP64 for both field precisions: the recurrences
  // run in FP64 registers (see tri_fast_line)
  const double* a;    // [n]
  const double* b;    // [n]
  const double* c;    // [n]
  const double* w;    // [n] cell widths along s (gauge weights)
  const double* lamu;
  const double* lamv;
  const double* skip;
  int nreal;          // rows of a line that exist (< N for a padded strided line)
};

template <typename T, int RPC, int P>
struct TriFastLayout {
  static constexpr int NT = 512;
  static constexpr int NL = NT / P;           // lines per tile
  static constexpr int N = RPC * P;           // line length
  static constexpr int NLP = NL + 1;          // row pitch
  static constexpr int CP = (RPC * NLP) | 1;  // chunk pitch (odd)
  static constexpr int TILE = P * CP;         // reals of the tile
  static_assert(RPC >= 2 && P >= 2 && P <= 64 && (P & (P - 1)) == 0, "unsupported chunking");
};

// LDS: the tile (field type), then the FP64 coefficient tables (4N).
template <typename T, int RPC, int P>
constexpr size_t tri_fast_coef_offset() {
  using L = TriFastLayout<T, RPC, P>;
  return ((size_t)L::TILE * sizeof(T) + 15) / 16 * 16;
}
template <typename T, int RPC, int P>
constexpr size_t tri_fast_lds_bytes() {
  using L = TriFastLayout<T, RPC, P>;
  return tri_fast_coef_offset<T, RPC, P>() + (size_t)4 * L::N * sizeof(double);
}

// 1/d: hardware reciprocal estimate refined by Newton steps.
__device__ __forceinline__ double fast_rcp(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-d, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float fast_rcp(float d) {
  float r = __builtin_amdgcn_rcpf(d);
  const float e = __builtin_fmaf(-d, r, 1.0f);
  return __builtin_fmaf(r, e, r);
}

// LDS position of point p of line ll of the tile.
template <typename T, int RPC, int P>
__device__ __forceinline__ int tri_fast_slot(int p, int ll) {
  using L = TriFastLayout<T, RPC, P>;
  const int ch = p / RPC;
  return ch * L::CP + (p - ch * RPC) * L::NLP + ll;
}

// Tile load: global -> LDS; all global loads of a thread are issued before
// its first LDS write.  Strided layout: line tid mod NL, points
// tid / NL + i P; contiguous layout: element tid + i NT of the tile's run.
// LAY >= 0: the layout as a constant (0 strided, 1 contiguous); -1: `layout`.
template <typename T, int RPC, int P, int LAY = -1>
__device__ __noinline__ void tri_fast_load(lptr<T> lds, gptr<const T> data, long long base,
                                           long long sp, int layout, int lines, int tid,
                                           int nreal) {
  using L = TriFastLayout<T, RPC, P>;
  T buf[RPC];
  if ((LAY >= 0 ? LAY : layout) == 0) {
    const int l = tid % L::NL, q = tid / L::NL;
    if (nreal >= L::N) {   // whole lines (uniform): no row mask
#pragma unroll
      for (int i = 0; i < RPC; ++i) buf[i] = base >= 0 ? data[base + (q + i * P) * sp] : (T)0;
    } else {               // a padded line: rows past nreal read as 0
#pragma unroll
      for (int i = 0; i < RPC; ++i)
        buf[i] = base >= 0 && q + i * P < nreal ? data[base + (q + i * P) * sp] : (T)0;
    }
#pragma unroll
    for (int i = 0; i < RPC; ++i) lds[tri_fast_slot<T, RPC, P>(q + i * P, l)] = buf[i];
  } else {
    if (nreal >= L::N) {   // whole lines (uniform): one contiguous run
#pragma unroll
      for (int i = 0; i < RPC; ++i) {
        const int e = tid + i * L::NT;
        buf[i] = e / L::N < lines ? data[base + e] : (T)0;
      }
    } else {               // padded lines: stride nreal, rows past it read as 0
#pragma unroll
      for (int i = 0; i < RPC; ++i) {
        const int e = tid + i * L::NT;
        const int ll = e / L::N, r = e - ll * L::N;
        buf[i] = ll < lines && r < nreal ? data[base + (long long)ll * nreal + r] : (T)0;
      }
    }
#pragma unroll
    for (int i = 0; i < RPC; ++i) {
      const int e = tid + i * L::NT;
      const int ll = e / L::N;
      lds[tri_fast_slot<T, RPC, P>(e - ll * L::N, ll)] = buf[i];
    }
  }
}

template <typename T, int RPC, int P>
__device__ __forceinline__ void tri_fast_store_body(lptr<const T> lds, gptr<T> data, long long base,
                                                    long long sp, int layout, int lines, int tid,
                                                    int nreal) {
  using L = TriFastLayout<T, RPC, P>;
  T buf[RPC];
  if (layout == 0) {
    const int l = tid % L::NL, q = tid / L::NL;
#pragma unroll
    for (int i = 0; i < RPC; ++i) buf[i] = lds[tri_fast_slot<T, RPC, P>(q + i * P, l)];
    if (base >= 0 && nreal >= L::N) {
#pragma unroll
      for (int i = 0; i < RPC; ++i) data[base + (q + i * P) * sp] = buf[i];
    } else if (base >= 0) {   // a padded line: rows past nreal are not stored
#pragma unroll
      for (int i = 0; i < RPC; ++i)
        if (q + i * P < nreal) data[base + (q + i * P) * sp] = buf[i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < RPC; ++i) {
      const int e = tid + i * L::NT;
      const int ll = e / L::N;
      buf[i] = lds[tri_fast_slot<T, RPC, P>(e - ll * L::N, ll)];
    }
    if (nreal >= L::N) {
#pragma unroll
      for (int i = 0; i < RPC; ++i) {
        const int e = tid + i * L::NT;
        if (e / L::N < lines) data[base + e] = buf[i];
      }
    } else {   // padded lines: stride nreal, rows past it not stored
#pragma unroll
      for (int i = 0; i < RPC; ++i) {
        const int e = tid + i * L::NT;
        const int ll = e / L::N, r = e - ll * L::N;
        if (ll < lines && r < nreal) data[base + (long long)ll * nreal + r] = buf[i];
      }
    }
  }
}

template <typename T, int RPC, int P, int LAY = -1>
__device__ __noinline__ void tri_fast_store(lptr<const T> lds, gptr<T> data, long long base,
                                            long long sp, int layout, int lines, int tid,
                                            int nreal) {
  tri_fast_store_body<T, RPC, P>(lds, data, base, sp, LAY >= 0 ? LAY : layout, lines, tid, nreal);
}

// Sum over the P lanes of a line.
template <typename T, int P>
__device__ __forceinline__ T line_sum(T v) {
#pragma unroll
  for (int off = 1; off < P; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Cyclic rotation inside a row of 16 lanes (DPP row_ror: lane i reads lane
// (i - R) mod 16 of its row); a VALU operation, no LDS traffic.
template <int R>
__device__ __forceinline__ int dpp_ror(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x120 + R, 0xF, 0xF, false);
}
template <int R>
__device__ __forceinline__ float dpp_ror(float v) {
  return __builtin_bit_cast(float, dpp_ror<R>(__builtin_bit_cast(int, v)));
}
template <int R>
__device__ __forceinline__ double dpp_ror(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)dpp_ror<R>((int)(unsigned)b);
  const unsigned hi = (unsigned)dpp_ror<R>((int)(unsigned)(b >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// v of the lane ST places before (AFTER = false) or after (AFTER = true)
// this one, cyclically within its group of P lanes.  A group of 16 lanes is
// one DPP row; larger groups go through ds_bpermute.
template <int P, int ST, bool AFTER, typename T>
__device__ __forceinline__ T group_rot(T v, int gbase, int c) {
  if constexpr (P == 16) {
    return dpp_ror<AFTER ? 16 - ST : ST>(v);
  } else {
    return __shfl(v, gbase + ((AFTER ? c + ST : c - ST) & (P - 1)), 64);
  }
}

// Parallel cyclic reduction of the interface equations, kept normalised:
// x_c + l x_{c-ST} + u x_{c+ST} = r.  Each step subtracts l times the
// equation of lane c-ST and u times that of lane c+ST, doubling the coupling
// distance; outside a non-periodic line the neighbour is the identity
// equation x = 0.
template <typename T, int P, int ST>
__device__ __forceinline__ void pcr(T& l, T& u, T& r, int c, int gbase, int periodic) {
  if constexpr (ST < P) {
    T lm = group_rot<P, ST, false>(l, gbase, c);
    T um = group_rot<P, ST, false>(u, gbase, c);
    T rm = group_rot<P, ST, false>(r, gbase, c);
    T lp = group_rot<P, ST, true>(l, gbase, c);
    T up = group_rot<P, ST, true>(u, gbase, c);
    T rp = group_rot<P, ST, true>(r, gbase, c);
    if (!periodic && c < ST) { lm = 0; um = 0; rm = 0; }
    if (!periodic && c + ST >= P) { lp = 0; up = 0; rp = 0; }
    const T inv = fast_rcp((T)1 - l * um - u * lp);
    const T rn = (r - l * rm - u * rp) * inv;
    l = -l * lm * inv;
    u = -u * up * inv;
    r = rn;
    pcr<T, P, 2 * ST>(l, u, r, c, gbase, periodic);
  }
}

// Eliminate the line held by this lane's group: chunk c of the line, LDS
// column col (row i at col[i * NLP]), coefficient tables ca/cb/cc/cw laid out
// [row in chunk][chunk], shift mu, and the singular-line flags.
//
// The arithmetic is FP64 whatever the field type T: an FP32 field is widened
// on reading and rounded once on writing.  Gauss elimination amplifies
// rounding by up to the condition number of the line (about 1e5 for a
// 512-point Dirichlet line with a small shift), so FP32 recurrences would
// leave errors near 1e-2 and make iterative refinement slow; in FP64 the
// FP32 solve is limited by its transforms instead.  The kernel is bound by
// HBM traffic, which only the field type sets.
// The elimination of one line of N = RPC P rows, chunk c of it on this
// lane (the P lanes of a line are consecutive lanes of a wave): the rows of
// the chunk are read and written through xget(i) / xset(i, v) (registers or
// the tile), coefficient tables ca/cb/cc/cw in LDS laid out [row in
// chunk][chunk], shift mu, and the singular-line flags.  FENCE: keep each
// row's coefficient loads in its own step (long chunks held in the tile).
template <int RPC, int P, bool FENCE, typename Get, typename Set>
__device__ __forceinline__ void tri_line_solve(Get xget, Set xset, lptr<const double> coef, int c,
                                               double mu, int sing, int wave_sing, int periodic) {
  using R = double;
  constexpr int N = RPC * P;
  const int lane = threadIdx.x & 63;
  const int gbase = lane - c;
  auto row_fence = [] {
    if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
  };
  const lptr<const R> ca = coef, cb = coef + N, cc = coef + 2 * N, cw = coef + 3 * N;

  if (wave_sing) {   // project the right-hand side of the null-space line
    R sw = 0, swf = 0;
#pragma unroll
    for (int i = 0; i < RPC; ++i) {
      const R wi = cw[i * P + c];
      sw += wi;
      swf += wi * xget(i);
    }
    sw = line_sum<R, P>(sw);
    swf = line_sum<R, P>(swf);
    if (sing) {
      const R mean = swf / sw;
#pragma unroll
      for (int i = 0; i < RPC; ++i) xset(i, xget(i) - mean);
    }
  }

  // phase 1: interior rows 0 .. RPC-2, top-down; x <- d (eliminated rhs),
  // qv = spike of the previous interface, cp = c / pivot
  constexpr int NI = RPC - 1;
  R cp[NI], qv[NI];
  R r = fast_rcp(cb[c] + mu);
  R xp = xget(0) * r;
  xset(0, xp);
  qv[0] = ca[c] * r;
  cp[0] = cc[c] * r;
#pragma unroll
  for (int i = 1; i < NI; ++i) {
    const R ai = ca[i * P + c], bi = cb[i * P + c], ci = cc[i * P + c];
    r = fast_rcp(bi + mu - ai * cp[i - 1]);
    xp = (xget(i) - ai * xp) * r;
    xset(i, xp);
    qv[i] = -ai * qv[i - 1] * r;
    cp[i] = ci * r;
    row_fence();
  }
  // first-row values of y = R^-1 f, v = R^-1 (a e_first), w = R^-1 (c e_last)
  const R yl = xp, vl = qv[NI - 1], wl = cc[(NI - 1) * P + c] * r;
  R yf = yl, vf = vl, wf = wl;
#pragma unroll
  for (int i = NI - 2; i >= 0; --i) {
    yf = xget(i) - cp[i] * yf;
    vf = qv[i] - cp[i] * vf;
    wf = -cp[i] * wf;
    row_fence();
  }

  // phase 2: interface row (last row of the chunk), reduced by PCR
  R ae = ca[NI * P + c], be = cb[NI * P + c] + mu, ce = cc[NI * P + c], fe = xget(NI);
  if (sing && c == P - 1) { ae = 0; be = 1; ce = 0; fe = 0; }   // pin x_{n-1} = 0
  const R yf_n = group_rot<P, 1, true>(yf, gbase, c);
  const R vf_n = group_rot<P, 1, true>(vf, gbase, c);
  const R wf_n = group_rot<P, 1, true>(wf, gbase, c);
  const R inv = fast_rcp(be - ae * wl - ce * vf_n);
  R lq = -ae * vl * inv;
  R uq = -ce * wf_n * inv;
  R rq = (fe - ae * yl - ce * yf_n) * inv;
  pcr<R, P, 1>(lq, uq, rq, c, gbase, periodic);
  // after the reduction the remaining couplings point back at this unknown
  const R Ic = periodic ? rq / ((R)1 + lq + uq) : rq;
  R Ip = group_rot<P, 1, false>(Ic, gbase, c);
  if (!periodic && c == 0) Ip = 0;

  // phase 3: back substitution of the interior
  xset(NI, Ic);
  R xn = yl - Ip * vl - Ic * wl;
  xset(NI - 1, xn);
#pragma unroll
  for (int i = NI - 2; i >= 0; --i) {
    xn = xget(i) - Ip * qv[i] - cp[i] * xn;
    xset(i, xn);
    row_fence();
  }

  if (wave_sing) {   // gauge: zero width-weighted mean of the null-space line
    R sw = 0, swx = 0;
#pragma unroll
    for (int i = 0; i < RPC; ++i) {
      const R wi = cw[i * P + c];
      sw += wi;
      swx += wi * xget(i);
    }
    sw = line_sum<R, P>(sw);
    swx = line_sum<R, P>(swx);
    if (sing) {
      const R mean = swx / sw;
#pragma unroll
      for (int i = 0; i < RPC; ++i) xset(i, xget(i) - mean);
    }
  }
}

// Eliminate the line held by this lane's group: chunk c of the line, LDS
// column col (row i at col[i * NLP]), coefficient tables ca/cb/cc/cw laid out
// [row in chunk][chunk], shift mu, and the singular-line flags.
//
// The arithmetic is FP64 whatever the field type T: an FP32 field is widened
// on reading and rounded once on writing.  Gauss elimination amplifies
// rounding by up to the condition number of the line (about 1e5 for a
// 512-point Dirichlet line with a small shift), so FP32 recurrences would
// leave errors near 1e-2 and make iterative refinement slow; in FP64 the
// FP32 solve is limited by its transforms instead.  The kernel is bound by
// HBM traffic, which only the field type sets.
template <typename T, int RPC, int P>
__device__ __forceinline__ void tri_fast_line(lptr<T> col, lptr<const double> coef, int c,
                                              double mu, int sing, int wave_sing, int periodic) {
  using L = TriFastLayout<T, RPC, P>;
  using R = double;
  // Long chunks of an FP64 field keep the eliminated right-hand side in the
  // tile (LDS) instead of registers: the pivots and spikes of RPC rows plus
  // RPC values would not fit 128 VGPRs.  FP32 fields keep it in registers
  // (the tile cannot hold FP64 intermediates).
  constexpr bool XL = sizeof(T) == 8 && RPC >= 12 && RPC * P >= 256;
  if constexpr (XL) {
    tri_line_solve<RPC, P, true>([&](int i) -> R { return (R)col[i * L::NLP]; },
                                 [&](int i, R v) { col[i * L::NLP] = (T)v; }, coef, c, mu, sing,
                                 wave_sing, periodic);
  } else {
    R xr[RPC];
#pragma unroll
    for (int i = 0; i < RPC; ++i) xr[i] = (R)col[i * L::NLP];
    tri_line_solve<RPC, P, false>([&](int i) -> R { return xr[i]; }, [&](int i, R v) { xr[i] = v; },
                                  coef, c, mu, sing, wave_sing, periodic);
#pragma unroll
    for (int i = 0; i < RPC; ++i) col[i * L::NLP] = (T)xr[i];
  }
}

// Coefficients of the elimination axis into LDS, [row in chunk][chunk];
// ends with a barrier.
template <typename T, int RPC, int P>
__device__ __forceinline__ void tri_fast_coefs(lptr<double> coef, const TriFastArgs<T>& A,
                                               int tid) {
  using L = TriFastLayout<T, RPC, P>;
  constexpr int N = L::N;
  for (int k = tid; k < N; k += L::NT) {
    const int ch = k / RPC, i = k - ch * RPC;
    const int s = i * P + ch;
    coef[s] = as_global(A.a)[k];
    coef[N + s] = as_global(A.b)[k];
    coef[2 * N + s] = as_global(A.c)[k];
    coef[3 * N + s] = as_global(A.w)[k];
  }
  __syncthreads();
}

// One tile of lines of the launch described by A, with the coefficients in
// LDS; ends with a barrier.
template <typename T, int RPC, int P, int LAY = -1>
__device__ __forceinline__ void tri_fast_tile(lptr<T> lds, lptr<const double> coef,
                                              const TriFastArgs<T>& A, int tile, int tid) {
  using L = TriFastLayout<T, RPC, P>;
  constexpr int N = L::N, NL = L::NL;
  LineGeom g = A.g;
  if (LAY >= 0) g.layout = LAY;   // a constant for the inlined geometry helpers
  const int c = tid % P;        // chunk of this thread
  const int l = tid / P;        // line of this thread within the tile
  const int nlt = 1 << g.lognl; // lines in a full tile of this launch (<= NL)
  const lptr<T> col = lds + c * L::CP + l;

  const TileOrigin o = tile_origin(g, tile);
  long long base;
  int lines = 0;
  if (g.layout == 0) {
    const int ll = tid % NL;
    base = ll < nlt ? line_base(g, o, ll) : -1;
  } else {
    base = (long long)o.L0 * g.n;   // g.n = N, or the real length of a padded line
    lines = min(g.nlines - o.L0, nlt);
  }
  tri_fast_load<T, RPC, P, LAY>(lds, as_global((const T*)A.data), base, g.sp, g.layout, lines, tid,
                                A.nreal);
  __syncthreads();

  const bool valid = l < nlt && line_base(g, o, l) >= 0;
  int u = 0, v = 0;
  if (valid) line_coords(g, o, l, A.nu, u, v);
  const double mu = valid ? A.lamu[u] + A.lamv[v] : -1.0;
  const bool sing = A.singular && valid && u == 0 && v == 0;
  const int wave_sing = __any(sing) ? 1 : 0;
  tri_fast_line<T, RPC, P>(col, coef, c, mu, sing ? 1 : 0, wave_sing, A.periodic);
  __syncthreads();

  tri_fast_store<T, RPC, P, LAY>(lds, as_global(A.data), base, g.sp, g.layout, lines, tid, A.nreal);
  __syncthreads();
}

template <typename T, int RPC, int P, int LAYOUT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
void tri_fast_kernel(TriFastArgs<T> A) {
  if (A.skip && A.skip[0] != 0.0) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const lptr<T> lds = as_lds(reinterpret_cast<T*>(smem_raw));
  const lptr<double> coef =
      as_lds(reinterpret_cast<double*>(smem_raw + tri_fast_coef_offset<T, RPC, P>()));
  const int tid = threadIdx.x;
  tri_fast_coefs<T, RPC, P>(coef, A, tid);
  const TileRange tr = xcd_tiles(A.g.ntiles);
  for (int tile = tr.first; tile < tr.end; tile += tr.step) {
    // chunks of 16 rows: thread index opaque per tile, so that the per-row
    // LDS addresses are recomputed in each tile instead of being held (and
    // spilled) across the loop; shorter chunks are faster with them held
    int t = tid;
    if constexpr (RPC >= 16) asm volatile("" : "+v"(t));
    tri_fast_tile<T, RPC, P, LAYOUT>(lds, coef, A, tile, t);
  }
}

// ---------------------------------------------------------------- direct form
// Contiguous lines only, no tile and no block barrier in the loop: each
// wave loops over its own groups of 64 / P lines (P lanes per line).  The
// group is one contiguous run of the field, read and written with
// coalesced 16-byte pieces (piece i + 64 k on lane i); the move between
// that order and the chunk order of the elimination (RPC consecutive
// points per lane) goes through a buffer of the wave's own in LDS, padded
// by one value per chunk so that the chunk reads and writes meet no bank
// conflicts.  The next group's loads are in flight while the current one
// is eliminated.  Only the coefficient tables are shared by the block.

template <typename T, int RPC>
struct DirectVec {
  static constexpr int BYTES = RPC * (int)sizeof(T);
  static_assert(BYTES % 16 == 0, "chunks of whole 16-byte pieces");
  static constexpr int PIECES = BYTES / 16;       // per lane and group
  static constexpr int PER = 16 / (int)sizeof(T); // values per piece
};

// Within-wave hand-off through LDS: the wave's LDS operations complete in
// issue order, so only the compiler must keep them in order.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

template <typename T, int RPC, int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
void tri_direct_kernel(TriFastArgs<T> A) {
  using V = DirectVec<T, RPC>;
  constexpr int N = RPC * P;
  constexpr int LPW = 64 / P;                  // lines per wave
  constexpr int WPB = 256 / 64;                // waves per block
  constexpr int GV = LPW * N;                  // values of a group
  constexpr int BUF = GV + GV / RPC;           // padded: one slot after every chunk
  if (A.skip && A.skip[0] != 0.0) return;
  __shared__ double coef_raw[4 * N];
  __shared__ T buf_raw[WPB * BUF];
  const lptr<double> coef = as_lds(coef_raw);
  for (int k = threadIdx.x; k < N; k += 256) {
    const int ch = k / RPC, i = k - ch * RPC;
    const int s = i * P + ch;
    coef[s] = as_global(A.a)[k];
    coef[N + s] = as_global(A.b)[k];
    coef[2 * N + s] = as_global(A.c)[k];
    coef[3 * N + s] = as_global(A.w)[k];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const lptr<T> wbuf = as_lds(buf_raw) + wave * BUF;
  const int c = lane % P;                      // chunk of this lane
  const int lw = lane / P;                     // line within the group
  const int groups = A.g.nlines / LPW;          // whole groups (checked at launch)
  const int gstep = gridDim.x * WPB;
  using Piece = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
  // The next group's pieces and eigenvalue shifts are read before the
  // current group's stores are issued, and placed after them, at the bottom
  // of the loop: the waits for those reads then leave the stores in flight.
  // With whole groups no lane skips a load or a store, so the compiler can
  // count them (a branch around them would make it wait for everything).
  Piece nxt[V::PIECES];
  double lu_n = 0.0, lv_n = 0.0;
  bool sing_n = false;
  // padded LDS slot of value e of the group
  auto slot = [](int e) { return e + e / RPC; };
  auto fetch = [&](int grp) {
    const Piece* src = reinterpret_cast<const Piece*>(A.data + (long long)grp * GV);
#pragma unroll
    for (int k = 0; k < V::PIECES; ++k) nxt[k] = src[lane + 64 * k];
    const int line = grp * LPW + lw;
    const int v = line / A.nu;
    const int u = line - v * A.nu;
    lu_n = A.lamu[u];
    lv_n = A.lamv[v];
    sing_n = A.singular && u == 0 && v == 0;
  };
  double xr[RPC];
  double mu = 0.0;
  bool sing = false;
  const int cb = slot(lw * N + c * RPC);
  // coalesced pieces -> chunk order, through the wave's buffer
  auto place = [&]() {
#pragma unroll
    for (int k = 0; k < V::PIECES; ++k) {
      const T* v = reinterpret_cast<const T*>(&nxt[k]);
      const int e0 = (lane + 64 * k) * V::PER;
#pragma unroll
      for (int e = 0; e < V::PER; ++e) wbuf[slot(e0 + e)] = v[e];
    }
    wave_lds_fence();
#pragma unroll
    for (int i = 0; i < RPC; ++i) xr[i] = (double)wbuf[cb + i];
    mu = lu_n + lv_n;
    sing = sing_n;
  };
  int grp = blockIdx.x * WPB + wave;
  if (grp < groups) {
    fetch(grp);
    place();
  }
  for (; grp < groups; grp += gstep) {
    const bool more = grp + gstep < groups;
    if (more) fetch(grp + gstep);
    const int wave_sing = __any(sing) ? 1 : 0;
    tri_line_solve<RPC, P, false>([&](int i) -> double { return xr[i]; },
                                  [&](int i, double x) { xr[i] = x; }, coef, c, mu,
                                  sing ? 1 : 0, wave_sing, A.periodic);
    // chunk order -> coalesced pieces
    wave_lds_fence();
#pragma unroll
    for (int i = 0; i < RPC; ++i) wbuf[cb + i] = (T)xr[i];
    wave_lds_fence();
    Piece* dst = reinterpret_cast<Piece*>(A.data + (long long)grp * GV);
#pragma unroll
    for (int k = 0; k < V::PIECES; ++k) {
      Piece out;
      T* o = reinterpret_cast<T*>(&out);
      const int e0 = (lane + 64 * k) * V::PER;
#pragma unroll
      for (int e = 0; e < V::PER; ++e) o[e] = wbuf[slot(e0 + e)];
      dst[lane + 64 * k] = out;
    }
    wave_lds_fence();
    if (more) place();
  }
}

// ---------------------------------------------------------------- async form
// The elimination with the next tile's HBM reads in flight while the current
// tile is eliminated: the tile is read straight into a staging area of LDS
// (stage_dma.h) and moved into its chunked place at the start of its turn.
// Everything is inlined (a call would wait for the staged reads), the
// eigenvalue shifts are kept in LDS for the same reason (a global load in
// the loop would wait for them too).  One block per CU.

static constexpr int TRI_ASYNC_LAM = 1024;   // longest transformed axis

template <typename T, int RPC, int P>
struct TriAsyncLayout {
  using L = TriFastLayout<T, RPC, P>;
  static constexpr int STAGE_BYTES = L::NL * L::N * (int)sizeof(T);
};

template <typename T, int RPC, int P, int LAYOUT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(1, 2)))
void tri_async_kernel(TriFastArgs<T> A) {
  using L = TriFastLayout<T, RPC, P>;
  using SL = StageLayout<T, L::NL, L::N>;
  constexpr int N = L::N, NL = L::NL, NT = L::NT;
  if (A.skip && A.skip[0] != 0.0) return;
  __shared__ __align__(16) unsigned char stage_raw[SL::BYTES];
  __shared__ __align__(16) T tile_raw[L::TILE];
  __shared__ __align__(16) double coef_raw[4 * N];
  __shared__ double lam_raw[2 * TRI_ASYNC_LAM];
  const lptr<T> lds = as_lds(tile_raw);
  const lptr<double> coef = as_lds(coef_raw);
  const lptr<double> lam = as_lds(lam_raw);
  const lptr<const T> stage = as_lds(reinterpret_cast<const T*>(stage_raw));
  const lptr<unsigned char> stage_lds = as_lds(stage_raw);
  const int tid0 = threadIdx.x;
  LineGeom g = A.g;
  g.layout = LAYOUT;   // one kernel per layout: its branches are constants
  const int nlt = 1 << g.lognl;

  for (int i = tid0; i < A.nu; i += NT) lam[i] = as_global(A.lamu)[i];
  for (int i = tid0; i < A.nv; i += NT) lam[TRI_ASYNC_LAM + i] = as_global(A.lamv)[i];
  tri_fast_coefs<T, RPC, P>(coef, A, tid0);   // (ends with a barrier)

  const TileRange tr = xcd_tiles(g.ntiles);
  if (tr.first < tr.end) stage_fetch<T, NL, N>(stage_lds, A.data, g, tr.first, tid0);
  // stores of the previous tile, issued after the staged reads: RPC per
  // thread when the tile was whole, else none counted
  bool stores_pending = false;
  for (int tile = tr.first; tile < tr.end; tile += tr.step) {
    // thread indices opaque per tile: the compiler recomputes the addresses
    // instead of holding them all live across the loop (registers)
    int tid = tid0;
    asm volatile("" : "+v"(tid));
    const int c = tid % P;
    const int l = tid / P;
    const lptr<T> col = lds + c * L::CP + l;
    // this wave's staged reads are done (the previous tile's stores may not be)
    if (stores_pending) vm_wait_keep<RPC>();
    else __builtin_amdgcn_s_waitcnt(0);
    lds_barrier();                   // ... and every wave's
    if (g.layout == 0) {
      const int ll = tid % NL, q = tid / NL;
#pragma unroll
      for (int i = 0; i < RPC; ++i)
        lds[tri_fast_slot<T, RPC, P>(q + i * P, ll)] = stage[(q + i * P) * NL + ll];
    } else {
#pragma unroll
      for (int i = 0; i < RPC; ++i) {
        const int e = tid + i * NT;
        const int ll = e / N;
        lds[tri_fast_slot<T, RPC, P>(e - ll * N, ll)] = stage[e];
      }
    }
    lds_barrier();
    if (tile + tr.step < tr.end) stage_fetch<T, NL, N>(stage_lds, A.data, g, tile + tr.step, tid);

    const TileOrigin o = tile_origin(g, tile);
    const bool valid = l < nlt && line_base(g, o, l) >= 0;
    int u = 0, v = 0;
    if (valid) line_coords(g, o, l, A.nu, u, v);
    const double mu = valid ? lam[u] + lam[TRI_ASYNC_LAM + v] : -1.0;
    const bool sing = A.singular && valid && u == 0 && v == 0;
    const int wave_sing = __any(sing) ? 1 : 0;
    tri_fast_line<T, RPC, P>(col, coef, c, mu, sing ? 1 : 0, wave_sing, A.periodic);
    lds_barrier();

    long long base;
    int lines = 0;
    if (g.layout == 0) {
      const int ll = tid % NL;
      base = ll < nlt ? line_base(g, o, ll) : -1;
    } else {
      base = (long long)o.L0 * N;
      lines = min(g.nlines - o.L0, nlt);
    }
    tri_fast_store_body<T, RPC, P>(lds, as_global(A.data), base, g.sp, g.layout, lines, tid,
                                   A.nreal);
    // strided tiles: every wave holds line 0, which always exists, so it
    // issues all RPC stores; contiguous tiles only when no line is missing
    stores_pending = g.layout == 0 || lines >= NL;
    lds_barrier();
  }
}

}  // namespace poisson_dev
