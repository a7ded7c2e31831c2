// tridiag_kernel.h - Gauss elimination of the reduced systems of
// Eq. (poi_reduced) along the elimination axis s, on gfx950.
//
// For every line (a column of fixed transformed wavenumbers (u, v)) solve
//   a_k x_{k-1} + (b_k + mu) x_k + c_k x_{k+1} = f_k,   k = 0 .. n-1,
// mu = lam_u[u] + lam_v[v] (Table 1 eigenvalues over the spacing squared),
// with a_0 and c_{n-1} the periodic wrap couplings (zero on a walled axis).
//
// A tile of nl lines is staged in LDS.  Each line is cut into P chunks
// (P a power of two <= 64), one per lane of a group of P consecutive lanes of
// a wavefront, so the whole line is eliminated by P threads at once:
//  phase 1  every chunk eliminates its interior rows (all rows but the last)
//           top-down with no pivoting (the rows are weakly diagonally
//           dominant: every mu <= 0), keeping the forward-eliminated
//           right-hand side in LDS and the pivot ratios in registers, and
//           expresses its interior as x = y - I_prev v - I_this w in terms of
//           the unknowns at the chunk interfaces (its own last row I_this and
//           the previous chunk's last row I_prev);
//  phase 2  the P interface equations form a tridiagonal system (cyclic on
//           a periodic axis) solved by parallel cyclic reduction with
//           cross-lane shuffles inside the group;
//  phase 3  every chunk back-substitutes its interior with the known
//           interface values.
// The line of wavenumber (0, 0) of a singular problem (no Dirichlet face) is
// projected (its width-weighted mean removed), its last unknown pinned to
// zero, and the result shifted to zero width-weighted mean.
// LDS layout: chunk c of line l, row k of the chunk at c*cpitch + k*nlp + l,
// with an odd cpitch so that the P lanes of a group hit distinct banks.
#pragma once
#include "device_common.h"

namespace poisson_dev {

template <typename T>
struct TriArgs {
  T* data;
  LineGeom g;
  int P;              // chunks per line
  int lcmax;          // longest chunk (rows)
  int nlp;            // LDS row pitch
  int cpitch;         // LDS chunk pitch
  int periodic;
  int singular;
  int nu;             // extent of u (contiguous layout: line index = u + nu v)
  const T* a;         // [n]
  const T* b;         // [n]
  const T* c;         // [n]
  const T* w;         // [n] cell widths along s (gauge weights)
  const T* lamu;      // [extent of u]
  const T* lamv;      // [extent of v]
  const double* skip; // optional: when *skip != 0 the launch does nothing
  unsigned n_magic;   // ceil(2^32 / n)
};

__device__ __forceinline__ int chunk_start(int c, int n, int P) { return (c * n) / P; }

template <typename T>
__device__ __forceinline__ T shfl(T v, int src) { return __shfl(v, src, 64); }

template <typename T>
__device__ __forceinline__ T group_sum(T v, int P) {
  for (int off = 1; off < P; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Tile load / store: all global loads (LDS reads) of a thread issued before
// the first LDS write (global store); not inlined, so that nothing of them
// stays live through the elimination.
template <typename T, int EPT, int NT>
__device__ __noinline__ void tri_load_tile(T* lds, const T* __restrict__ data, GEOM_PARAMS,
                                           int tile, const int* rowoff, unsigned n_magic,
                                           int tid) {
  const LineGeom g = GEOM_REBUILD;
  const TileOrigin o = tile_origin(g, tile);
  const int nl = 1 << g.lognl;
  const long long sbase = g.layout == 0 ? line_base(g, o, tid & (nl - 1)) : 0;
  T buf[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    int ll, p;
    const long long off = tile_elem<NT>(g, o, sbase, n_magic, tid, i, ll, p);
    buf[i] = off >= 0 ? as_global(data)[off] : (T)0;
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    int ll, p;
    tile_elem<NT>(g, o, sbase, n_magic, tid, i, ll, p);
    if (p < g.n && ll < nl) as_lds(lds)[as_lds(rowoff)[p] + ll] = buf[i];
  }
}

template <typename T, int EPT, int NT>
__device__ __noinline__ void tri_store_tile(const T* lds, T* __restrict__ data, GEOM_PARAMS,
                                            int tile, const int* rowoff, unsigned n_magic,
                                            int tid) {
  const LineGeom g = GEOM_REBUILD;
  const TileOrigin o = tile_origin(g, tile);
  const int nl = 1 << g.lognl;
  const long long sbase = g.layout == 0 ? line_base(g, o, tid & (nl - 1)) : 0;
  T buf[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    int ll, p;
    tile_elem<NT>(g, o, sbase, n_magic, tid, i, ll, p);
    buf[i] = (p < g.n && ll < nl) ? as_lds(lds)[as_lds(rowoff)[p] + ll] : (T)0;
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    int ll, p;
    const long long off = tile_elem<NT>(g, o, sbase, n_magic, tid, i, ll, p);
    if (off >= 0) as_global(data)[off] = buf[i];
  }
}

template <typename T, int LC, int NT>
// at least 4 waves per SIMD: two 512-thread tiles resident per CU
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
void tridiag_kernel(TriArgs<T> A) {
  if (A.skip && A.skip[0] != 0.0) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int tid = threadIdx.x;
  const LineGeom& g = A.g;
  const int n = g.n, nl = 1 << g.lognl, nlp = A.nlp, P = A.P, cpitch = A.cpitch;
  T* __restrict__ data = A.data;
  const int lane = tid & 63;
  const int c = lane & (P - 1);                   // chunk of this thread
  const int gbase = lane - c;                     // first lane of the group
  const int l = (tid >> 6) * (64 / P) + (lane / P);   // line of this thread
  const int s0 = chunk_start(c, n, P);
  const int e0 = chunk_start(c + 1, n, P) - 1;    // interface row
  const int ni = e0 - s0;                         // interior rows (< LC)
  T* col = lds + c * cpitch + l;                  // row k of my chunk: col[k * nlp]

  // LDS offset of every row of a line (chunk block + row within the chunk)
  int* rowoff = reinterpret_cast<int*>(lds + P * cpitch);
  if (tid < P) {
    const int a0 = chunk_start(tid, n, P), a1 = chunk_start(tid + 1, n, P);
    for (int r = a0; r < a1; ++r) rowoff[r] = tid * cpitch + (r - a0) * nlp;
  }
  __syncthreads();

  // tile values per thread: nl * n / NT = n / P <= lcmax <= LC + 1
  constexpr int EPT = LC + 1;
  const unsigned n_magic = A.n_magic;

  const TileRange tr = xcd_tiles(g.ntiles);
  for (int tile = tr.first; tile < tr.end; tile += tr.step) {
    const TileOrigin o = tile_origin(g, tile);
    tri_load_tile<T, EPT, NT>(lds, data, GEOM_ARGS(g), tile, rowoff, n_magic, tid);
    __syncthreads();

    // this line's shift and status
    const bool valid = l < nl && line_base(g, o, l) >= 0;
    int u = 0, v = 0;
    if (valid) line_coords(g, o, l, A.nu, u, v);
    const T mu = valid ? A.lamu[u] + A.lamv[v] : (T)-1;
    const bool sing = A.singular && valid && u == 0 && v == 0;
    const bool wave_sing = __any(sing);

    if (wave_sing) {   // project the right-hand side of the null-space line
      T sw = 0, swf = 0;
      for (int k = 0; k <= ni; ++k) {
        const T wk = A.w[s0 + k];
        sw += wk;
        swf += wk * col[k * nlp];
      }
      sw = group_sum(sw, P);
      swf = group_sum(swf, P);
      if (sing) {
        const T mean = swf / sw;
        for (int k = 0; k <= ni; ++k) col[k * nlp] -= mean;
      }
    }

    // phase 1: top-down elimination of the interior rows s0 .. e0-1
    T cp[LC], qv[LC];
    T dprev = 0, qprev = 0, cprev = 0, rlast = 0;
#pragma unroll
    for (int i = 0; i < LC; ++i) {
      cp[i] = 0;
      qv[i] = 0;
      if (i < ni) {
        const int k = s0 + i;
        const T ak = A.a[k];
        const T bk = A.b[k] + mu;
        const T ck = A.c[k];
        const T f = col[i * nlp];
        const T den = i > 0 ? bk - ak * cprev : bk;
        const T r = (T)1 / den;
        const T d = (i > 0 ? f - ak * dprev : f) * r;
        const T q = (i > 0 ? -ak * qprev : ak) * r;
        col[i * nlp] = d;
        cp[i] = ck * r;
        qv[i] = q;
        cprev = cp[i];
        dprev = d;
        qprev = q;
        rlast = r;
      }
    }
    // end values of y = T^-1 f, v = T^-1 (a_s e_first), w = T^-1 (c_{e-1} e_last)
    T yl = 0, vl = 0, wl = 0, yf = 0, vf = 0, wf = 0;
    if (ni > 0) {
      yl = dprev;
      vl = qprev;
      wl = A.c[e0 - 1] * rlast;
      yf = yl;
      vf = vl;
      wf = wl;
#pragma unroll
      for (int i = LC - 2; i >= 0; --i) {
        if (i < ni - 1) {
          yf = col[i * nlp] - cp[i] * yf;
          vf = qv[i] - cp[i] * vf;
          wf = -cp[i] * wf;
        }
      }
    }
    const T wq = wl;    // forward-eliminated w right-hand side at the last interior row

    // phase 2: interface equation of row e0
    T ae = A.a[e0], be = A.b[e0] + mu, ce = A.c[e0], fe = col[ni * nlp];
    if (sing && c == P - 1) { ae = 0; be = 1; ce = 0; fe = 0; }   // pin x_{n-1} = 0
    const int nxt = gbase + ((c + 1) & (P - 1));
    const T yf_n = shfl(yf, nxt), vf_n = shfl(vf, nxt), wf_n = shfl(wf, nxt);
    T Lq = -ae * vl;
    T Dq = be - ae * wl - ce * vf_n;
    T Uq = -ce * wf_n;
    T Rq = fe - ae * yl - ce * yf_n;
    for (int st = 1; st < P; st <<= 1) {
      const int cm = c - st, cpl = c + st;
      const int srcm = gbase + (cm & (P - 1));
      const int srcp = gbase + (cpl & (P - 1));
      T Lm = shfl(Lq, srcm), Dm = shfl(Dq, srcm), Um = shfl(Uq, srcm), Rm = shfl(Rq, srcm);
      T Lp = shfl(Lq, srcp), Dp = shfl(Dq, srcp), Up = shfl(Uq, srcp), Rp = shfl(Rq, srcp);
      if (!A.periodic && cm < 0) { Lm = 0; Dm = 1; Um = 0; Rm = 0; }
      if (!A.periodic && cpl >= P) { Lp = 0; Dp = 1; Up = 0; Rp = 0; }
      const T k1 = Lq / Dm;
      const T k2 = Uq / Dp;
      const T Ln = -Lm * k1;
      const T Un = -Up * k2;
      Dq = Dq - Um * k1 - Lp * k2;
      Rq = Rq - Rm * k1 - Rp * k2;
      Lq = Ln;
      Uq = Un;
    }
    // after the reduction the remaining couplings point back at this unknown
    const T Ic = Rq / (A.periodic ? Lq + Dq + Uq : Dq);
    const int prv = gbase + ((c - 1) & (P - 1));
    T Ip = shfl(Ic, prv);
    if (!A.periodic && c == 0) Ip = 0;

    // phase 3: back substitution of the interior
    if (ni > 0) {
      T x = dprev - Ip * qprev - Ic * wq;
      col[(ni - 1) * nlp] = x;
#pragma unroll
      for (int i = LC - 2; i >= 0; --i) {
        if (i < ni - 1) {
          x = col[i * nlp] - Ip * qv[i] - cp[i] * x;
          col[i * nlp] = x;
        }
      }
    }
    col[ni * nlp] = Ic;

    if (wave_sing) {   // gauge: zero width-weighted mean of the null-space line
      T sw = 0, swx = 0;
      for (int k = 0; k <= ni; ++k) {
        const T wk = A.w[s0 + k];
        sw += wk;
        swx += wk * col[k * nlp];
      }
      sw = group_sum(sw, P);
      swx = group_sum(swx, P);
      if (sing) {
        const T mean = swx / sw;
        for (int k = 0; k <= ni; ++k) col[k * nlp] -= mean;
      }
    }
    __syncthreads();

    tri_store_tile<T, EPT, NT>(lds, data, GEOM_ARGS(g), tile, rowoff, n_magic, tid);
    __syncthreads();
  }
}

}  // namespace poisson_dev
