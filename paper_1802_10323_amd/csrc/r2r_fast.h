// r2r_fast.h - size-specialised version of the batched real-to-real
// transforms (Table 2 / Table 1) for the common lengths n = 2M,
// M in {16, 32, 48, 64, 96, 128, 192, 256}, and for single solves also
// M in {72, 80, 144, 160} (radix-3 and radix-5 passes).
//
// Same mathematics as r2r_kernel.h (one complex FFT of length M per line
// plus the per-type pre/post steps), but the FFT length, its radix plan,
// the lines per tile (NL) and the threads per line (QT) are compile-time
// constants of each (non-inlined) stage, so LDS offsets, twiddle indices and
// loop counts fold to constants.  A persistent block copies its twiddle
// tables into LDS once and then loops over tiles.  The pre-steps (inverse
// combine, DCT-IV pre-twiddle) are done while the tile is brought into LDS
// and the post-steps (forward split, DCT-IV post-twiddle) while it is
// written out, so the FFT passes are the only LDS round trips in between.
// Two kernel forms: r2r_fast_kernel reads each tile from HBM when it starts
// on it; the staging kernels (r2r_async_kernel, n = 256 and 512) have the
// next tile's reads in flight during the current tile.
//
// LDS per block: the tile (2M rows of NL+1 values) plus 3M complex twiddles:
// the FFT table (M) and either the DCT-IV pre/post tables (M + M) or half
// of the even/odd split table (M/2 + 1, the other half follows from
// w_{M-k} = -conj(w_k)) and the quarter-wave table (M + 1).  For M = 256 in
// FP64 that is exactly 80 KiB, so two blocks share a CU.
//
// Thread t of NT = QT*NL works on line l = t mod NL (consecutive lanes =
// consecutive lines, i.e. consecutive x on a strided axis) and handles the
// butterflies / elements q, q + QT, q + 2 QT, ... of that line, q = t / NL.
// The fused pre/post steps on the contiguous axis instead put a line's
// points on consecutive lanes (line t / QT, element t mod QT), matching the
// line-major order of the data there.
#pragma once
#include <type_traits>
#include "r2r_kernel.h"
#include "stage_dma.h"

namespace poisson_dev {

// ---------------------------------------------------------------- radix plan

struct RadixPlan {
  int count;
  int r[12];
};

// mode 0: as many radix-8 passes as possible (then 4, 2); mode 1: radix 4
// (then one radix 2); radix 3 and 5 passes last.
constexpr RadixPlan make_radix_plan(int m, int mode) {
  RadixPlan p{0, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};
  int e2 = 0;
  while (m % 2 == 0) { m /= 2; ++e2; }
  int n8 = e2 / 3, n4 = 0, n2 = 0;
  const int rem = e2 % 3;
  if (rem == 1) {
    if (n8 > 0) { --n8; n4 = 2; } else { n2 = 1; }
  }
  if (rem == 2) n4 = 1;
  if (mode == 1) {
    n8 = 0;
    n4 = e2 / 2;
    n2 = e2 % 2;
  }
  int n16 = 0;
  if (mode == 2) {   // radix 16 first, the rest as one radix 2, 4 or 8
    n16 = e2 / 4;
    n8 = e2 % 4 == 3 ? 1 : 0;
    n4 = e2 % 4 == 2 ? 1 : 0;
    n2 = e2 % 4 == 1 ? 1 : 0;
  }
  for (int i = 0; i < n16; ++i) p.r[p.count++] = 16;
  for (int i = 0; i < n8; ++i) p.r[p.count++] = 8;
  for (int i = 0; i < n4; ++i) p.r[p.count++] = 4;
  for (int i = 0; i < n2; ++i) p.r[p.count++] = 2;
  while (m % 3 == 0) { m /= 3; p.r[p.count++] = 3; }
  while (m % 5 == 0) { m /= 5; p.r[p.count++] = 5; }
  return p;
}

constexpr int plan_ns(const RadixPlan& p, int pass) {
  int ns = 1;
  for (int i = 0; i < pass; ++i) ns *= p.r[i];
  return ns;
}

// Compile-time configuration of the specialised kernel: complex length M,
// threads per line QT, lines per tile NL (QT * NL = 512 threads) and the
// radix order of the FFT (MODE 0: radix 8 first, MODE 1: radix 4 first,
// MODE 2: radix 16 first).
template <int M_, int QT_, int NL_, int MODE_>
struct FastCfg {
  static constexpr int M = M_, QT = QT_, NL = NL_, MODE = MODE_;
  static_assert(QT * NL == 512, "transform blocks have 512 threads (the batched kernel relies on it)");
  static_assert(M % QT == 0, "whole complex values per thread");
};

// The four variants of each length that the autotuner chooses from:
// bit 0 selects the tile shape (base or alternative), bit 1 the radix order.
template <int M>
struct FastShapes;
#define POISSON_FAST_SHAPES(M_, QT0, NL0, QT1, NL1) \
  template <>                                       \
  struct FastShapes<M_> {                           \
    static constexpr int QT[2] = {QT0, QT1};        \
    static constexpr int NL[2] = {NL0, NL1};        \
  };
POISSON_FAST_SHAPES(16, 4, 128, 8, 64)
POISSON_FAST_SHAPES(32, 4, 128, 8, 64)
POISSON_FAST_SHAPES(48, 8, 64, 16, 32)
POISSON_FAST_SHAPES(64, 8, 64, 16, 32)
POISSON_FAST_SHAPES(96, 16, 32, 32, 16)
POISSON_FAST_SHAPES(128, 16, 32, 32, 16)
POISSON_FAST_SHAPES(192, 32, 16, 64, 8)
POISSON_FAST_SHAPES(256, 32, 16, 64, 8)
// lengths 2M with a factor 5 or 9 (radix-5 / radix-3 passes), one tile
// shape each: QT must be a power of two dividing M, and a thread's M/QT
// complex values must fit the registers (10 or more spill to scratch)
POISSON_FAST_SHAPES(72, 8, 64, 8, 64)
POISSON_FAST_SHAPES(80, 16, 32, 16, 32)
POISSON_FAST_SHAPES(144, 16, 32, 16, 32)
POISSON_FAST_SHAPES(160, 32, 16, 32, 16)
#undef POISSON_FAST_SHAPES

template <int M, int V>
using FastVar = FastCfg<M, FastShapes<M>::QT[V & 1], FastShapes<M>::NL[V & 1], (V >> 1) & 1>;

// Tile shape of the staging transform (shape 0 and 1: those of FastVar;
// shape 2: FP32 length 512 with 32 lines per tile, so that the rows of a
// strided tile are 128 bytes long, as in FP64 with 16 lines).
template <int M, int SHAPE>
using AsyncVar = std::conditional_t<SHAPE == 2, FastCfg<M, 16, 32, 2>, FastVar<M, SHAPE>>;

template <typename T>
struct R2RFastArgs {
  T* data;
  LineGeom g;
  int kind;
  int inverse;
  T scale;
  const cplx<T>* tw_fft;     // M
  const cplx<T>* tw_split;   // M + 1
  const cplx<T>* tw_quarter; // M + 1
  const cplx<T>* tw_pre;     // M
  const cplx<T>* tw_post;    // M
  const double* skip;
  double* out64;             // optional (FP32): write the widened result there, not in data
};

template <typename T, typename C>
struct FastLayout {
  static constexpr int M = C::M;
  static constexpr int QT = C::QT, NL = C::NL;
  static constexpr int NT = QT * NL;
  static constexpr int N = 2 * M;
  static constexpr int NLP = NL + 1;         // odd LDS row pitch
  static constexpr int E = M / QT;           // complex values per thread
  static constexpr int EPT = 2 * E;          // tile reals per thread
  static constexpr int TILE = N * NLP;       // reals of the tile in LDS
  static constexpr int AUX = 2 * M;          // pre/post or split/quarter tables (complex)
  static constexpr int SPLIT = M / 2 + 1;    // split-table entries kept in LDS
  static constexpr RadixPlan plan = make_radix_plan(M, C::MODE);
  static_assert(SPLIT + M + 1 <= AUX, "split + quarter tables exceed the LDS slot");
};

template <typename T, typename C>
constexpr size_t fast_lds_bytes() {
  using L = FastLayout<T, C>;
  [[maybe_unused]] constexpr int M = L::M;
  return (size_t)L::TILE * sizeof(T) + (size_t)(M + L::AUX) * sizeof(cplx<T>);
}

// complex element i of an LDS table (address-space structs are read and
// written field by field)
template <typename T>
__device__ __forceinline__ cplx<T> ldc(lptr<const cplx<T>> p, int i) {
  return {p[i].re, p[i].im};
}
template <typename T>
__device__ __forceinline__ void stc(lptr<cplx<T>> p, int i, cplx<T> v) {
  p[i].re = v.re;
  p[i].im = v.im;
}

// ---------------------------------------------------------------- stages
// Each stage is a non-inlined function specialised on the sizes, so that it
// gets a register allocation of its own (a kernel inlining all stages and
// transform types needs far more registers than any one stage) and the
// call passes only a few scalars.

// One Stockham pass of radix R (Ns = NS) over the tile, in place in LDS.
template <typename T, typename C, int R, int NS, bool FWD>
__device__ __forceinline__ void fast_pass_body(lptr<T> lds, lptr<const cplx<T>> tw, int l, int q) {
  using L = FastLayout<T, C>;
  [[maybe_unused]] constexpr int M = L::M;
  constexpr int B = M / R;                       // butterflies per line
  constexpr int SB = (B + L::QT - 1) / L::QT;    // per thread
  constexpr int TS = M / (NS * R);               // twiddle stride
  cplx<T> v[SB][R];
#pragma unroll
  for (int s = 0; s < SB; ++s) {
    const int j = q + s * L::QT;
    if (B % L::QT == 0 || j < B) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int idx = j + r * B;
        v[s][r] = {lds[(2 * idx) * L::NLP + l], lds[(2 * idx + 1) * L::NLP + l]};
      }
      if (NS > 1) {
        const int k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cplx<T> w = ldc(tw, r * k * TS);
          if (!FWD) w.im = -w.im;
          v[s][r] = cmul(v[s][r], w);
        }
      }
    }
  }
  lds_barrier();
#pragma unroll
  for (int s = 0; s < SB; ++s) {
    const int j = q + s * L::QT;
    if (B % L::QT == 0 || j < B) {
      SmallDFT<R, T, FWD>::run(v[s]);
      const int k = NS > 1 ? j % NS : 0;
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int idx = base + r * NS;
        lds[(2 * idx) * L::NLP + l] = v[s][r].re;
        lds[(2 * idx + 1) * L::NLP + l] = v[s][r].im;
      }
    }
  }
  lds_barrier();
}

template <typename T, typename C, int R, int NS, bool FWD>
__device__ __noinline__ void fast_pass_call(lptr<T> lds, lptr<const cplx<T>> tw, int l, int q) {
  fast_pass_body<T, C, R, NS, FWD>(lds, tw, l, q);
}

// INL: inline the stage (async kernel) or call its non-inlined copy
template <typename T, typename C, int R, int NS, bool FWD, bool INL = false>
__device__ __forceinline__ void fast_pass(lptr<T> lds, lptr<const cplx<T>> tw, int l, int q) {
  if constexpr (INL) fast_pass_body<T, C, R, NS, FWD>(lds, tw, l, q);
  else fast_pass_call<T, C, R, NS, FWD>(lds, tw, l, q);
}

template <typename T, typename C, bool FWD, int P, bool INL = false>
__device__ __forceinline__ void fast_passes(lptr<T> lds, lptr<const cplx<T>> tw, int l, int q) {
  using L = FastLayout<T, C>;
  [[maybe_unused]] constexpr int M = L::M;
  if constexpr (P < L::plan.count) {
    constexpr int R = L::plan.r[P];
    constexpr int NS = plan_ns(L::plan, P);
    fast_pass<T, C, R, NS, FWD, INL>(lds, tw, l, q);
    fast_passes<T, C, FWD, P + 1, INL>(lds, tw, l, q);
  }
}

// Tile load: global -> LDS rows with the input permutation of the type.
// All of a thread's loads are issued before its first LDS write.
template <typename T, typename C>
__device__ __forceinline__ void fast_load_body(lptr<T> lds, gptr<const T> data, long long base,
                                       long long sp, int layout, int lines, int kind,
                                       int inverse, int l, int q, int tid) {
  using L = FastLayout<T, C>;
  [[maybe_unused]] constexpr int M = L::M;
  constexpr int N = L::N;
  T buf[L::EPT];
  if (layout == 0) {
#pragma unroll
    for (int i = 0; i < L::EPT; ++i)
      buf[i] = base >= 0 ? data[base + (q + i * L::QT) * sp] : (T)0;
#pragma unroll
    for (int i = 0; i < L::EPT; ++i) {
      const int p = q + i * L::QT;
      bool neg;
      const int r = load_row(kind, inverse, p, N, neg);
      lds[r * L::NLP + l] = neg ? -buf[i] : buf[i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < L::EPT; ++i) {
      const int e = tid + i * L::NT;
      buf[i] = (e / N) < lines ? data[base + e] : (T)0;
    }
#pragma unroll
    for (int i = 0; i < L::EPT; ++i) {
      const int e = tid + i * L::NT;
      const int ll = e / N, p = e % N;
      bool neg;
      const int r = load_row(kind, inverse, p, N, neg);
      lds[r * L::NLP + ll] = neg ? -buf[i] : buf[i];
    }
  }
}

template <typename T, typename C>
__device__ __noinline__ void fast_load_call(lptr<T> lds, gptr<const T> data, long long base,
                                       long long sp, int layout, int lines, int kind,
                                       int inverse, int l, int q, int tid) {
  fast_load_body<T, C>(lds, data, base, sp, layout, lines, kind, inverse, l, q, tid);
}

// INL: inline the stage (async kernel) or call its non-inlined copy
template <typename T, typename C, bool INL = false>
__device__ __forceinline__ void fast_load(lptr<T> lds, gptr<const T> data, long long base,
                                       long long sp, int layout, int lines, int kind,
                                       int inverse, int l, int q, int tid) {
  if constexpr (INL) fast_load_body<T, C>(lds, data, base, sp, layout, lines, kind, inverse, l, q, tid);
  else fast_load_call<T, C>(lds, data, base, sp, layout, lines, kind, inverse, l, q, tid);
}

// Tile store: LDS rows -> global with the output permutation, sign, scale.
// O: the element type written (T, or double for the widened last pass of
// an FP32 solve).
template <typename T, typename C, typename O = T>
__device__ __forceinline__ void fast_store_body(lptr<const T> lds, gptr<O> data, long long base,
                                        long long sp, int layout, int lines, int kind,
                                        int inverse, T scale, int l, int q, int tid) {
  using L = FastLayout<T, C>;
  [[maybe_unused]] constexpr int M = L::M;
  constexpr int N = L::N;
  T buf[L::EPT];
  if (layout == 0) {
#pragma unroll
    for (int i = 0; i < L::EPT; ++i) {
      bool neg;
      const int r = store_row(kind, inverse, q + i * L::QT, N, neg);
      const T v = lds[r * L::NLP + l] * scale;
      buf[i] = neg ? -v : v;
    }
    if (base >= 0) {
#pragma unroll
      for (int i = 0; i < L::EPT; ++i) data[base + (q + i * L::QT) * sp] = (O)buf[i];
    }
  } else {   // two adjacent points of a line per lane (one 16-byte store for FP64)
#pragma unroll
    for (int i = 0; i < L::EPT; ++i) {
      const int e = 2 * (tid + (i >> 1) * L::NT) + (i & 1);
      const int ll = e / N, p = e % N;
      bool neg;
      const int r = store_row(kind, inverse, p, N, neg);
      const T v = lds[r * L::NLP + ll] * scale;
      buf[i] = neg ? -v : v;
    }
    const gptr<O> row = data + base;
#pragma unroll
    for (int i = 0; i < L::EPT; i += 2) {
      const int e = 2 * (tid + (i >> 1) * L::NT);   // even: e and e + 1 share a line
      if ((e / N) < lines) {
        row[e] = (O)buf[i];
        row[e + 1] = (O)buf[i + 1];
      }
    }
  }
}

template <typename T, typename C, typename O = T>
__device__ __noinline__ void fast_store_call(lptr<const T> lds, gptr<O> data, long long base,
                                        long long sp, int layout, int lines, int kind,
                                        int inverse, T scale, int l, int q, int tid) {
  fast_store_body<T, C, O>(lds, data, base, sp, layout, lines, kind, inverse, scale, l, q, tid);
}

// INL: inline the stage (async kernel) or call its non-inlined copy
template <typename T, typename C, bool INL = false, typename O = T>
__device__ __forceinline__ void fast_store(lptr<const T> lds, gptr<O> data, long long base,
                                        long long sp, int layout, int lines, int kind,
                                        int inverse, T scale, int l, int q, int tid) {
  if constexpr (INL)
    fast_store_body<T, C, O>(lds, data, base, sp, layout, lines, kind, inverse, scale, l, q, tid);
  else
    fast_store_call<T, C, O>(lds, data, base, sp, layout, lines, kind, inverse, scale, l, q, tid);
}

// Forward P/NN/DD, fused with the store: from Z (FFT of z_j = v_2j + i
// v_2j+1, the reordered line) the real DFT X_k of v, pairs (k, M-k) at
// once: with E = (Z_k + conj Z_{M-k})/2, O = -i (Z_k - conj Z_{M-k})/2 and
// w = e^{-2 pi i k/n}, X_k = E + w O and X_{M-k} = conj(E - w O); then the
// stored coefficients (Table 2's interleaving, or the quarter twiddle of
// DCT-II/DST-II), written straight to the field (the forward output order
// of these types is the tile's row order).  Strided layout: lines on
// consecutive lanes (rows of NL values); contiguous: a line's points on
// consecutive lanes.
template <typename T, typename C>
__device__ __forceinline__ void split_store_body(lptr<const T> lds, lptr<const cplx<T>> split,
                                                  lptr<const cplx<T>> quarter, int kind,
                                                  gptr<T> data, long long base, long long sp,
                                                  int layout, int lines, T scale, int l, int q,
                                                  int tid) {
  using L = FastLayout<T, C>;
  constexpr int M = L::M, N = L::N, NLP = L::NLP, QT = L::QT;
  constexpr int NP = M / 2 + 1;
  constexpr int SP = (NP + QT - 1) / QT;
  const int ln = layout == 0 ? l : tid / QT;
  const int qq = layout == 0 ? q : tid % QT;
  if (layout == 0 ? base < 0 : ln >= lines) return;   // line outside the field
  // the pairs of one thread, written through put(point, value)
  auto pairs = [&](auto put) {
#pragma unroll
    for (int s = 0; s < SP; ++s) {
      const int k = qq + s * QT;
      if (k < NP) {
        const int kc = (M - k) % M;
        const int j = M - k;
        const cplx<T> z = {lds[(2 * k) * NLP + ln], lds[(2 * k + 1) * NLP + ln]};
        const cplx<T> zc = {lds[(2 * kc) * NLP + ln], -lds[(2 * kc + 1) * NLP + ln]};
        const cplx<T> E = {(T)0.5 * (z.re + zc.re), (T)0.5 * (z.im + zc.im)};
        const cplx<T> D = csub(z, zc);
        const cplx<T> O = {(T)0.5 * D.im, (T)-0.5 * D.re};
        const cplx<T> wO = cmul(ldc(split, k), O);
        const cplx<T> X = cadd(E, wO);
        const cplx<T> Y = cconj(csub(E, wO));
        if (kind == K_P) {
          if (k == 0) {
            put(0, X.re);
            put(N - 1, Y.re);
          } else {
            put(2 * k - 1, X.re);
            put(2 * k, -X.im);
            if (j != k) {
              put(2 * j - 1, Y.re);
              put(2 * j, -Y.im);
            }
          }
        } else {
          const bool rev = kind == K_DD;
          const cplx<T> u = cmul(ldc(quarter, k), X);
          put(rev ? N - 1 - k : k, (T)2 * u.re);
          if (k > 0) put(rev ? k - 1 : N - k, (T)-2 * u.im);
          if (j != k) {
            const cplx<T> u2 = cmul(ldc(quarter, j), Y);
            put(rev ? N - 1 - j : j, (T)2 * u2.re);
            if (j != M) put(rev ? j - 1 : N - j, (T)-2 * u2.im);
          }
        }
      }
    }
  };
  if (layout == 0) {
    pairs([&](int r, T v) { data[base + r * sp] = v * scale; });
  } else {   // contiguous: the line's row pointer once, 32-bit offsets in it
    const gptr<T> row = data + (base + (long long)ln * N);
    pairs([&](int r, T v) { row[r] = v * scale; });
  }
}

// DCT-IV / DST-IV, fused with the store: V_k = Z_k times the post-twiddle;
// output point 2k is 2 Re V_k and point n-1-2k is -2 Im V_k (D-N: odd
// points change sign).  Lane mapping as in split_store_body.
template <typename T, typename C, typename O = T>
__device__ __forceinline__ void post_store_body(lptr<const T> lds, lptr<const cplx<T>> post,
                                                 int kind, gptr<O> data, long long base,
                                                 long long sp, int layout, int lines, T scale,
                                                 int l, int q, int tid) {
  using L = FastLayout<T, C>;
  constexpr int N = L::N, NLP = L::NLP, QT = L::QT;
  const int ln = layout == 0 ? l : tid / QT;
  const int qq = layout == 0 ? q : tid % QT;
  const long long lb = layout == 0 ? base : base + (long long)ln * N;
  const long long ps = layout == 0 ? sp : 1;
  if (layout == 0 ? base < 0 : ln >= lines) return;   // line outside the field
#pragma unroll
  for (int s = 0; s < L::E; ++s) {
    const int k = qq + s * QT;
    const cplx<T> V = cmul(cplx<T>{lds[(2 * k) * NLP + ln], lds[(2 * k + 1) * NLP + ln]},
                           ldc(post, k));
    const T ye = ((T)2 * V.re) * scale;      // point 2k (even)
    const T yo = ((T)-2 * V.im) * scale;     // point n-1-2k (odd)
    data[lb + (2 * k) * ps] = (O)ye;
    data[lb + (N - 1 - 2 * k) * ps] = (O)(kind == K_ND ? yo : -yo);
  }
}

// Non-inlined copies for the synchronous kernels (own register allocation).
template <typename T, typename C>
__device__ __noinline__ void split_store_call(lptr<const T> lds, lptr<const cplx<T>> split,
                                              lptr<const cplx<T>> quarter, int kind, gptr<T> data,
                                              long long base, long long sp, int layout, int lines,
                                              T scale, int l, int q, int tid) {
  split_store_body<T, C>(lds, split, quarter, kind, data, base, sp, layout, lines, scale, l, q, tid);
}

template <typename T, typename C, typename O = T>
__device__ __noinline__ void post_store_call(lptr<const T> lds, lptr<const cplx<T>> post, int kind,
                                             gptr<O> data, long long base, long long sp, int layout,
                                             int lines, T scale, int l, int q, int tid) {
  post_store_body<T, C, O>(lds, post, kind, data, base, sp, layout, lines, scale, l, q, tid);
}

// Inverse P/NN/DD, fused with the placement: from the stored coefficients
// X of a line (the real DFT of Table 2's storage, or the quarter-twiddled
// DCT-II/DST-II spectrum), the length-M complex spectrum
// Z'_k = (X_k + conj X_{M-k}) + i (X_k - conj X_{M-k}) e^{2 pi i k/n}
// whose inverse FFT interleaves the even and odd output points; written
// into the tile (column ln, pairs k = qq + s QT) from the input points of
// the line, point(p) (tile row r holds point r, D-D: point n-1-r).
//
// combine_read: the points thread qq needs, v[s] = the four rows of
// wavenumbers k = qq + s QT and M - k; combine_write: the math and the tile
// writes.
template <typename T, typename C>
struct CombineRegs {
  static constexpr int SP = (FastLayout<T, C>::M / 2 + 1 + FastLayout<T, C>::QT - 1) /
                            FastLayout<T, C>::QT;
  T v[SP][4];
};

template <typename T, typename C, typename Point>
__device__ __forceinline__ void combine_read(Point point, CombineRegs<T, C>& R, int kind, int qq) {
  using L = FastLayout<T, C>;
  constexpr int M = L::M, N = L::N, QT = L::QT;
  constexpr int NP = M / 2 + 1;
  auto row = [&](int r) -> T { return point(kind == K_DD ? N - 1 - r : r); };
#pragma unroll
  for (int s = 0; s < CombineRegs<T, C>::SP; ++s) {
    const int k = qq + s * QT;
    const int j = M - k;
    if (k < NP) {
      if (kind == K_P) {
        R.v[s][0] = row(k == 0 ? 0 : 2 * k - 1);
        R.v[s][1] = k == 0 ? (T)0 : row(2 * k);
        R.v[s][2] = row(j == M ? N - 1 : 2 * j - 1);
        R.v[s][3] = j == M ? (T)0 : row(2 * j);
      } else {
        R.v[s][0] = row(k);
        R.v[s][1] = k == 0 ? (T)0 : row(N - k);
        R.v[s][2] = row(j);
        R.v[s][3] = row(N - j);
      }
    }
  }
}

template <typename T, typename C>
__device__ __forceinline__ void combine_write(const CombineRegs<T, C>& R, lptr<T> lds,
                                              lptr<const cplx<T>> split,
                                              lptr<const cplx<T>> quarter, int kind, int ln,
                                              int qq) {
  using L = FastLayout<T, C>;
  constexpr int M = L::M, NLP = L::NLP, QT = L::QT;
  constexpr int NP = M / 2 + 1;
#pragma unroll
  for (int s = 0; s < CombineRegs<T, C>::SP; ++s) {
    const int k = qq + s * QT;
    if (k < NP) {
      const int j = M - k;
      cplx<T> xk, xj;
      if (kind == K_P) {
        xk = {R.v[s][0], k == 0 ? (T)0 : -R.v[s][1]};
        xj = {R.v[s][2], j == M ? (T)0 : -R.v[s][3]};
      } else {
        xk = cmul(cconj(ldc(quarter, k)), cplx<T>{(T)0.5 * R.v[s][0], (T)-0.5 * R.v[s][1]});
        xj = cmul(cconj(ldc(quarter, j)), cplx<T>{(T)0.5 * R.v[s][2], (T)-0.5 * R.v[s][3]});
      }
      const cplx<T> sk = ldc(split, k);
      const cplx<T> s1 = cadd(xk, cconj(xj));
      const cplx<T> d1 = cmul(csub(xk, cconj(xj)), cconj(sk));
      lds[(2 * k) * NLP + ln] = s1.re - d1.im;
      lds[(2 * k + 1) * NLP + ln] = s1.im + d1.re;
      if (k > 0 && j != k) {
        const cplx<T> s2 = cadd(xj, cconj(xk));
        const cplx<T> d2 = cmul(csub(cconj(xk), xj), sk);
        lds[(2 * j) * NLP + ln] = s2.re - d2.im;
        lds[(2 * j + 1) * NLP + ln] = s2.im + d2.re;
      }
    }
  }
}

// Both: all reads first (global reads stay in flight together), then the
// math.  SYNC: the points are read from the tile itself (a barrier between
// the reads and the writes).
template <typename T, typename C, bool SYNC = false, typename Point>
__device__ __forceinline__ void combine_to_tile(Point point, lptr<T> lds,
                                                lptr<const cplx<T>> split,
                                                lptr<const cplx<T>> quarter, int kind, int ln,
                                                int qq) {
  CombineRegs<T, C> R;
  combine_read<T, C>(point, R, kind, qq);
  if constexpr (SYNC) lds_barrier();
  combine_write<T, C>(R, lds, split, quarter, kind, ln, qq);
}

// Points read by pre_to_tile for thread qq: v[s] = the two points of
// complex index j = qq + s QT.
template <typename T, typename C>
struct PreRegs {
  T v[FastLayout<T, C>::E][2];
};

template <typename T, typename C, typename Point>
__device__ __forceinline__ void pre_read(Point point, PreRegs<T, C>& R, int kind, int qq) {
  using L = FastLayout<T, C>;
  constexpr int N = L::N, QT = L::QT;
#pragma unroll
  for (int s = 0; s < L::E; ++s) {
    const int j = qq + s * QT;
    R.v[s][0] = point(kind == K_ND ? 2 * j : N - 1 - 2 * j);
    R.v[s][1] = point(kind == K_ND ? N - 1 - 2 * j : 2 * j);
  }
}

template <typename T, typename C>
__device__ __forceinline__ void pre_write(const PreRegs<T, C>& R, lptr<T> lds,
                                          lptr<const cplx<T>> pre, int ln, int qq) {
  using L = FastLayout<T, C>;
  constexpr int NLP = L::NLP, QT = L::QT;
#pragma unroll
  for (int s = 0; s < L::E; ++s) {
    const int j = qq + s * QT;
    const cplx<T> z = cmul(cplx<T>{R.v[s][0], R.v[s][1]}, ldc(pre, j));
    lds[(2 * j) * NLP + ln] = z.re;
    lds[(2 * j + 1) * NLP + ln] = z.im;
  }
}

// The input step of the DCT-IV / DST-IV types: the pre-twiddled complex
// sequence of the half-length FFT, written into the tile (reads first;
// SYNC as for combine_to_tile).
template <typename T, typename C, bool SYNC = false, typename Point>
__device__ __forceinline__ void pre_to_tile(Point point, lptr<T> lds, lptr<const cplx<T>> pre,
                                            int kind, int ln, int qq) {
  PreRegs<T, C> R;
  pre_read<T, C>(point, R, kind, qq);
  if constexpr (SYNC) lds_barrier();
  pre_write<T, C>(R, lds, pre, ln, qq);
}

// The two above from global memory, for the synchronous kernels: the lanes
// run over lines on a strided axis (each load reads a row of NL values) and
// over a line's points on the contiguous one; lines outside the field read 0.
template <typename T, typename C>
__device__ __noinline__ void load_combine_call(lptr<T> lds, gptr<const T> data, long long base,
                                               long long sp, int layout, int lines,
                                               lptr<const cplx<T>> split,
                                               lptr<const cplx<T>> quarter, int kind, int l,
                                               int q, int tid) {
  using L = FastLayout<T, C>;
  constexpr int N = L::N, QT = L::QT;
  const int ln = layout == 0 ? l : tid / QT;
  const int qq = layout == 0 ? q : tid % QT;
  const long long lb = layout == 0 ? base : base + (long long)ln * N;
  const long long ps = layout == 0 ? sp : 1;
  const bool in = layout == 0 ? base >= 0 : ln < lines;
  auto point = [&](int p) -> T { return in ? data[lb + p * ps] : (T)0; };
  combine_to_tile<T, C>(point, lds, split, quarter, kind, ln, qq);
}

template <typename T, typename C>
__device__ __noinline__ void load_pre_call(lptr<T> lds, gptr<const T> data, long long base,
                                           long long sp, int layout, int lines,
                                           lptr<const cplx<T>> pre, int kind, int l, int q,
                                           int tid) {
  using L = FastLayout<T, C>;
  constexpr int N = L::N, QT = L::QT;
  const int ln = layout == 0 ? l : tid / QT;
  const int qq = layout == 0 ? q : tid % QT;
  const long long lb = layout == 0 ? base : base + (long long)ln * N;
  const long long ps = layout == 0 ? sp : 1;
  const bool in = layout == 0 ? base >= 0 : ln < lines;
  auto point = [&](int p) -> T { return in ? data[lb + p * ps] : (T)0; };
  pre_to_tile<T, C>(point, lds, pre, kind, ln, qq);
}

// ---------------------------------------------------------------- kernel

// LDS regions of the specialised transform: the tile, then the FFT twiddles
// (M), then the pre/post (DCT-IV types) or split/quarter tables (2M).
template <typename T, typename C>
struct FastLds {
  lptr<T> tile;
  lptr<cplx<T>> twf, twa;
};
template <typename T, typename C>
__device__ __forceinline__ FastLds<T, C> fast_lds(unsigned char* smem) {
  using L = FastLayout<T, C>;
  [[maybe_unused]] constexpr int M = L::M;
  FastLds<T, C> r;
  r.tile = as_lds(reinterpret_cast<T*>(smem));
  r.twf = as_lds(reinterpret_cast<cplx<T>*>(reinterpret_cast<T*>(smem) + L::TILE));
  r.twa = r.twf + M;
  return r;
}

// Twiddle tables of transform `kind` (those of the DCT-IV types, or those
// of the others) into LDS; ends with a barrier.  The values depend only on
// n = 2M and the type class.
template <typename T, typename C>
__device__ __forceinline__ void fast_twiddles(const FastLds<T, C>& S, const R2RFastArgs<T>& A,
                                              int tid) {
  using L = FastLayout<T, C>;
  [[maybe_unused]] constexpr int M = L::M;
  constexpr int NT = L::NT;
  for (int i = tid; i < M; i += NT) stc(S.twf, i, ldg(A.tw_fft, i));
  if (A.kind >= K_ND) {
    for (int i = tid; i < M; i += NT) {
      stc(S.twa, i, ldg(A.tw_pre, i));
      stc(S.twa, M + i, ldg(A.tw_post, i));
    }
  } else {
    for (int i = tid; i < L::SPLIT; i += NT) stc(S.twa, i, ldg(A.tw_split, i));
    for (int i = tid; i <= M; i += NT) stc(S.twa, L::SPLIT + i, ldg(A.tw_quarter, i));
  }
  lds_barrier();
}

// One tile of lines of the launch described by A, with the twiddles of its
// type class already in LDS; ends with a barrier.
template <typename T, typename C>
__device__ __forceinline__ void fast_tile(const FastLds<T, C>& S, const R2RFastArgs<T>& A,
                                          int tile, int tid) {
  using L = FastLayout<T, C>;
  [[maybe_unused]] constexpr int M = L::M;
  constexpr int NL = L::NL;
  const int l = tid % NL;
  const int q = tid / NL;
  const LineGeom& g = A.g;
  const int kind = A.kind, inverse = A.inverse;
  const bool ivk = kind >= K_ND;
  const lptr<const cplx<T>> tw_fft = S.twf;
  const lptr<const cplx<T>> tw_a = S.twa;                           // pre or split
  const lptr<const cplx<T>> tw_b = S.twa + (ivk ? M : L::SPLIT);    // post or quarter

  const TileOrigin o = tile_origin(g, tile);
  long long base;
  int lines = 0;
  if (g.layout == 0) {
    base = l < (1 << g.lognl) ? line_base(g, o, l) : -1;
  } else {
    base = (long long)o.L0 * L::N;
    lines = g.nlines - o.L0;
  }
  // the DCT-IV pre-twiddle and the inverse combine read the field directly
  if (ivk)
    load_pre_call<T, C>(S.tile, as_global((const T*)A.data), base, g.sp, g.layout, lines, tw_a,
                        kind, l, q, tid);
  else if (inverse)
    load_combine_call<T, C>(S.tile, as_global((const T*)A.data), base, g.sp, g.layout, lines,
                            tw_a, tw_b, kind, l, q, tid);
  else
    fast_load<T, C>(S.tile, as_global((const T*)A.data), base, g.sp, g.layout, lines, kind,
                    inverse, l, q, tid);
  lds_barrier();

  if (!(inverse && kind <= K_DD)) fast_passes<T, C, true, 0>(S.tile, tw_fft, l, q);
  else fast_passes<T, C, false, 0>(S.tile, tw_fft, l, q);

  // the DCT-IV post-twiddle and the forward split write the field directly;
  // an FP32 pass with out64 writes the widened values there instead
  bool widened = false;
  if constexpr (sizeof(T) == 4) {
    if (A.out64) {
      widened = true;
      if (ivk)
        post_store_call<T, C, double>(S.tile, tw_b, kind, as_global(A.out64), base, g.sp, g.layout,
                                      lines, A.scale, l, q, tid);
      else
        fast_store<T, C, false, double>(S.tile, as_global(A.out64), base, g.sp, g.layout, lines,
                                        kind, inverse, A.scale, l, q, tid);
    }
  }
  if (!widened) {
    if (ivk)
      post_store_call<T, C>(S.tile, tw_b, kind, as_global(A.data), base, g.sp, g.layout, lines,
                            A.scale, l, q, tid);
    else if (!inverse)
      split_store_call<T, C>(S.tile, tw_a, tw_b, kind, as_global(A.data), base, g.sp, g.layout,
                             lines, A.scale, l, q, tid);
    else
      fast_store<T, C>(S.tile, as_global(A.data), base, g.sp, g.layout, lines, kind, inverse,
                       A.scale, l, q, tid);
  }
  lds_barrier();
}

template <typename T, typename C>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
void r2r_fast_kernel(R2RFastArgs<T> A) {
  if (A.skip && A.skip[0] != 0.0) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const FastLds<T, C> S = fast_lds<T, C>(smem_raw);
  const int tid = threadIdx.x;
  fast_twiddles<T, C>(S, A, tid);
  const TileRange tr = xcd_tiles(A.g.ntiles);
  for (int tile = tr.first; tile < tr.end; tile += tr.step) fast_tile<T, C>(S, A, tile, tid);
}

// ---------------------------------------------------------------- async form
// The same transform with the next tile's HBM reads in flight while the
// current tile is transformed: global_load_lds moves the next tile straight
// into a staging area of LDS (no registers involved), the tile is copied
// from there into its permuted place at the start of its turn.  Needs LDS
// for the stage, the tile and the twiddles (one block per CU), 16-byte
// pieces that never straddle a line (strided axes: even nx in FP64, nx a
// multiple of 4 in FP32).

template <typename T, typename C>
struct AsyncLayout {
  using L = FastLayout<T, C>;
  static constexpr int EPL = 16 / (int)sizeof(T);            // elements per 16-byte piece
  static constexpr int STAGE = L::NL * L::N;                   // staged elements
  static constexpr int CHUNKS = STAGE * (int)sizeof(T) / 1024; // 1 KiB per wave instruction
  static constexpr int PER_WAVE = CHUNKS / (L::NT / 64);
  static constexpr int LANES_PER_ROW = L::NL / EPL;             // strided: pieces per row
  static constexpr int ROWS_PER_CHUNK = 64 / LANES_PER_ROW;
  static_assert(CHUNKS % (L::NT / 64) == 0, "stage chunks split evenly over the waves");
  static_assert(L::NL % EPL == 0 && 64 % LANES_PER_ROW == 0, "rows of whole pieces");
};

template <typename T, typename C>
constexpr size_t async_lds_bytes() {
  return (size_t)AsyncLayout<T, C>::STAGE * sizeof(T) + fast_lds_bytes<T, C>();
}

// Issue the reads of tile `tile` into the stage (asynchronous: completion
// is awaited by the vector-memory counter before the stage is read).
template <typename T, typename C>
__device__ __forceinline__ void async_fetch(lptr<unsigned char> stage, const R2RFastArgs<T>& A,
                                            int layout, int tile, int tid) {
  using AL = AsyncLayout<T, C>;
  using L = FastLayout<T, C>;
  const LineGeom& g = A.g;
  const TileOrigin o = tile_origin(g, tile);
  const int wave = tid >> 6, lane = tid & 63;
  const T* data = A.data;
  const int nlt = 1 << g.lognl;
#pragma unroll
  for (int j = 0; j < AL::PER_WAVE; ++j) {
    const int c = wave * AL::PER_WAVE + j;     // chunk of this instruction (wave-uniform)
    const T* src = data;                        // a valid address for pieces outside the field
    if (layout == 0) {
      const int row = c * AL::ROWS_PER_CHUNK + lane / AL::LANES_PER_ROW;
      const int l = (lane % AL::LANES_PER_ROW) * AL::EPL;
      const long long b = l < nlt ? line_base(g, o, l) : -1;
      if (b >= 0) src = data + b + (long long)row * g.sp;
    } else {
      const int e = (c * 64 + lane) * AL::EPL;
      if (e / L::N < g.nlines - o.L0 && e / L::N < nlt) src = data + (long long)o.L0 * L::N + e;
    }
    stage_dma16(src, (unsigned)(size_t)(stage + c * 1024));
  }
}

// Stage -> tile rows with the input permutation of the type.
template <typename T, typename C>
__device__ __forceinline__ void async_place(lptr<const T> stage, lptr<T> lds, int kind, int inverse,
                                            int layout, int l, int q, int tid) {
  using L = FastLayout<T, C>;
  constexpr int N = L::N;
  T buf[L::EPT];
  if (layout == 0) {
#pragma unroll
    for (int i = 0; i < L::EPT; ++i) buf[i] = stage[(q + i * L::QT) * L::NL + l];
#pragma unroll
    for (int i = 0; i < L::EPT; ++i) {
      bool neg;
      const int r = load_row(kind, inverse, q + i * L::QT, N, neg);
      lds[r * L::NLP + l] = neg ? -buf[i] : buf[i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < L::EPT; ++i) buf[i] = stage[tid + i * L::NT];
#pragma unroll
    for (int i = 0; i < L::EPT; ++i) {
      const int e = tid + i * L::NT;
      const int ll = e / N, p = e % N;
      bool neg;
      const int r = load_row(kind, inverse, p, N, neg);
      lds[r * L::NLP + ll] = neg ? -buf[i] : buf[i];
    }
  }
}

// The two above from the stage of the staging kernels.  The strided layout
// keeps the lines on consecutive lanes; the contiguous one puts a line's
// points on consecutive lanes (the stage holds whole lines there), so that
// both read the stage without bank conflicts.
template <typename T, typename C>
__device__ __forceinline__ void async_place_combine(lptr<const T> stage, lptr<T> lds,
                                                    lptr<const cplx<T>> split,
                                                    lptr<const cplx<T>> quarter, int kind,
                                                    int layout, int l, int q, int tid) {
  using L = FastLayout<T, C>;
  constexpr int N = L::N, NL = L::NL, QT = L::QT;
  const int ln = layout == 0 ? l : tid / QT;
  const int qq = layout == 0 ? q : tid % QT;
  auto point = [&](int p) -> T { return layout == 0 ? stage[p * NL + ln] : stage[ln * N + p]; };
  combine_to_tile<T, C>(point, lds, split, quarter, kind, ln, qq);
}

template <typename T, typename C>
__device__ __forceinline__ void async_place_pre(lptr<const T> stage, lptr<T> lds,
                                                lptr<const cplx<T>> pre, int kind, int layout,
                                                int l, int q, int tid) {
  using L = FastLayout<T, C>;
  constexpr int N = L::N, NL = L::NL, QT = L::QT;
  const int ln = layout == 0 ? l : tid / QT;
  const int qq = layout == 0 ? q : tid % QT;
  auto point = [&](int p) -> T { return layout == 0 ? stage[p * NL + ln] : stage[ln * N + p]; };
  pre_to_tile<T, C>(point, lds, pre, kind, ln, qq);
}

// The widened store of the last pass of an FP32 solve (staging kernels):
// the inverse output (or the DCT-IV post-twiddled one) as FP64 into
// A.out64.  FP32 only.
template <typename T, typename C, bool IVK>
__device__ __forceinline__ void async_store_wide(lptr<const T> lds, lptr<const cplx<T>> post,
                                                 int kind, int inverse, const R2RFastArgs<T>& A,
                                                 int layout, long long base, int lines, int l,
                                                 int q, int tid) {
  if constexpr (sizeof(T) == 4) {
    if constexpr (IVK)
      post_store_body<T, C, double>(lds, post, kind, as_global(A.out64), base, A.g.sp, layout,
                                    lines, A.scale, l, q, tid);
    else
      fast_store_body<T, C, double>(lds, as_global(A.out64), base, A.g.sp, layout, lines, kind,
                                    inverse, A.scale, l, q, tid);
  }
}

// Register budget of the staging kernel.  FP64 M = 256 in the 16-line tile
// shape (DFT and DCT-IV types): one block fills a CU's LDS, so the kernel may use up to 256 VGPRs
// and keep every stage's addresses live across the tile loop (fastest).  Otherwise the per-thread
// indices are made opaque at the top of each tile, so that the addresses are
// recomputed per stage and the kernel fits 128 VGPRs (FP64 M = 128 would
// spill otherwise; two FP32 blocks share a CU).
template <typename T, typename C, int KIND>
struct AsyncBudget {
  // (the DCT-II / DST-II pipelines of that length would spill)
  static constexpr bool WIDE = sizeof(T) == 8 && C::M == 256 && FastLayout<T, C>::NL == 16 &&
                               KIND != K_NN && KIND != K_DD;
};

// One kernel per transform type and direction: with the type a constant
// every stage inlines into a short straight-line pipeline (a call would make
// the callee wait for all outstanding memory operations, the next tile's
// reads included).  Two kernels per configuration, one per register budget
// (AsyncBudget): r2r_async_kernel keeps the thread's indices as they are,
// r2r_async_tight_kernel makes them opaque at the top of each tile.  The
// shared parts are macros so that both compile to the same straight code.
#define POISSON_ASYNC_SETUP                                                                    \
  using L = FastLayout<T, C>;                                                                  \
  using AL = AsyncLayout<T, C>;                                                                \
  constexpr int M = L::M, NL = L::NL;                                                          \
  constexpr int kind = KIND, inverse = INV;                                                    \
  constexpr int layout = LAYOUT;  /* 0 strided, 1 contiguous: one kernel each */              \
  if (A.skip && A.skip[0] != 0.0) return;                                                      \
  /* two LDS objects, so that the staged reads (asynchronous writes to */                     \
  /* stage_raw) are told apart from the accesses to the tile */                               \
  __shared__ __align__(16) unsigned char stage_raw[AL::STAGE * sizeof(T)];                     \
  __shared__ __align__(16) unsigned char tile_raw[fast_lds_bytes<T, C>()];                     \
  const lptr<const T> stage = as_lds(reinterpret_cast<const T*>(stage_raw));                   \
  const FastLds<T, C> S = fast_lds<T, C>(tile_raw);                                            \
  const int tid = threadIdx.x;                                                                 \
  const int l = tid % NL, q = tid / NL;                                                        \
  LineGeom g = A.g;                                                                            \
  g.layout = layout;             /* a constant for the inlined geometry helpers */             \
  constexpr bool ivk = kind >= K_ND;                                                           \
  const lptr<const cplx<T>> tw_fft = S.twf;                                                    \
  const lptr<const cplx<T>> tw_a = S.twa;                                                      \
  const lptr<const cplx<T>> tw_b = S.twa + (ivk ? M : L::SPLIT);                               \
  fast_twiddles<T, C>(S, A, tid);                                                              \
  const TileRange tr = xcd_tiles(g.ntiles);                                                    \
  const lptr<unsigned char> stage_lds = as_lds(stage_raw);                                     \
  if (tr.first < tr.end) async_fetch<T, C>(stage_lds, A, layout, tr.first, tid);              \
  /* Stores of the previous tile issued after the staged reads, a lower */                     \
  /* bound per wave for a whole tile (KEEP strided, KEEP_C contiguous): */                     \
  /* the plain and DCT-IV stores write every element (EPT) through a */                       \
  /* run-time stride, one instruction each, except the plain store on */                      \
  /* the contiguous axis, which writes two adjacent elements per lane */                      \
  /* (EPT/2 instructions at least); the forward split writes 4 points */                      \
  /* for every pair k of 1 <= k < M/2, and each wave has such lanes in */                     \
  /* each of the first M/(2 QT) steps: 4 instructions on the strided */                       \
  /* axis, at least 2 on the contiguous one (two adjacent points may */                       \
  /* become one store).  Ragged tiles keep nothing in flight. */                              \
  constexpr int KEEP = (ivk || inverse) ? L::EPT : 4 * (M / (2 * L::QT));                      \
  constexpr int KEEP_C = ivk ? L::EPT : inverse ? L::EPT / 2 : 2 * (M / (2 * L::QT));          \
  static_assert(KEEP_C >= 1 && KEEP < 64, "vector-memory counter range");                     \
  bool stores_pending = false;

#define POISSON_ASYNC_TILE(LT, QT, TIDT)                                                        \
  /* this wave's staged reads are done (the previous tile's stores may not be) */             \
  if (stores_pending) {                                                                        \
    if (layout == 0) vm_wait_keep<KEEP>();                                                   \
    else vm_wait_keep<KEEP_C>();                                                               \
  }                                                                                            \
  else __builtin_amdgcn_s_waitcnt(0);                                                          \
  lds_barrier();                 /* ... and every wave's */                                    \
  if constexpr (ivk)                                                                           \
    async_place_pre<T, C>(stage, S.tile, tw_a, kind, layout, LT, QT, TIDT);                  \
  else if constexpr (inverse)                                                                  \
    async_place_combine<T, C>(stage, S.tile, tw_a, tw_b, kind, layout, LT, QT, TIDT);        \
  else                                                                                         \
    async_place<T, C>(stage, S.tile, kind, inverse, layout, LT, QT, TIDT);                   \
  lds_barrier();                                                                               \
  if (tile + tr.step < tr.end)                                                                 \
    async_fetch<T, C>(stage_lds, A, layout, tile + tr.step, TIDT);                            \
  if constexpr (!(inverse && kind <= K_DD)) fast_passes<T, C, true, 0, true>(S.tile, tw_fft, LT, QT); \
  else fast_passes<T, C, false, 0, true>(S.tile, tw_fft, LT, QT);                             \
  const TileOrigin o = tile_origin(g, tile);                                                   \
  long long base;                                                                              \
  int lines = 0;                                                                               \
  if (layout == 0) {                                                                         \
    base = LT < (1 << g.lognl) ? line_base(g, o, LT) : -1;                                     \
  } else {                                                                                     \
    base = (long long)o.L0 * L::N;                                                             \
    lines = g.nlines - o.L0;                                                                   \
  }                                                                                            \
  if (sizeof(T) == 4 && A.out64) { /* widened last pass of an FP32 solve */                   \
    async_store_wide<T, C, ivk>(S.tile, tw_b, kind, inverse, A, layout, base, lines, LT, QT,   \
                                TIDT);                                                         \
    stores_pending = false;                                                                    \
  } else if constexpr (ivk) {                                                                  \
    post_store_body<T, C>(S.tile, tw_b, kind, as_global(A.data), base, g.sp, layout, lines, \
                           A.scale, LT, QT, TIDT);                                             \
    stores_pending = layout == 0 || lines >= NL;                                             \
  } else if constexpr (!inverse) {                                                             \
    split_store_body<T, C>(S.tile, tw_a, tw_b, kind, as_global(A.data), base, g.sp, layout,  \
                            lines, A.scale, LT, QT, TIDT);                                     \
    stores_pending = layout == 0 || lines >= NL;                                             \
  } else {                                                                                     \
    fast_store<T, C, true>(S.tile, as_global(A.data), base, g.sp, layout, lines, kind,       \
                           inverse, A.scale, LT, QT, TIDT);                                    \
    /* strided tiles: each wave holds line 0, which always exists, so it */                   \
    /* issues all its stores; contiguous tiles only when no line is missing */                \
    stores_pending = layout == 0 || lines >= NL;                                             \
  }                                                                                            \
  lds_barrier();

template <typename T, typename C, int KIND, int INV, int LAYOUT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(1, 2)))
void r2r_async_kernel(R2RFastArgs<T> A) {
  POISSON_ASYNC_SETUP
  for (int tile = tr.first; tile < tr.end; tile += tr.step) {
    POISSON_ASYNC_TILE(l, q, tid)
  }
}

template <typename T, typename C, int KIND, int INV, int LAYOUT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
void r2r_async_tight_kernel(R2RFastArgs<T> A) {
  POISSON_ASYNC_SETUP
  for (int tile = tr.first; tile < tr.end; tile += tr.step) {
    int lt = l, qt = q, tidt = tid;
    asm volatile("" : "+v"(lt), "+v"(qt), "+v"(tidt));
    POISSON_ASYNC_TILE(lt, qt, tidt)
  }
}

// ---------------------------------------------------------------- cache hints
// A global load or store with the nontemporal hint (NT) or a plain one.
template <bool NT, typename V, typename P>
__device__ __forceinline__ void st_hint(V v, P p) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}
template <bool NT, typename P>
__device__ __forceinline__ auto ld_hint(P p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

// ---------------------------------------------------------------- full-tile stores
// The forward real-DFT / DCT-II / DST-II split and the DCT-IV / DST-IV
// post-twiddle of split_store_body and post_store_body, for strided tiles
// whose lines all exist: every lane issues the same number of stores with
// no branch around them (a lane's outputs differ only by selects), so that
// the compiler's waits for loads issued before them can leave the stores in
// flight.  `out` is point 0 of the lane's line, `sp` the point stride.
//
// Split: lane qq takes wavenumbers k = qq + s*QT, s < M/(2 QT), each with
// its partner j = M - k, four outputs per k; the lane with k = 0 has two
// outputs there and takes the middle wavenumber M/2 (two outputs) in the
// same step.
template <typename T, typename C, int KIND>
__device__ __forceinline__ void split_store_full(lptr<const T> lds, lptr<const cplx<T>> split,
                                                 lptr<const cplx<T>> quarter, gptr<T> out,
                                                 long long sp, T scale, int ln, int qq) {
  using L = FastLayout<T, C>;
  constexpr int M = L::M, N = L::N, NLP = L::NLP, QT = L::QT, H = M / 2;
  static_assert(H % QT == 0, "wavenumbers split evenly over the lanes of a line");
  auto xy = [&](int k, cplx<T>& X, cplx<T>& Y) {
    const int kc = (M - k) % M;
    const cplx<T> z = {lds[(2 * k) * NLP + ln], lds[(2 * k + 1) * NLP + ln]};
    const cplx<T> zc = {lds[(2 * kc) * NLP + ln], -lds[(2 * kc + 1) * NLP + ln]};
    const cplx<T> E = {(T)0.5 * (z.re + zc.re), (T)0.5 * (z.im + zc.im)};
    const cplx<T> D = csub(z, zc);
    const cplx<T> O = {(T)0.5 * D.im, (T)-0.5 * D.re};
    const cplx<T> wO = cmul(ldc(split, k), O);
    X = cadd(E, wO);
    Y = cconj(csub(E, wO));
  };
  const bool zero = qq == 0;
#pragma unroll
  for (int s = 0; s < H / QT; ++s) {
    const int k = qq + s * QT, j = M - k;
    cplx<T> X, Y;
    xy(k, X, Y);
    int r[4];
    T v[4];
    if constexpr (KIND == K_P) {
      r[0] = 2 * k - 1; r[1] = 2 * k; r[2] = 2 * j - 1; r[3] = 2 * j;
      v[0] = X.re; v[1] = -X.im; v[2] = Y.re; v[3] = -Y.im;
      if (s == 0) {
        cplx<T> Xm, Ym;
        xy(H, Xm, Ym);
        r[0] = zero ? 0 : r[0];
        r[1] = zero ? N - 1 : r[1];
        r[2] = zero ? 2 * H - 1 : r[2];
        r[3] = zero ? 2 * H : r[3];
        v[1] = zero ? Y.re : v[1];
        v[2] = zero ? Xm.re : v[2];
        v[3] = zero ? -Xm.im : v[3];
      }
    } else {
      constexpr bool rev = KIND == K_DD;
      const cplx<T> u = cmul(ldc(quarter, k), X);
      const cplx<T> u2 = cmul(ldc(quarter, j), Y);
      r[0] = rev ? N - 1 - k : k; r[1] = rev ? k - 1 : N - k;
      r[2] = rev ? N - 1 - j : j; r[3] = rev ? j - 1 : N - j;
      v[0] = (T)2 * u.re; v[1] = (T)-2 * u.im; v[2] = (T)2 * u2.re; v[3] = (T)-2 * u2.im;
      if (s == 0) {
        cplx<T> Xm, Ym;
        xy(H, Xm, Ym);
        const cplx<T> um = cmul(ldc(quarter, H), Xm);
        r[1] = zero ? (rev ? N - 1 - M : M) : r[1];
        r[2] = zero ? (rev ? N - 1 - H : H) : r[2];
        r[3] = zero ? (rev ? H - 1 : N - H) : r[3];
        v[1] = zero ? v[2] : v[1];
        v[2] = zero ? (T)2 * um.re : v[2];
        v[3] = zero ? (T)-2 * um.im : v[3];
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) out[(long long)r[t] * sp] = v[t] * scale;
  }
}

// DCT-IV / DST-IV post-twiddle (post_store_body) for full strided tiles.
template <typename T, typename C, int KIND, bool NT>
__device__ __forceinline__ void post_store_full(lptr<const T> lds, lptr<const cplx<T>> post,
                                                gptr<T> out, long long sp, T scale, int ln,
                                                int qq) {
  using L = FastLayout<T, C>;
  constexpr int N = L::N, NLP = L::NLP, QT = L::QT;
#pragma unroll
  for (int s = 0; s < L::E; ++s) {
    const int k = qq + s * QT;
    const cplx<T> V = cmul(cplx<T>{lds[(2 * k) * NLP + ln], lds[(2 * k + 1) * NLP + ln]},
                           ldc(post, k));
    const T ye = ((T)2 * V.re) * scale;
    const T yo = ((T)-2 * V.im) * scale;
    st_hint<NT>(ye, &out[(long long)(2 * k) * sp]);
    st_hint<NT>(KIND == K_ND ? yo : -yo, &out[(long long)(N - 1 - 2 * k) * sp]);
  }
}

// ---------------------------------------------------------------- register-staged form
// FP64 length 512 on the strided axes with 32 lines per tile, so that each
// row of a tile is 256 contiguous bytes of the field (16 lines give
// 128-byte rows, which cost a strided sweep of a 512^3 field about a tenth
// of its bandwidth: measured 0.43 against 0.48 ms for an in-place read and
// write of every tile).  The tile (135 KiB) and the twiddles fill the LDS,
// so the next tile is read into registers while the current one is
// transformed and stored, and each input step runs from registers into the
// tile as the tile is placed: the forward real DFT / DCT-II / DST-II place
// the thread's rows at their permuted positions, the DCT-IV / DST-IV types
// read the two points of each complex index and apply the pre-twiddle, and
// the inverse real DFT / DCT-II / DST-II read the four rows of each of the
// thread's wavenumber pairs (k, M - k) and combine them.  Each thread reads
// two adjacent lines with 16-byte loads.
//
// HINTED: the forward DCT-IV / DST-IV and every inverse type read and
// write the field with the nontemporal hint (the launch asks for it on
// fields of 512 MiB and more).  Measured on the 512^3 cube: the forward
// DCT-IV along y, the inverse real DFT along z and the inverse DCT-IV along
// y ran 3-7 % faster, and the forward real DFT along z, which runs after
// the hinted forward y, 4 % faster (the solve 2.19 -> 2.11 ms; an RK3 step
// of the periodic 512^3 Taylor-Green vortex 18.65 -> 18.48 ms).  The forward
// real DFT / DCT-II / DST-II (its split stores scatter the rows) keeps plain
// accesses: with the hint it ran 15-25 % slower.  On fields that fit the
// 256 MB Infinity Cache the hint cost 2-5 % (64 x 512 x 512: 0.277 ->
// 0.284 ms, 128 x 512 x 512: 0.490 -> 0.517 ms); at 256 x 512 x 512 it
// was neutral.
template <typename T, typename C, int KIND, int INV, bool HINTED>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(1, 2)))
void r2r_regstage_kernel(R2RFastArgs<T> A) {
  using L = FastLayout<T, C>;
  constexpr int M = L::M, NL = L::NL, QT = L::QT, N = L::N, EPT = L::EPT, NLP = L::NLP;
  constexpr int kind = KIND, inverse = INV;
  constexpr bool ivk = kind >= K_ND;
  constexpr bool plain = !ivk;      // rows of the thread; IV types: pre-twiddle pairs
  constexpr bool nt = HINTED && (inverse || ivk);   // nontemporal loads and stores
  if (A.skip && A.skip[0] != 0.0) return;
  __shared__ __align__(16) unsigned char tile_raw[fast_lds_bytes<T, C>()];
  const FastLds<T, C> S = fast_lds<T, C>(tile_raw);
  const int tid = threadIdx.x;
  LineGeom g = A.g;
  g.layout = 0;
  const lptr<const cplx<T>> tw_fft = S.twf;
  const lptr<const cplx<T>> tw_a = S.twa;
  const lptr<const cplx<T>> tw_b = S.twa + (ivk ? M : L::SPLIT);
  fast_twiddles<T, C>(S, A, tid);
  const TileRange tr = xcd_tiles(g.ntiles);
  // The plain types read two adjacent lines per thread (16-byte loads): a
  // thread's EPT points then take EPT/2 load instructions, so that they and
  // the EPT stores of the tile before stay within the 63 operations the
  // vector-memory counter tracks (beyond it the compiler's waits drain the
  // stores along with the loads).  Thread t reads lines 2*(t mod NL/2) + {0,1}
  // at rows t / (NL/2) + i*QP.
  constexpr int NL2 = NL / 2, QP = L::NT / NL2, EPP = N / QP;
  static_assert(EPP * QP == N && 2 * EPP == EPT, "line-pair rows");
  using T2 = T __attribute__((ext_vector_type(2)));
  T2 buf[plain ? EPP : 1];
  // DCT-IV / DST-IV: the two points of each of the thread's EPP/2 complex
  // indices j = t / (NL/2) + s*QP, for both lines
  T2 pv[ivk ? EPP / 2 : 1][2];
  // a tile is 32 consecutive x positions of one band (nx >= 32 and even,
  // a 16-byte aligned field, checked at launch): a uniform base plus a
  // 32-bit lane offset (the launch checks that every offset fits), so no
  // load needs a 64-bit lane address
  const size_t pair_step = (size_t)QP * (size_t)g.sp;
  // Inverse real DFT / DCT-II / DST-II: the wavenumber pairs (k, M - k) of
  // a thread are k = qp + s*QP, s < M / (2 QP); their four input rows are
  // read into registers and combined there.  The lane with k = 0 has two
  // of its four rows unused and reads the two rows of the middle
  // wavenumber M/2 into them.
  static_assert(2 * QP * (EPP / 4) == M, "wavenumber pairs split evenly over the lanes");
  auto combine_rows = [](int k, bool zero, int (&r)[4]) {
    constexpr int H = M / 2;
    auto row = [](int x) { return kind == K_DD ? N - 1 - x : x; };
    const int j = M - k;
    if constexpr (kind == K_P) {
      r[0] = zero ? 0 : 2 * k - 1;
      r[1] = zero ? 2 * H - 1 : 2 * k;
      r[2] = zero ? N - 1 : 2 * j - 1;
      r[3] = zero ? 2 * H : 2 * j;
    } else {
      r[0] = row(k);
      r[1] = zero ? row(H) : row(N - k);
      r[2] = row(j);
      r[3] = zero ? row(N - H) : row(N - j);
    }
  };
  const unsigned sp32 = (unsigned)g.sp;
  auto fetch = [&](int tile, int lt, int qt, int tt) {
    const TileOrigin o = tile_origin(g, tile);
    const gptr<const T> tb = as_global(static_cast<const T*>(A.data)) + (o.x0 + (long long)o.b0 * g.sb);
    if constexpr (plain && inverse) {
      const int lp = tt % NL2, qp = tt / NL2;
      const bool ok = o.x0 + 2 * lp < g.nx;
#pragma unroll
      for (int s = 0; s < EPP / 4; ++s) {
        int r[4];
        combine_rows(qp + s * QP, s == 0 && qp == 0, r);
#pragma unroll
        for (int a = 0; a < 4; ++a)
          buf[4 * s + a] = ok ? ld_hint<nt>(reinterpret_cast<const gptr<const T2>>(
                                    &tb[2u * (unsigned)lp + (unsigned)r[a] * sp32]))
                              : T2{(T)0, (T)0};
      }
    } else if constexpr (plain) {
      const int lp = tt % NL2, qp = tt / NL2;
      const unsigned lane_off = 2u * (unsigned)lp + (unsigned)qp * sp32;
      if (o.x0 + 2 * lp < g.nx) {
#pragma unroll
        for (int i = 0; i < EPP; ++i)
          buf[i] = ld_hint<nt>(reinterpret_cast<const gptr<const T2>>(&(tb + i * pair_step)[lane_off]));
      } else {
#pragma unroll
        for (int i = 0; i < EPP; ++i) buf[i] = T2{(T)0, (T)0};
      }
    } else {
      const int lp = tt % NL2, qp = tt / NL2;
      const bool ok = o.x0 + 2 * lp < g.nx;
#pragma unroll
      for (int i = 0; i < EPP / 2; ++i) {
        const int j = qp + i * QP;
        const int r0 = kind == K_ND ? 2 * j : N - 1 - 2 * j;
        const int r1 = kind == K_ND ? N - 1 - 2 * j : 2 * j;
        if (ok) {
          pv[i][0] = ld_hint<nt>(reinterpret_cast<const gptr<const T2>>(
              &tb[2u * (unsigned)lp + (unsigned)r0 * sp32]));
          pv[i][1] = ld_hint<nt>(reinterpret_cast<const gptr<const T2>>(
              &tb[2u * (unsigned)lp + (unsigned)r1 * sp32]));
        } else {
          pv[i][0] = T2{(T)0, (T)0};
          pv[i][1] = T2{(T)0, (T)0};
        }
      }
    }
    (void)lt;
    (void)qt;
  };
  // registers -> tile: the DCT-IV / DST-IV pre-twiddle, or the rows (the
  // forward types at their permuted rows, the inverse ones unpermuted)
  auto place = [&](int l, int q, int tt) {
    if constexpr (ivk) {
      const int lp = tt % NL2, qp = tt / NL2;
#pragma unroll
      for (int i = 0; i < EPP / 2; ++i) {
        const int j = qp + i * QP;
        const cplx<T> w = ldc(tw_a, j);
        const cplx<T> z0 = cmul(cplx<T>{pv[i][0].x, pv[i][1].x}, w);
        const cplx<T> z1 = cmul(cplx<T>{pv[i][0].y, pv[i][1].y}, w);
        S.tile[(2 * j) * NLP + 2 * lp] = z0.re;
        S.tile[(2 * j + 1) * NLP + 2 * lp] = z0.im;
        S.tile[(2 * j) * NLP + 2 * lp + 1] = z1.re;
        S.tile[(2 * j + 1) * NLP + 2 * lp + 1] = z1.im;
      }
      (void)l;
      (void)q;
    } else if constexpr (inverse) {
      constexpr int H = M / 2;
      const int lp = tt % NL2, qp = tt / NL2;
      const bool zero = qp == 0;
      // x_k from the rows of wavenumber k (kinds as in combine_write)
      auto xform = [&](int k, T a, T b) -> cplx<T> {
        if constexpr (kind == K_P) return cplx<T>{a, -b};
        else return cmul(cconj(ldc(tw_b, k)), cplx<T>{(T)0.5 * a, (T)-0.5 * b});
      };
      // outputs 2k, 2k+1 of the pair (xk, xj) and 2j, 2j+1
      auto pair_out = [&](int k, cplx<T> xk, cplx<T> xj, T (&o)[4]) {
        const cplx<T> sk = ldc(tw_a, k);
        const cplx<T> s1 = cadd(xk, cconj(xj));
        const cplx<T> d1 = cmul(csub(xk, cconj(xj)), cconj(sk));
        const cplx<T> s2 = cadd(xj, cconj(xk));
        const cplx<T> d2 = cmul(csub(cconj(xk), xj), sk);
        o[0] = s1.re - d1.im;
        o[1] = s1.im + d1.re;
        o[2] = s2.re - d2.im;
        o[3] = s2.im + d2.re;
      };
#pragma unroll
      for (int s = 0; s < EPP / 4; ++s) {
        const int k = qp + s * QP, j = M - k;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const T v0 = h ? buf[4 * s].y : buf[4 * s].x, v1 = h ? buf[4 * s + 1].y : buf[4 * s + 1].x;
          const T v2 = h ? buf[4 * s + 2].y : buf[4 * s + 2].x, v3 = h ? buf[4 * s + 3].y : buf[4 * s + 3].x;
          T o[4];
          pair_out(k, xform(k, v0, v1), xform(j, v2, v3), o);
          int r[4] = {2 * k, 2 * k + 1, 2 * j, 2 * j + 1};
          if (s == 0) {
            // k = 0 (rows 0, 1) and the middle wavenumber (rows M, M + 1)
            cplx<T> x0, xM;
            if constexpr (kind == K_P) {
              x0 = {v0, (T)0};
              xM = {v2, (T)0};
            } else {
              x0 = xform(0, v0, (T)0);
              xM = xform(M, v2, v2);
            }
            T oz[4], om[4];
            pair_out(0, x0, xM, oz);
            const cplx<T> xh = xform(H, v1, v3);
            pair_out(H, xh, xh, om);
            o[0] = zero ? oz[0] : o[0];
            o[1] = zero ? oz[1] : o[1];
            o[2] = zero ? om[0] : o[2];
            o[3] = zero ? om[1] : o[3];
            r[2] = zero ? 2 * H : r[2];
            r[3] = zero ? 2 * H + 1 : r[3];
          }
#pragma unroll
          for (int a = 0; a < 4; ++a) S.tile[r[a] * NLP + 2 * lp + h] = o[a];
        }
      }
    } else {
      const int lp = tt % NL2, qp = tt / NL2;
#pragma unroll
      for (int i = 0; i < EPP; ++i) {
        bool neg = false;
        const int r = load_row(kind, inverse, qp + i * QP, N, neg);
        S.tile[r * NLP + 2 * lp] = neg ? -buf[i].x : buf[i].x;
        S.tile[r * NLP + 2 * lp + 1] = neg ? -buf[i].y : buf[i].y;
      }
    }
  };
  if (tr.first < tr.end) {
    fetch(tr.first, tid % NL, tid / NL, tid);
    place(tid % NL, tid / NL, tid);
  }
  // The next tile is placed at the bottom of the loop, after the current
  // tile's stores: its loads were issued before those stores in the same
  // iteration, so the waits for them leave the stores in flight (placed at
  // the top, the waits would be counted from the first tile's state, which
  // has no stores, and would drain every store of the previous tile).
  for (int tile = tr.first; tile < tr.end; tile += tr.step) {
    // thread indices opaque per tile: addresses are recomputed in each step
    // instead of being held across the loop
    int l = tid % NL, q = tid / NL, tt = tid;
    asm volatile("" : "+v"(l), "+v"(q), "+v"(tt));
    lds_barrier();
    const bool more = tile + tr.step < tr.end;
    if (more) fetch(tile + tr.step, l, q, tt);
    if constexpr (!(inverse && kind <= K_DD)) fast_passes<T, C, true, 0, true>(S.tile, tw_fft, l, q);
    else fast_passes<T, C, false, 0, true>(S.tile, tw_fft, l, q);
    const TileOrigin o = tile_origin(g, tile);
    const long long base = line_base(g, o, l);
    if constexpr (ivk)
      post_store_full<T, C, KIND, nt>(S.tile, tw_b, as_global(A.data) + base, g.sp, A.scale, l, q);
    else if constexpr (!inverse)
      split_store_full<T, C, KIND>(S.tile, tw_a, tw_b, as_global(A.data) + base, g.sp, A.scale, l, q);
    else {
      // every line of the tile exists (nx a multiple of 32): no branch
      // around the stores, so the waits for the next tile's loads count them
      const gptr<T> out = as_global(A.data) + base;
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        bool neg;
        const int r = store_row(kind, inverse, q + i * QT, N, neg);
        const T v = S.tile[r * NLP + l] * A.scale;
        st_hint<nt>(neg ? -v : v, &out[(long long)(q + i * QT) * g.sp]);
      }
    }
    lds_barrier();
    if (more) place(l, q, tt);
  }
}

// Tile shape of the register-staged form: two radix-16 passes over the
// tile instead of three (8, 8, 4), one LDS round trip and two barriers
// fewer per tile.
using RegStageCfg = FastCfg<256, 16, 32, 2>;

#undef POISSON_ASYNC_TILE
#undef POISSON_ASYNC_SETUP

}  // namespace poisson_dev
