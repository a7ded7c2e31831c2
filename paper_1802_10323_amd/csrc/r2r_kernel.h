// r2r_kernel.h - batched real-to-real transforms of Table 2 / Table 1 on gfx950.
//
// Every transform of length n (n even) is computed through one complex FFT
// of length m = n/2 held in LDS:
//
//  P  (DFT, Table 2 interleaved storage): z_j = a_2j + i a_2j+1, FFT, then the
//      even/odd split X_k = E_k + e^{-2 pi i k/n} O_k; inverse = the reverse.
//  NN (DCT-II / (1/2n) DCT-III): the even/odd reordering of Makhoul (1980)
//      turns the DCT-II into a real DFT of length n followed by the
//      post-twiddle e^{-i pi k/(2n)}.
//  DD (DST-II / (1/2n) DST-III): DST-II(a)_k = DCT-II((-1)^p a)_{n-1-k}.
//  ND (DCT-IV, self-inverse up to 2n): z_j = (a_2j + i a_{n-1-2j})
//      e^{-i pi (4j+1)/(4n)}, FFT, then V_k = Z_k e^{-i pi k/n} gives
//      y_2k = 2 Re V_k and y_{n-1-2k} = -2 Im V_k.
//  DN (DST-IV): DST-IV(a)_k = (-1)^k DCT-IV(reversed a)_k.
//  DDN (DST-I of n node values, the non-staggered Dirichlet pair): the real
//      DFT of length n' = 2(n+1) of the odd extension (0, a, 0, -a reversed)
//      holds 2 sum a_p sin(pi (p+1) q / (n+1)) in its sine slot 2q.
//  NNN (DCT-I of n node values, the non-staggered Neumann pair): the real
//      DFT of length n' = 2(n-1) of the even extension (a, a_{n-2} .. a_1)
//      is the DCT-I: cosine slots 2q-1, slot 0 and slot n'-1.
//      Both are their own inverses up to n', so the backward transform runs
//      the same steps with the scale 1/n'.
//
// A kernel launch processes tiles of lines (see device_common.h).  Per tile:
//   1. load: global -> LDS with the input permutation and sign of the type;
//   2. pre-step: DCT-IV pre-twiddle, or (inverse P/NN/DD) the recombination
//      of the real spectrum into the length-m complex spectrum;
//   3. Stockham radix-R passes (R in {2,3,4,5,8}), in place in LDS: every
//      thread stages its butterflies in registers between two barriers;
//   4. post-step: even/odd split (forward P/NN/DD) or DCT-IV post-twiddle;
//   5. store: LDS -> global with the output permutation, sign and scale.
// Complex element j of line l occupies LDS rows 2j (real) and 2j+1 (imag).
#pragma once
#include "device_common.h"

namespace poisson_dev {

enum Kind { K_P = 0, K_NN = 1, K_DD = 2, K_ND = 3, K_DN = 4, K_DDN = 5, K_NNN = 6 };

template <typename T>
struct R2RArgs {
  T* data;
  LineGeom g;
  int kind;
  int inverse;
  int m;                     // complex FFT length: n / 2 (node pairs: (n + 1) or (n - 1))
  int npass;
  int radix[16];
  unsigned ns_magic[16];     // ceil(2^32 / Ns) of each pass (Ns = product of earlier radices)
  unsigned n_magic;          // ceil(2^32 / n)
  int nlp;                   // LDS row pitch (elements)
  T scale;                   // applied at the store (1, 1/n or 1/2n)
  const cplx<T>* tw_fft;     // m     : e^{-2 pi i t/m}
  const cplx<T>* tw_split;   // m + 1 : e^{-2 pi i k/n}
  const cplx<T>* tw_quarter; // m + 1 : e^{-i pi k/(2n)}
  const cplx<T>* tw_pre;     // m     : e^{-i pi (4j+1)/(4n)}
  const cplx<T>* tw_post;    // m     : e^{-i pi k/n}
  const double* skip;        // optional: when *skip != 0 the launch does nothing
  double* out64;             // optional (FP32): write the widened result there, not in data
};

// ---------------------------------------------------------------- small DFTs
// y_q = sum_r v_r e^{-+2 pi i r q / R}; FWD selects the minus sign.

template <int R, typename T, bool FWD>
struct SmallDFT;

template <typename T, bool FWD>
struct SmallDFT<2, T, FWD> {
  static __device__ __forceinline__ void run(cplx<T>* v) {
    const cplx<T> a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
  }
};

template <typename T, bool FWD>
struct SmallDFT<4, T, FWD> {
  static __device__ __forceinline__ void run(cplx<T>* v) {
    const cplx<T> a = cadd(v[0], v[2]);
    const cplx<T> b = csub(v[0], v[2]);
    const cplx<T> c = cadd(v[1], v[3]);
    const cplx<T> d = mul_mi<T, FWD>(csub(v[1], v[3]));
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, d);
    v[3] = csub(b, d);
  }
};

template <typename T, bool FWD>
struct SmallDFT<8, T, FWD> {
  static __device__ __forceinline__ void run(cplx<T>* v) {
    cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
    SmallDFT<4, T, FWD>::run(e);
    SmallDFT<4, T, FWD>::run(o);
    const T h = (T)0.70710678118654752440;   // 1/sqrt(2)
    // o1 *= e^{-+i pi/4}, o2 *= -+i, o3 *= e^{-+3 i pi/4}
    const cplx<T> o1 = FWD ? cplx<T>{(o[1].re + o[1].im) * h, (o[1].im - o[1].re) * h}
                           : cplx<T>{(o[1].re - o[1].im) * h, (o[1].im + o[1].re) * h};
    const cplx<T> o2 = mul_mi<T, FWD>(o[2]);
    const cplx<T> o3 = FWD ? cplx<T>{(o[3].im - o[3].re) * h, -(o[3].re + o[3].im) * h}
                           : cplx<T>{-(o[3].re + o[3].im) * h, (o[3].re - o[3].im) * h};
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

template <typename T, bool FWD>
struct SmallDFT<3, T, FWD> {
  static __device__ __forceinline__ void run(cplx<T>* v) {
    const T s3 = (T)0.86602540378443864676;  // sin(2 pi/3)
    const cplx<T> t = cadd(v[1], v[2]);
    const cplx<T> d = csub(v[1], v[2]);
    const cplx<T> base = {v[0].re - (T)0.5 * t.re, v[0].im - (T)0.5 * t.im};
    // -+ i s3 d
    const cplx<T> rot = mul_mi<T, FWD>(cplx<T>{s3 * d.re, s3 * d.im});
    v[0] = cadd(v[0], t);
    v[1] = cadd(base, rot);
    v[2] = csub(base, rot);
  }
};

template <typename T, bool FWD>
struct SmallDFT<5, T, FWD> {
  static __device__ __forceinline__ void run(cplx<T>* v) {
    const T c1 = (T)0.30901699437494742410, s1 = (T)0.95105651629515357212;   // 2 pi/5
    const T c2 = (T)-0.80901699437494742410, s2 = (T)0.58778525229247312917;  // 4 pi/5
    const cplx<T> p1 = cadd(v[1], v[4]), m1 = csub(v[1], v[4]);
    const cplx<T> p2 = cadd(v[2], v[3]), m2 = csub(v[2], v[3]);
    const cplx<T> a1 = {v[0].re + c1 * p1.re + c2 * p2.re, v[0].im + c1 * p1.im + c2 * p2.im};
    const cplx<T> a2 = {v[0].re + c2 * p1.re + c1 * p2.re, v[0].im + c2 * p1.im + c1 * p2.im};
    const cplx<T> b1 = mul_mi<T, FWD>(cplx<T>{s1 * m1.re + s2 * m2.re, s1 * m1.im + s2 * m2.im});
    const cplx<T> b2 = mul_mi<T, FWD>(cplx<T>{s2 * m1.re - s1 * m2.re, s2 * m1.im - s1 * m2.im});
    v[0] = cadd(v[0], cadd(p1, p2));
    v[1] = cadd(a1, b1);
    v[4] = csub(a1, b1);
    v[2] = cadd(a2, b2);
    v[3] = csub(a2, b2);
  }
};

// Length 16 as 4 x 4: inputs n = 4 n1 + n2, outputs k = k1 + 4 k2; length-4
// DFTs over n1, the twiddles W16^(n2 k1), length-4 DFTs over n2.
template <typename T, bool FWD>
struct SmallDFT<16, T, FWD> {
  // v * W16^m (W16 = exp(-+ 2 pi i / 16)) for the products m = n2 k1 that occur
  template <int M_>
  static __device__ __forceinline__ cplx<T> tw16(cplx<T> v) {
    const T c1 = (T)0.92387953251128675613;   // cos(pi/8)
    const T s1 = (T)0.38268343236508977173;   // sin(pi/8)
    const T h = (T)0.70710678118654752440;    // cos(pi/4)
    T wr = 1, wi = 0;                         // cos, sin of 2 pi m / 16
    if constexpr (M_ == 0) return v;
    if constexpr (M_ == 4) return mul_mi<T, FWD>(v);
    if constexpr (M_ == 1) { wr = c1; wi = s1; }
    if constexpr (M_ == 2) { wr = h; wi = h; }
    if constexpr (M_ == 3) { wr = s1; wi = c1; }
    if constexpr (M_ == 6) { wr = -h; wi = h; }
    if constexpr (M_ == 9) { wr = -c1; wi = -s1; }
    if (FWD) wi = -wi;
    return cplx<T>{v.re * wr - v.im * wi, v.re * wi + v.im * wr};
  }
  template <int N2>
  static __device__ __forceinline__ void column(cplx<T>* v, cplx<T> (&y)[4][4]) {
    cplx<T> c[4] = {v[N2], v[4 + N2], v[8 + N2], v[12 + N2]};
    SmallDFT<4, T, FWD>::run(c);
    y[N2][0] = c[0];
    y[N2][1] = tw16<N2 * 1>(c[1]);
    y[N2][2] = tw16<N2 * 2>(c[2]);
    y[N2][3] = tw16<N2 * 3>(c[3]);
  }
  static __device__ __forceinline__ void run(cplx<T>* v) {
    cplx<T> y[4][4];
    column<0>(v, y);
    column<1>(v, y);
    column<2>(v, y);
    column<3>(v, y);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cplx<T> c[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
      SmallDFT<4, T, FWD>::run(c);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = c[k2];
    }
  }
};

// ---------------------------------------------------------------- LDS access

template <typename T>
__device__ __forceinline__ cplx<T> ld_c(const T* lds, int nlp, int l, int j) {
  return {lds[(2 * j) * nlp + l], lds[(2 * j + 1) * nlp + l]};
}
template <typename T>
__device__ __forceinline__ void st_c(T* lds, int nlp, int l, int j, cplx<T> v) {
  lds[(2 * j) * nlp + l] = v.re;
  lds[(2 * j + 1) * nlp + l] = v.im;
}

// ---------------------------------------------------------------- FFT pass
// One Stockham pass of radix R over all lines of the tile: butterfly j of a
// line reads elements j + r m/R, twiddles them by W_m^{r k (m/(Ns R))} with
// k = j mod Ns, and writes (j - k) R + k + r Ns.  Not inlined: each radix
// then gets its own register allocation instead of the union of all of them.

template <int R, typename T, bool FWD, int EMAX, int NT>
__device__ __noinline__ void fft_pass(T* lds, int m, int Ns, unsigned ns_magic, int lognl, int nlp,
                                      const cplx<T>* __restrict__ tw, int tid) {
  constexpr int S = (EMAX + R - 1) / R;
  const int nbf = m / R;
  const int total = nbf << lognl;
  const int tstride = m / (Ns * R);
  cplx<T> v[S][R];
  int lsave[S], jout[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int b = tid + s * NT;
    lsave[s] = -1;
    jout[s] = 0;
    if (b < total) {
      const int l = b & ((1 << lognl) - 1);
      const int j = b >> lognl;
      const int k = Ns > 1 ? j - Ns * fast_div(j, ns_magic) : 0;
#pragma unroll
      for (int r = 0; r < R; ++r) v[s][r] = ld_c(lds, nlp, l, j + r * nbf);
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cplx<T> w = ldg(tw, r * k * tstride);
          if (!FWD) w.im = -w.im;
          v[s][r] = cmul(v[s][r], w);
        }
      }
      lsave[s] = l;
      jout[s] = (j - k) * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < S; ++s) {
    if (lsave[s] >= 0) {
      SmallDFT<R, T, FWD>::run(v[s]);
#pragma unroll
      for (int r = 0; r < R; ++r) st_c(lds, nlp, lsave[s], jout[s] + r * Ns, v[s][r]);
    }
  }
  __syncthreads();
}

template <typename T, bool FWD, int EMAX, int NT>
__device__ void fft_all(T* lds, const R2RArgs<T>& A, int lognl, int nlp, int tid) {
  int Ns = 1;
  for (int ip = 0; ip < A.npass; ++ip) {
    const int R = A.radix[ip];
    const unsigned mg = A.ns_magic[ip];
    switch (R) {
      case 8: fft_pass<8, T, FWD, EMAX, NT>(lds, A.m, Ns, mg, lognl, nlp, A.tw_fft, tid); break;
      case 4: fft_pass<4, T, FWD, EMAX, NT>(lds, A.m, Ns, mg, lognl, nlp, A.tw_fft, tid); break;
      case 2: fft_pass<2, T, FWD, EMAX, NT>(lds, A.m, Ns, mg, lognl, nlp, A.tw_fft, tid); break;
      case 3: fft_pass<3, T, FWD, EMAX, NT>(lds, A.m, Ns, mg, lognl, nlp, A.tw_fft, tid); break;
      default: fft_pass<5, T, FWD, EMAX, NT>(lds, A.m, Ns, mg, lognl, nlp, A.tw_fft, tid); break;
    }
    Ns *= R;
  }
}

// ---------------------------------------------------------------- permutations

// Makhoul order: v_j = a_2j, v_{n-1-j} = a_2j+1.  Row of a_p in that order.
__device__ __forceinline__ int makhoul_row(int p, int n) {
  return (p & 1) ? n - 1 - (p >> 1) : (p >> 1);
}
// DCT-IV packing: a_p (p even) -> Re z_{p/2}; a_p (p odd) -> Im z_{(n-1-p)/2}.
__device__ __forceinline__ int iv_row(int p, int n) { return (p & 1) ? n - p : p; }

// LDS row that receives input point p, and whether it is negated.
__device__ __forceinline__ int load_row(int kind, int inverse, int p, int n, bool& neg) {
  neg = false;
  switch (kind) {
    case K_P: return p;
    case K_NN: return inverse ? p : makhoul_row(p, n);
    case K_DD:
      if (inverse) return n - 1 - p;
      neg = p & 1;
      return makhoul_row(p, n);
    case K_ND: return iv_row(p, n);
    default: return iv_row(n - 1 - p, n);
  }
}

// LDS row that holds output point q, and whether it is negated.
__device__ __forceinline__ int store_row(int kind, int inverse, int q, int n, bool& neg) {
  neg = false;
  switch (kind) {
    case K_P: return q;
    case K_NN: return inverse ? makhoul_row(q, n) : q;
    case K_DD:
      if (!inverse) return q;
      neg = q & 1;
      return makhoul_row(q, n);
    case K_ND: return q;
    default:
      neg = q & 1;
      return q;
  }
}

// ---------------------------------------------------------------- pre / post

// Forward P/NN/DD: from Z (FFT of z_j = v_2j + i v_2j+1) to the real DFT
// X_k of v, k = 0..m, and then to the stored coefficients.  Pairs (k, m-k)
// are handled together: with E = (Z_k + conj Z_{m-k})/2,
// O = -i (Z_k - conj Z_{m-k})/2, w = e^{-2 pi i k/n}:
// X_k = E + w O and X_{m-k} = conj(E - w O).
template <typename T, int EMAX, int NT>
__device__ __noinline__ void split_forward(T* lds, int kind, int n, int m, int lognl, int nlp,
                                           const cplx<T>* __restrict__ tw_split,
                                           const cplx<T>* __restrict__ tw_quarter, int tid) {
  constexpr int S = EMAX / 2 + 1;
  const int total = (m / 2 + 1) << lognl;
  cplx<T> X[S], Y[S];
  int ks[S], ls[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int b = tid + s * NT;
    ls[s] = -1;
    ks[s] = 0;
    if (b < total) {
      const int l = b & ((1 << lognl) - 1);
      const int k = b >> lognl;
      const cplx<T> zk = ld_c(lds, nlp, l, k);
      const cplx<T> zc = cconj(ld_c(lds, nlp, l, (m - k) % m));
      const cplx<T> E = {(T)0.5 * (zk.re + zc.re), (T)0.5 * (zk.im + zc.im)};
      const cplx<T> D = csub(zk, zc);
      const cplx<T> O = {(T)0.5 * D.im, (T)-0.5 * D.re};
      const cplx<T> wO = cmul(ldg(tw_split, k), O);
      X[s] = cadd(E, wO);
      Y[s] = cconj(csub(E, wO));
      ls[s] = l;
      ks[s] = k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < S; ++s) {
    if (ls[s] < 0) continue;
    const int l = ls[s], k = ks[s], j = m - k;   // j == m when k == 0
    if (kind == K_P) {
      if (k == 0) {
        lds[l] = X[s].re;
        lds[(n - 1) * nlp + l] = Y[s].re;
      } else {
        lds[(2 * k - 1) * nlp + l] = X[s].re;
        lds[(2 * k) * nlp + l] = -X[s].im;
        if (j != k) {
          lds[(2 * j - 1) * nlp + l] = Y[s].re;
          lds[(2 * j) * nlp + l] = -Y[s].im;
        }
      }
    } else {
      // DCT-II outputs y_r = 2 Re(q_r X_r), y_{n-r} = -2 Im(q_r X_r);
      // the DST-II stores y_r at n-1-r.
      const bool rev = kind == K_DD;
      const cplx<T> u = cmul(ldg(tw_quarter, k), X[s]);
      lds[(rev ? n - 1 - k : k) * nlp + l] = (T)2 * u.re;
      if (k > 0) lds[(rev ? k - 1 : n - k) * nlp + l] = (T)-2 * u.im;
      if (j != k) {
        const cplx<T> u2 = cmul(ldg(tw_quarter, j), Y[s]);
        lds[(rev ? n - 1 - j : j) * nlp + l] = (T)2 * u2.re;
        if (j != m) lds[(rev ? j - 1 : n - j) * nlp + l] = (T)-2 * u2.im;
      }
    }
  }
  __syncthreads();
}

// Inverse P/NN/DD: rebuild the length-m complex spectrum
// Z'_k = (X_k + conj X_{m-k}) + i (X_k - conj X_{m-k}) e^{2 pi i k/n}
// whose unnormalised inverse FFT is n times (a_2j + i a_2j+1) (P) or the
// Makhoul-ordered sequence (NN, DD).  X comes from the stored coefficients:
// P: X_k = A_{2k-1} - i A_{2k}, X_0 = A_0, X_m = A_{n-1};
// NN/DD: X_k = (1/2) e^{i pi k/(2n)} (y_k - i y_{n-k}) with y_n = 0.
template <typename T>
__device__ __forceinline__ cplx<T> spectrum_at(const T* lds, int nlp, int l, int k, int kind,
                                               int n, int m, const cplx<T>* quarter) {
  if (kind == K_P) {
    if (k == 0) return {lds[l], (T)0};
    if (k == m) return {lds[(n - 1) * nlp + l], (T)0};
    return {lds[(2 * k - 1) * nlp + l], -lds[(2 * k) * nlp + l]};
  }
  const T yk = lds[k * nlp + l];
  const T ynk = k == 0 ? (T)0 : lds[(n - k) * nlp + l];
  const cplx<T> q = cconj(ldg(quarter, k));
  return cmul(q, cplx<T>{(T)0.5 * yk, (T)-0.5 * ynk});
}

template <typename T, int EMAX, int NT>
__device__ __noinline__ void combine_inverse(T* lds, int kind, int n, int m, int lognl, int nlp,
                                             const cplx<T>* __restrict__ tw_split,
                                             const cplx<T>* __restrict__ tw_quarter, int tid) {
  constexpr int S = EMAX / 2 + 1;
  const int total = (m / 2 + 1) << lognl;
  cplx<T> Zk[S], Zj[S];
  int ks[S], ls[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int b = tid + s * NT;
    ls[s] = -1;
    ks[s] = 0;
    if (b < total) {
      const int l = b & ((1 << lognl) - 1);
      const int k = b >> lognl;
      const int j = m - k;
      const cplx<T> Xk = spectrum_at(lds, nlp, l, k, kind, n, m, tw_quarter);
      const cplx<T> Xj = spectrum_at(lds, nlp, l, j, kind, n, m, tw_quarter);
      {
        const cplx<T> s1 = cadd(Xk, cconj(Xj));
        const cplx<T> d1 = cmul(csub(Xk, cconj(Xj)), cconj(ldg(tw_split, k)));
        Zk[s] = {s1.re - d1.im, s1.im + d1.re};     // s1 + i d1
      }
      {
        const cplx<T> s2 = cadd(Xj, cconj(Xk));
        const cplx<T> d2 = cmul(csub(Xj, cconj(Xk)), cconj(ldg(tw_split, j)));
        Zj[s] = {s2.re - d2.im, s2.im + d2.re};
      }
      ls[s] = l;
      ks[s] = k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < S; ++s) {
    if (ls[s] < 0) continue;
    const int k = ks[s], j = m - k;
    st_c(lds, nlp, ls[s], k, Zk[s]);
    if (k > 0 && j != k) st_c(lds, nlp, ls[s], j, Zj[s]);
  }
  __syncthreads();
}

// DCT-IV pre-twiddle, in place (each element is read and written by the
// same thread).
template <typename T, int NT>
__device__ __noinline__ void iv_pre(T* lds, int m, int lognl, int nlp,
                                    const cplx<T>* __restrict__ tw_pre, int tid) {
  const int total = m << lognl;
  for (int b = tid; b < total; b += NT) {
    const int l = b & ((1 << lognl) - 1);
    const int j = b >> lognl;
    st_c(lds, nlp, l, j, cmul(ld_c(lds, nlp, l, j), ldg(tw_pre, j)));
  }
  __syncthreads();
}

// DCT-IV post-step: V_k = Z_k e^{-i pi k/n}; y_2k = 2 Re V_k, y_{n-1-2k} = -2 Im V_k.
template <typename T, int EMAX, int NT>
__device__ __noinline__ void iv_post(T* lds, int n, int m, int lognl, int nlp,
                                     const cplx<T>* __restrict__ tw_post, int tid) {
  constexpr int S = EMAX;
  const int total = m << lognl;
  cplx<T> V[S];
  int ks[S], ls[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int b = tid + s * NT;
    ls[s] = -1;
    ks[s] = 0;
    if (b < total) {
      const int l = b & ((1 << lognl) - 1);
      const int k = b >> lognl;
      V[s] = cmul(ld_c(lds, nlp, l, k), ldg(tw_post, k));
      ls[s] = l;
      ks[s] = k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < S; ++s) {
    if (ls[s] < 0) continue;
    lds[(2 * ks[s]) * nlp + ls[s]] = (T)2 * V[s].re;
    lds[(n - 1 - 2 * ks[s]) * nlp + ls[s]] = (T)-2 * V[s].im;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- tile load / store
// All EPT global loads of a thread are issued before the first LDS write
// (and all LDS reads before the first global store), so a wavefront keeps
// EPT memory requests in flight.  Not inlined, so that nothing of this
// phase stays live across the FFT passes.

template <typename T, int EPT, int NT>
__device__ __noinline__ void r2r_load_tile(T* lds, const T* __restrict__ data, GEOM_PARAMS,
                                           int tile, int kind, int inverse, int nlp,
                                           unsigned n_magic, int tid) {
  const LineGeom g = GEOM_REBUILD;
  const TileOrigin o = tile_origin(g, tile);
  const long long sbase = g.layout == 0 ? line_base(g, o, tid & ((1 << g.lognl) - 1)) : 0;
  T buf[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    int l, p;
    const long long off = tile_elem<NT>(g, o, sbase, n_magic, tid, i, l, p);
    buf[i] = off >= 0 ? as_global(data)[off] : (T)0;
  }
  if (kind >= K_DDN) {   // odd / even extension of the node values (n' = 2m rows)
    const int m = kind == K_DDN ? g.n + 1 : g.n - 1;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      int l, p;
      tile_elem<NT>(g, o, sbase, n_magic, tid, i, l, p);
      if (p < g.n && l < (1 << g.lognl)) {
        if (kind == K_DDN) {
          lds[(p + 1) * nlp + l] = buf[i];
          lds[(2 * m - 1 - p) * nlp + l] = -buf[i];
        } else {
          lds[p * nlp + l] = buf[i];
          if (p > 0 && p < m) lds[(2 * m - p) * nlp + l] = buf[i];
        }
      }
    }
    if (kind == K_DDN)
      for (int l = tid; l < (1 << g.lognl); l += NT) {
        lds[l] = (T)0;
        lds[m * nlp + l] = (T)0;
      }
    return;
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    int l, p;
    tile_elem<NT>(g, o, sbase, n_magic, tid, i, l, p);
    if (p < g.n && l < (1 << g.lognl)) {
      bool neg;
      const int r = load_row(kind, inverse, p, g.n, neg);
      lds[r * nlp + l] = neg ? -buf[i] : buf[i];
    }
  }
}

// O: the element type written (T, or double for the widened last pass of
// an FP32 solve).
template <typename T, int EPT, int NT, typename O = T>
__device__ __noinline__ void r2r_store_tile(const T* lds, O* __restrict__ data, GEOM_PARAMS,
                                            int tile, int kind, int inverse, int nlp,
                                            unsigned n_magic, T scale, int tid) {
  const LineGeom g = GEOM_REBUILD;
  const TileOrigin o = tile_origin(g, tile);
  const long long sbase = g.layout == 0 ? line_base(g, o, tid & ((1 << g.lognl) - 1)) : 0;
  T buf[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    int l, q;
    tile_elem<NT>(g, o, sbase, n_magic, tid, i, l, q);
    buf[i] = (T)0;
    if (q < g.n && l < (1 << g.lognl)) {
      bool neg = false;
      int r;
      if (kind == K_DDN) r = 2 * (q + 1);                       // sine slot of wavenumber q+1
      else if (kind == K_NNN) r = q == 0 ? 0 : (q == g.n - 1 ? 2 * (g.n - 1) - 1 : 2 * q - 1);
      else r = store_row(kind, inverse, q, g.n, neg);
      const T v = lds[r * nlp + l] * scale;
      buf[i] = neg ? -v : v;
    }
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    int l, q;
    const long long off = tile_elem<NT>(g, o, sbase, n_magic, tid, i, l, q);
    if (off >= 0) as_global(data)[off] = (O)buf[i];
  }
}

// ---------------------------------------------------------------- kernel

template <typename T, int EMAX, int NT>
// at least 4 waves per SIMD: two 512-thread tiles resident per CU
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
void r2r_kernel(R2RArgs<T> A) {
  if (A.skip && A.skip[0] != 0.0) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int tid = threadIdx.x;
  const LineGeom& g = A.g;
  const int lognl = g.lognl, nlp = A.nlp;
  const int kind = A.kind, inverse = A.inverse;
  const bool node = kind >= K_DDN;     // node pairs: the forward real DFT in both directions
  const int n = node ? 2 * A.m : g.n;  // rows of the tile
  T* __restrict__ data = A.data;
  const bool fwd_fft = !(inverse && kind <= K_DD);

  const TileRange tr = xcd_tiles(g.ntiles);
  for (int tile = tr.first; tile < tr.end; tile += tr.step) {
    r2r_load_tile<T, 2 * EMAX, NT>(lds, data, GEOM_ARGS(g), tile, kind, inverse, nlp, A.n_magic, tid);
    __syncthreads();

    if (kind == K_ND || kind == K_DN) iv_pre<T, NT>(lds, A.m, lognl, nlp, A.tw_pre, tid);
    else if (inverse && !node)
      combine_inverse<T, EMAX, NT>(lds, kind, n, A.m, lognl, nlp, A.tw_split, A.tw_quarter, tid);

    if (fwd_fft) fft_all<T, true, EMAX, NT>(lds, A, lognl, nlp, tid);
    else fft_all<T, false, EMAX, NT>(lds, A, lognl, nlp, tid);

    if (kind == K_ND || kind == K_DN) iv_post<T, EMAX, NT>(lds, n, A.m, lognl, nlp, A.tw_post, tid);
    else if (!inverse || node)
      split_forward<T, EMAX, NT>(lds, node ? (int)K_P : kind, n, A.m, lognl, nlp, A.tw_split,
                                 A.tw_quarter, tid);

    bool widened = false;
    if constexpr (sizeof(T) == 4) {
      if (A.out64) {   // last pass of an FP32 solve: the widened result into out64
        widened = true;
        r2r_store_tile<T, 2 * EMAX, NT, double>(lds, A.out64, GEOM_ARGS(g), tile, kind, inverse,
                                                nlp, A.n_magic, A.scale, tid);
      }
    }
    if (!widened)
      r2r_store_tile<T, 2 * EMAX, NT>(lds, data, GEOM_ARGS(g), tile, kind, inverse, nlp,
                                      A.n_magic, A.scale, tid);
    __syncthreads();
  }
}

}  // namespace poisson_dev
