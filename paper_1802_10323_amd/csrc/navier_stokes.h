// navier_stokes.h - the prediction of one Runge-Kutta substep (Sec. 2,
// Eq. (up)) on a tri-periodic uniform staggered grid:
//
//   AD  = -div(u u) + nu lap(u)            at every face
//   u*  = u + dt (alpha_k AD + beta_k AD_prev - gamma_k grad p)
//
// Layout: every field nx*ny*nz doubles, x fastest.  Velocity component c
// at index (i, j, k) lives on the low face of cell (i, j, k) normal to
// axis c (u at (i dx, (j + 1/2) dy, (k + 1/2) dz)); p at the cell centre.
// The three components sit one after another in one buffer (u, v, w).
//
// Advection in divergence form with second-order central differences:
// the square of a component at cell centres from the mean of its two
// faces, the cross products on cell edges from the means of the two
// nearest values of each factor; a face's derivative is the difference of
// the products on its two sides over the spacing.  Diffusion is the
// three-point second difference per axis.
//
// Three kernels compute it, each thread the three faces its cell owns:
// rk3_predict_kernel (one cell per thread, neighbours through the
// caches), rk3_predict_tiled_kernel (z-marching LDS plane tiles) and
// rk3_predict_div_kernel (the tiled form with the right-hand side of the
// pressure equation, and optionally the previous substep's projection,
// fused in; the default).  Traffic per cell: velocity 24 B, p 8 B,
// AD_prev 24 B (read when beta_k != 0), AD 24 B (written when the next
// substep needs it), u* 24 B.
#pragma once
#include <type_traits>
#include "refine_kernels.h"

namespace poisson_dev {

struct RK3Args {
  const double* vel;       // u, v, w (3 npts); with CORRECT: u* of the previous substep
  const double* p;         // npts
  const double* ad_prev;   // 3 npts, read when READ_PREV
  double* ad;              // 3 npts, written when WRITE_AD
  double* star;            // 3 npts: the prediction u*
  const double* phi_prev;  // CORRECT: Phi of the previous substep (npts)
  double* p_out;           // CORRECT: p + Phi of the previous substep (npts)
  double c_gdt;            // CORRECT: gamma dt of the previous substep
  double idx, idy, idz;    // 1 / spacing
  double kx, ky, kz;       // nu / spacing^2
  double a_dt, b_dt, g_dt; // dt alpha_k, dt beta_k, dt gamma_k
  int nx, ny, nz;
  long long npts;
};

static constexpr int RK3_NT = 256;
static constexpr int RK3_BLOCKS = 8192;

template <bool READ_PREV, bool WRITE_AD>
__global__ __launch_bounds__(RK3_NT) void rk3_predict_kernel(RK3Args A) {
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const long long N = A.npts;
  const long long plane = (long long)nx * ny;
  const double* __restrict__ U = A.vel;
  const double* __restrict__ V = A.vel + N;
  const double* __restrict__ W = A.vel + 2 * N;
  const double* __restrict__ P = A.p;
  const long long step = (long long)gridDim.x * RK3_NT;
  const long long first = blockIdx.x * (long long)RK3_NT + threadIdx.x;
  GridWalk at(first, step, nx, ny);
  for (long long c = first; c < N; c += step, at.advance()) {
    const int i = at.i, j = at.j, k = at.k;
    // periodic neighbour offsets
    const long long xm = i > 0 ? -1 : nx - 1, xp = i + 1 < nx ? 1 : -(long long)(nx - 1);
    const long long ym = j > 0 ? -(long long)nx : (long long)nx * (ny - 1);
    const long long yp = j + 1 < ny ? (long long)nx : -(long long)nx * (ny - 1);
    const long long zm = k > 0 ? -plane : plane * (nz - 1);
    const long long zp = k + 1 < nz ? plane : -plane * (nz - 1);

    const double u0 = U[c], uxm = U[c + xm], uxp = U[c + xp], uym = U[c + ym], uyp = U[c + yp],
                 uzm = U[c + zm], uzp = U[c + zp], uxpym = U[c + xp + ym], uxpzm = U[c + xp + zm];
    const double v0 = V[c], vxm = V[c + xm], vxp = V[c + xp], vym = V[c + ym], vyp = V[c + yp],
                 vzm = V[c + zm], vzp = V[c + zp], vxmyp = V[c + xm + yp], vypzm = V[c + yp + zm];
    const double w0 = W[c], wxm = W[c + xm], wxp = W[c + xp], wym = W[c + ym], wyp = W[c + yp],
                 wzm = W[c + zm], wzp = W[c + zp], wxmzp = W[c + xm + zp], wymzp = W[c + ym + zp];
    const double p0 = P[c], pxm = P[c + xm], pym = P[c + ym], pzm = P[c + zm];

    // products: squares at the centres of this cell and the one below;
    // cross products on the edges at this cell's low corner and beyond
    const double uu0 = 0.25 * (u0 + uxp) * (u0 + uxp), uum = 0.25 * (uxm + u0) * (uxm + u0);
    const double vv0 = 0.25 * (v0 + vyp) * (v0 + vyp), vvm = 0.25 * (vym + v0) * (vym + v0);
    const double ww0 = 0.25 * (w0 + wzp) * (w0 + wzp), wwm = 0.25 * (wzm + w0) * (wzm + w0);
    // uv on the x-y edge (i, j): u over j-1, j; v over i-1, i
    const double uv00 = 0.25 * (uym + u0) * (vxm + v0);
    const double uv01 = 0.25 * (u0 + uyp) * (vxmyp + vyp);      // edge (i, j+1)
    const double uv10 = 0.25 * (uxpym + uxp) * (v0 + vxp);      // edge (i+1, j)
    // uw on the x-z edge (i, k)
    const double uw00 = 0.25 * (uzm + u0) * (wxm + w0);
    const double uw01 = 0.25 * (u0 + uzp) * (wxmzp + wzp);      // edge (i, k+1)
    const double uw10 = 0.25 * (uxpzm + uxp) * (w0 + wxp);      // edge (i+1, k)
    // vw on the y-z edge (j, k)
    const double vw00 = 0.25 * (vzm + v0) * (wym + w0);
    const double vw01 = 0.25 * (v0 + vzp) * (wymzp + wzp);      // edge (j, k+1)
    const double vw10 = 0.25 * (vypzm + vyp) * (w0 + wyp);      // edge (j+1, k)

    const double adu = -((uu0 - uum) * A.idx + (uv01 - uv00) * A.idy + (uw01 - uw00) * A.idz) +
                       (A.kx * (uxp - 2.0 * u0 + uxm) + A.ky * (uyp - 2.0 * u0 + uym) +
                        A.kz * (uzp - 2.0 * u0 + uzm));
    const double adv = -((uv10 - uv00) * A.idx + (vv0 - vvm) * A.idy + (vw01 - vw00) * A.idz) +
                       (A.kx * (vxp - 2.0 * v0 + vxm) + A.ky * (vyp - 2.0 * v0 + vym) +
                        A.kz * (vzp - 2.0 * v0 + vzm));
    const double adw = -((uw10 - uw00) * A.idx + (vw10 - vw00) * A.idy + (ww0 - wwm) * A.idz) +
                       (A.kx * (wxp - 2.0 * w0 + wxm) + A.ky * (wyp - 2.0 * w0 + wym) +
                        A.kz * (wzp - 2.0 * w0 + wzm));

    double su = A.a_dt * adu - A.g_dt * (p0 - pxm) * A.idx;
    double sv = A.a_dt * adv - A.g_dt * (p0 - pym) * A.idy;
    double sw = A.a_dt * adw - A.g_dt * (p0 - pzm) * A.idz;
    if (READ_PREV) {
      su += A.b_dt * A.ad_prev[c];
      sv += A.b_dt * A.ad_prev[c + N];
      sw += A.b_dt * A.ad_prev[c + 2 * N];
    }
    if (WRITE_AD) {
      A.ad[c] = adu;
      A.ad[c + N] = adv;
      A.ad[c + 2 * N] = adw;
    }
    A.star[c] = u0 + su;
    A.star[c + N] = v0 + sv;
    A.star[c + 2 * N] = w0 + sw;
  }
}

// The same prediction, z-marching over LDS plane tiles: a block owns a
// 64 x 4 (x, y) tile of columns and RK3_KC consecutive planes.  Each plane
// of u, v, w and p is loaded once per block, with a one-cell periodic halo
// in x and y, into a ring of four LDS planes; computing plane k reads
// planes k-1, k, k+1 from the ring while plane k+2 arrives.  One barrier
// per plane.  Every LDS slot (lx, ly) of a tile holds the value at
// ((i0 + lx) mod nx, (j0 + ly) mod ny), so ragged and wrapped tiles need
// no special case: threads outside the grid load, but do not store.
// HBM traffic is the per-cell figure above plus 2 / RK3_KC of the planes
// (the two halo planes of a block's z range).
static constexpr int RK3_TX = 64, RK3_TY = 4, RK3_KC = 64;
static constexpr int RK3_HX = RK3_TX + 2, RK3_HY = RK3_TY + 2;
static constexpr int RK3_PL = RK3_HX * RK3_HY;                  // slots per plane and field
static constexpr int RK3_HALO = 2 * RK3_HX + 2 * RK3_TY;        // halo slots per plane
static_assert(RK3_TX * RK3_TY == RK3_NT && RK3_HALO <= RK3_NT, "tile shape");

// AD and u* of the three faces a cell owns, from three LDS planes (field
// order u, v, w, p; row pitch Y) at slot c.  Shared by the tile kernels,
// so that a face computed twice (a tile's own cell and a neighbour tile's
// edge) is computed by the same code.
struct RK3Cell {
  double ad[3];
  double star[3];
};

template <int PL, int Y>
__device__ __forceinline__ RK3Cell rk3_cell(const double (*Rm)[PL], const double (*R0)[PL],
                                            const double (*Rp)[PL], int c, const RK3Args& A,
                                            const double (&prev)[3]) {
  constexpr int X = 1;
  const double u0 = R0[0][c], uxm = R0[0][c - X], uxp = R0[0][c + X], uym = R0[0][c - Y],
               uyp = R0[0][c + Y], uzm = Rm[0][c], uzp = Rp[0][c], uxpym = R0[0][c + X - Y],
               uxpzm = Rm[0][c + X];
  const double v0 = R0[1][c], vxm = R0[1][c - X], vxp = R0[1][c + X], vym = R0[1][c - Y],
               vyp = R0[1][c + Y], vzm = Rm[1][c], vzp = Rp[1][c], vxmyp = R0[1][c - X + Y],
               vypzm = Rm[1][c + Y];
  const double w0 = R0[2][c], wxm = R0[2][c - X], wxp = R0[2][c + X], wym = R0[2][c - Y],
               wyp = R0[2][c + Y], wzm = Rm[2][c], wzp = Rp[2][c], wxmzp = Rp[2][c - X],
               wymzp = Rp[2][c - Y];
  const double p0 = R0[3][c], pxm = R0[3][c - X], pym = R0[3][c - Y], pzm = Rm[3][c];

  const double uu0 = 0.25 * (u0 + uxp) * (u0 + uxp), uum = 0.25 * (uxm + u0) * (uxm + u0);
  const double vv0 = 0.25 * (v0 + vyp) * (v0 + vyp), vvm = 0.25 * (vym + v0) * (vym + v0);
  const double ww0 = 0.25 * (w0 + wzp) * (w0 + wzp), wwm = 0.25 * (wzm + w0) * (wzm + w0);
  const double uv00 = 0.25 * (uym + u0) * (vxm + v0);
  const double uv01 = 0.25 * (u0 + uyp) * (vxmyp + vyp);
  const double uv10 = 0.25 * (uxpym + uxp) * (v0 + vxp);
  const double uw00 = 0.25 * (uzm + u0) * (wxm + w0);
  const double uw01 = 0.25 * (u0 + uzp) * (wxmzp + wzp);
  const double uw10 = 0.25 * (uxpzm + uxp) * (w0 + wxp);
  const double vw00 = 0.25 * (vzm + v0) * (wym + w0);
  const double vw01 = 0.25 * (v0 + vzp) * (wymzp + wzp);
  const double vw10 = 0.25 * (vypzm + vyp) * (w0 + wyp);

  RK3Cell r;
  r.ad[0] = -((uu0 - uum) * A.idx + (uv01 - uv00) * A.idy + (uw01 - uw00) * A.idz) +
            (A.kx * (uxp - 2.0 * u0 + uxm) + A.ky * (uyp - 2.0 * u0 + uym) +
             A.kz * (uzp - 2.0 * u0 + uzm));
  r.ad[1] = -((uv10 - uv00) * A.idx + (vv0 - vvm) * A.idy + (vw01 - vw00) * A.idz) +
            (A.kx * (vxp - 2.0 * v0 + vxm) + A.ky * (vyp - 2.0 * v0 + vym) +
             A.kz * (vzp - 2.0 * v0 + vzm));
  r.ad[2] = -((uw10 - uw00) * A.idx + (vw10 - vw00) * A.idy + (ww0 - wwm) * A.idz) +
            (A.kx * (wxp - 2.0 * w0 + wxm) + A.ky * (wyp - 2.0 * w0 + wym) +
             A.kz * (wzp - 2.0 * w0 + wzm));
  r.star[0] = u0 + (A.a_dt * r.ad[0] - A.g_dt * (p0 - pxm) * A.idx + A.b_dt * prev[0]);
  r.star[1] = v0 + (A.a_dt * r.ad[1] - A.g_dt * (p0 - pym) * A.idy + A.b_dt * prev[1]);
  r.star[2] = w0 + (A.a_dt * r.ad[2] - A.g_dt * (p0 - pzm) * A.idz + A.b_dt * prev[2]);
  return r;
}

template <bool READ_PREV, bool WRITE_AD>
__global__ __launch_bounds__(RK3_NT) void rk3_predict_tiled_kernel(RK3Args A) {
  __shared__ double ring[4][4][RK3_PL];    // [plane slot][u, v, w, p][slot]
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const long long N = A.npts;
  const long long plane = (long long)nx * ny;
  const int tx = threadIdx.x & (RK3_TX - 1), ty = threadIdx.x / RK3_TX;
  const int i0 = blockIdx.x * RK3_TX, j0 = blockIdx.y * RK3_TY, k0 = blockIdx.z * RK3_KC;
  const int kend = min(k0 + RK3_KC, nz);
  auto wrap = [](int a, int n) { a %= n; return a < 0 ? a + n : a; };
  // this thread's interior slot and (for the first RK3_HALO threads) halo slot
  const int own_slot = (ty + 1) * RK3_HX + tx + 1;
  const long long own_off = wrap(i0 + tx, nx) + (long long)nx * wrap(j0 + ty, ny);
  int halo_slot = -1;
  long long halo_off = 0;
  {
    const int t = threadIdx.x;
    int lx = 0, ly = 0;
    if (t < RK3_HX) { lx = t - 1; ly = -1; }
    else if (t < 2 * RK3_HX) { lx = t - RK3_HX - 1; ly = RK3_TY; }
    else if (t < 2 * RK3_HX + RK3_TY) { lx = -1; ly = t - 2 * RK3_HX; }
    else if (t < RK3_HALO) { lx = RK3_TX; ly = t - 2 * RK3_HX - RK3_TY; }
    if (t < RK3_HALO) {
      halo_slot = (ly + 1) * RK3_HX + lx + 1;
      halo_off = wrap(i0 + lx, nx) + (long long)nx * wrap(j0 + ly, ny);
    }
  }
  const bool active = i0 + tx < nx && j0 + ty < ny;
  const double* __restrict__ src[4] = {A.vel, A.vel + N, A.vel + 2 * N, A.p};

  // plane q (k0 - 1 <= q <= kend) sits in ring slot (q - k0 + 1) & 3
  auto fetch = [&](int q, double (&own)[4], double (&halo)[4]) {
    const long long base = plane * wrap(q, nz);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      own[f] = src[f][base + own_off];
      halo[f] = halo_slot >= 0 ? src[f][base + halo_off] : 0.0;
    }
  };
  auto put = [&](int q, const double (&own)[4], const double (&halo)[4]) {
    double(*r)[RK3_PL] = ring[(q - k0 + 1) & 3];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      r[f][own_slot] = own[f];
      if (halo_slot >= 0) r[f][halo_slot] = halo[f];
    }
  };
  {
    double own[4], halo[4];
    for (int q = k0 - 1; q <= min(k0 + 1, kend); ++q) {
      fetch(q, own, halo);
      put(q, own, halo);
    }
  }
  __syncthreads();

  for (int k = k0; k < kend; ++k) {
    double own[4], halo[4];
    const bool more = k + 2 <= kend;
    if (more) fetch(k + 2, own, halo);
    const long long g = own_off + plane * k;
    double prev[3] = {0.0, 0.0, 0.0};
    if (READ_PREV && active) {
      prev[0] = A.ad_prev[g];
      prev[1] = A.ad_prev[g + N];
      prev[2] = A.ad_prev[g + 2 * N];
    }
    const RK3Cell r = rk3_cell<RK3_PL, RK3_HX>(ring[(k - k0) & 3], ring[(k - k0 + 1) & 3],
                                               ring[(k - k0 + 2) & 3], own_slot, A, prev);
    if (active) {
      if (WRITE_AD) {
        A.ad[g] = r.ad[0];
        A.ad[g + N] = r.ad[1];
        A.ad[g + 2 * N] = r.ad[2];
      }
      A.star[g] = r.star[0];
      A.star[g + N] = r.star[1];
      A.star[g + 2 * N] = r.star[2];
    }
    if (more) put(k + 2, own, halo);
    __syncthreads();
  }
}

// The tiled prediction with the right-hand side of the pressure equation,
// div(u*) / (gamma_k dt), fused (Eq. (poi_ns)): the divergence of a cell
// needs u* on its high x face and v* on its high y face, which for the
// tile's last column and row belong to the neighbouring tiles, so the
// tile holds a two-cell halo on its high sides (rows and columns of
// 64 + 3 and 4 + 3 slots) and recomputes those faces: wave 0 the cells of
// the row beyond the tile, four lanes of wave 1 the column beyond it,
// with the same cell function as the tile's own faces.  u* and v* of a
// plane pass to the neighbouring threads through a double-buffered LDS
// exchange; w* of the plane above is the next iteration's own value, so
// plane k's divergence is formed in iteration k + 1, and each block
// computes one plane beyond its z range (w* only is used there).  The
// right-hand side costs 8 B per cell instead of the 32 B of a separate
// sweep over u*.
static constexpr int RK3D_HX = RK3_TX + 3, RK3D_HY = RK3_TY + 3;  // lx in [-1, TX+1], ly in [-1, TY+1]
static constexpr int RK3D_PL = RK3D_HX * RK3D_HY;
static constexpr int RK3D_HALO = RK3D_PL - RK3_TX * RK3_TY;
static_assert(RK3D_HALO <= RK3_NT && RK3_TX + RK3_TY <= RK3_NT, "fused tile shape");

// CORRECT: the previous substep's projection is applied as the planes
// arrive instead of in a sweep of its own: the kernel reads u* and Phi of
// the previous substep (and p before it) and forms, at every slot of the
// tile, u = u* - gamma dt grad Phi and p + Phi, the velocity and pressure
// that sweep would have written (same arithmetic); it writes p + Phi of
// its own cells to p_out (a second buffer: the neighbouring tiles still
// read p).  The z gradient takes Phi of the plane below from the previous
// fetch of the same slot.
//
// FULL (nx a multiple of RK3_TX, ny of RK3_TY, nz of RK3_KC): every cell of
// every tile exists, so no lane skips a load or a store in the z loop, and
// the compiler's waits for a plane's reads leave the later reads and the
// stores in flight.  The previous AD of a plane (the own cell's, and for
// the edge lanes the edge cell's) is read before the plane three ahead,
// the halo reads of lanes without a halo slot read their own cell instead,
// and the first plane and the last two are peeled off the loop (no
// divergence yet; no plane left to read; w* only).  The other shapes keep
// the general loop, in which these reads and stores sit behind branches.
template <bool READ_PREV, bool WRITE_AD, bool CORRECT, bool FULL>
__global__ __launch_bounds__(RK3_NT) void rk3_predict_div_kernel(RK3Args A, double* __restrict__ rhs,
                                                                 double inv_gdt) {
  __shared__ double ring[4][4][RK3D_PL];             // [plane slot][u, v, w, p][slot]
  __shared__ double xu[2][RK3_TY][RK3_TX + 1];        // u* of a plane: the tile and column TX
  __shared__ double xv[2][RK3_TY + 1][RK3_TX];        // v* of a plane: the tile and row TY
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const long long N = A.npts;
  const long long plane = (long long)nx * ny;
  const int t = threadIdx.x;
  const int tx = t & (RK3_TX - 1), ty = t / RK3_TX;
  const int i0 = blockIdx.x * RK3_TX, j0 = blockIdx.y * RK3_TY, k0 = blockIdx.z * RK3_KC;
  const int kend = min(k0 + RK3_KC, nz);
  auto wrap = [](int a, int n) { a %= n; return a < 0 ? a + n : a; };
  auto slot_of = [](int lx, int ly) { return (ly + 1) * RK3D_HX + lx + 1; };
  auto off_of = [&](int lx, int ly) {
    return wrap(i0 + lx, nx) + (long long)nx * wrap(j0 + ly, ny);
  };
  const int own_slot = slot_of(tx, ty);
  const long long own_off = off_of(tx, ty);
  // halo slots, row by row: row -1 (67), rows 0..TY-1 (columns -1, TX, TX+1), rows TY, TY+1 (67 each)
  int halo_slot = -1;
  long long halo_off = 0;
  if (t < RK3D_HALO) {
    int lx, ly;
    if (t < RK3D_HX) { ly = -1; lx = t - 1; }
    else if (t < RK3D_HX + 3 * RK3_TY) {
      const int r = t - RK3D_HX;
      ly = r / 3;
      lx = r % 3 == 0 ? -1 : RK3_TX - 1 + r % 3;
    } else {
      const int r = t - RK3D_HX - 3 * RK3_TY;
      ly = RK3_TY + r / RK3D_HX;
      lx = r % RK3D_HX - 1;
    }
    halo_slot = slot_of(lx, ly);
    halo_off = off_of(lx, ly);
  }
  // edge faces: wave 0 the row TY (v* there), lanes 0..TY-1 of wave 1 the column TX (u* there)
  int edge_slot = -1;
  long long edge_off = 0;
  if (t < RK3_TX) {
    edge_slot = slot_of(t, RK3_TY);
    edge_off = off_of(t, RK3_TY);
  } else if (t < RK3_TX + RK3_TY) {
    edge_slot = slot_of(RK3_TX, t - RK3_TX);
    edge_off = off_of(RK3_TX, t - RK3_TX);
  }
  const bool active = i0 + tx < nx && j0 + ty < ny;
  // fields read per slot: u, v, w, p; with CORRECT also Phi and its x and y
  // neighbours below the slot
  constexpr int NF = CORRECT ? 7 : 4;
  const double* __restrict__ src[7] = {A.vel, A.vel + N, A.vel + 2 * N, A.p,
                                       A.phi_prev, A.phi_prev, A.phi_prev};
  long long own_o[3] = {own_off, 0, 0}, halo_o[3] = {halo_off, 0, 0};
  if (CORRECT) {
    own_o[1] = off_of(tx - 1, ty);
    own_o[2] = off_of(tx, ty - 1);
    if (halo_slot >= 0) {
      const int hl = halo_slot % RK3D_HX - 1, hr = halo_slot / RK3D_HX - 1;
      halo_o[1] = off_of(hl - 1, hr);
      halo_o[2] = off_of(hl, hr - 1);
    }
  }
  double phib_own = 0.0, phib_halo = 0.0;   // CORRECT: Phi of the plane below, at the two slots

  // plane q (k0 - 1 <= q <= kend + 1) sits in ring slot (q - k0 + 1) & 3
  auto fetch = [&](int q, double (&own)[7], double (&halo)[7]) {
    const long long base = plane * wrap(q, nz);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int o = f < 5 ? 0 : f - 4;
      own[f] = src[f][base + own_o[o]];
      halo[f] = halo_slot >= 0 ? src[f][base + halo_o[o]] : 0.0;
    }
  };
  auto correct = [&](double (&val)[7], double& phib) {
    if (CORRECT) {
      const double ph = val[4];
      val[0] = val[0] - A.c_gdt * ((ph - val[5]) * A.idx);
      val[1] = val[1] - A.c_gdt * ((ph - val[6]) * A.idy);
      val[2] = val[2] - A.c_gdt * ((ph - phib) * A.idz);
      val[3] = val[3] + ph;
      phib = ph;
    }
  };
  auto put = [&](int q, double (&own)[7], double (&halo)[7]) {
    correct(own, phib_own);
    if (halo_slot >= 0) correct(halo, phib_halo);
    double(*r)[RK3D_PL] = ring[(q - k0 + 1) & 3];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      r[f][own_slot] = own[f];
      if (halo_slot >= 0) r[f][halo_slot] = halo[f];
    }
  };
  if (CORRECT) {
    const long long base = plane * wrap(k0 - 2, nz);
    phib_own = A.phi_prev[base + own_off];
    if (halo_slot >= 0) phib_halo = A.phi_prev[base + halo_off];
  }
  auto load_prev = [&](long long g, double (&prev)[3]) {
    prev[0] = prev[1] = prev[2] = 0.0;
    if (READ_PREV) {
      prev[0] = A.ad_prev[g];
      prev[1] = A.ad_prev[g + N];
      prev[2] = A.ad_prev[g + 2 * N];
    }
  };
  // FULL: the halo reads of lanes without a halo slot read their own cell
  long long hsel_o[3] = {halo_o[0], halo_o[1], halo_o[2]};
  if (halo_slot < 0) {
    hsel_o[0] = own_o[0];
    hsel_o[1] = own_o[1];
    hsel_o[2] = own_o[2];
  }
  auto fetch_full = [&](int q, double (&own)[7], double (&halo)[7]) {
    const long long base = plane * wrap(q, nz);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int o = f < 5 ? 0 : f - 4;
      own[f] = src[f][base + own_o[o]];
      halo[f] = src[f][base + hsel_o[o]];
    }
  };
  {
    double own[7], halo[7];
    for (int q = k0 - 1; q <= k0 + 1; ++q) {
      if (FULL) fetch_full(q, own, halo);
      else fetch(q, own, halo);
      put(q, own, halo);
    }
  }
  // plane reads run two planes ahead of the arithmetic: plane k + 2 is in
  // flight while plane k is computed
  double own_n[7], halo_n[7];
  // FULL: the previous AD of plane k (the own cell's and the edge cell's),
  // read one plane ahead
  double prev_n[3], eprev_n[3];
  const long long edge_o = edge_slot >= 0 ? edge_off : own_off;
  if (FULL) {
    load_prev(own_off + plane * wrap(k0, nz), prev_n);
    load_prev(edge_o + plane * wrap(k0, nz), eprev_n);
    fetch_full(k0 + 2, own_n, halo_n);
  } else if (k0 + 2 <= kend + 1) {
    fetch(k0 + 2, own_n, halo_n);
  }
  __syncthreads();

  double star_below[3] = {0.0, 0.0, 0.0};   // this thread's u*, v*, w* of plane k - 1
  if constexpr (FULL) {
    // FIRST: no divergence yet; MORE: plane k + 3 is read (and the next
    // plane has edge cells); LAST: k == kend.  The reads of a step go out
    // in the order previous AD of plane k + 1, plane k + 3, before the
    // step's stores: waiting for this step's previous AD then waits for
    // nothing issued after the last step's reads.
    auto step = [&](int k, auto first_c, auto more_c, auto last_c) {
      constexpr bool FIRST = decltype(first_c)::value;
      constexpr bool MORE = decltype(more_c)::value;
      constexpr bool LAST = decltype(last_c)::value;
      const long long base = plane * wrap(k, nz);
      const long long g = own_off + base;
      double prev[3], eprev[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        prev[c] = prev_n[c];
        eprev[c] = eprev_n[c];
      }
      if constexpr (!LAST) load_prev(own_off + plane * wrap(k + 1, nz), prev_n);
      if constexpr (MORE) load_prev(edge_o + plane * wrap(k + 1, nz), eprev_n);
      double own_f[7], halo_f[7];
      if constexpr (MORE) fetch_full(k + 3, own_f, halo_f);
      const double(*Rm)[RK3D_PL] = ring[(k - k0) & 3];
      const double(*R0)[RK3D_PL] = ring[(k - k0 + 1) & 3];
      const double(*Rp)[RK3D_PL] = ring[(k - k0 + 2) & 3];
      const RK3Cell r = rk3_cell<RK3D_PL, RK3D_HX>(Rm, R0, Rp, own_slot, A, prev);
      // the outputs are stored with the nontemporal hint (an RK3 step of
      // the periodic 512^3 Taylor-Green vortex: 18.45 -> 17.96 ms with
      // these stores hinted; hinting the previous-AD reads as well was
      // slower, 17.89 -> 18.04 ms)
      if constexpr (!LAST) {
        if (WRITE_AD) {
          __builtin_nontemporal_store(r.ad[0], &A.ad[g]);
          __builtin_nontemporal_store(r.ad[1], &A.ad[g + N]);
          __builtin_nontemporal_store(r.ad[2], &A.ad[g + 2 * N]);
        }
        __builtin_nontemporal_store(r.star[0], &A.star[g]);
        __builtin_nontemporal_store(r.star[1], &A.star[g + N]);
        __builtin_nontemporal_store(r.star[2], &A.star[g + 2 * N]);
        if (CORRECT) __builtin_nontemporal_store(R0[3][own_slot], &A.p_out[g]);
      }
      if constexpr (!FIRST) {                 // divergence of plane k - 1
        const int b = (k - 1 - k0) & 1;
        const double du = xu[b][ty][tx + 1] - xu[b][ty][tx];
        const double dv = xv[b][ty + 1][tx] - xv[b][ty][tx];
        const double dw = r.star[2] - star_below[2];
        __builtin_nontemporal_store((du * A.idx + dv * A.idy + dw * A.idz) * inv_gdt,
                                    &rhs[g - base + plane * (k - 1)]);
      }
      if constexpr (!LAST) {
        const int b = (k - k0) & 1;
        xu[b][ty][tx] = r.star[0];
        xv[b][ty][tx] = r.star[1];
        if (edge_slot >= 0) {
          const RK3Cell e = rk3_cell<RK3D_PL, RK3D_HX>(Rm, R0, Rp, edge_slot, A, eprev);
          if (t < RK3_TX) xv[b][RK3_TY][t] = e.star[1];
          else xu[b][t - RK3_TX][RK3_TX] = e.star[0];
        }
      }
      star_below[0] = r.star[0];
      star_below[1] = r.star[1];
      star_below[2] = r.star[2];
      if constexpr (!LAST) put(k + 2, own_n, halo_n);
      if constexpr (MORE) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          own_n[f] = own_f[f];
          halo_n[f] = halo_f[f];
        }
      }
      __syncthreads();
    };
    using yes = std::true_type;
    using no = std::false_type;
    step(k0, yes{}, yes{}, no{});
    for (int k = k0 + 1; k < kend - 1; ++k) step(k, no{}, yes{}, no{});
    step(kend - 1, no{}, no{}, no{});
    step(kend, no{}, no{}, yes{});
    return;
  }
  for (int k = k0; k <= kend; ++k) {        // k == kend: w* above the range only
    double own_f[7], halo_f[7];
    const bool more = k + 3 <= kend + 1;
    if (more) fetch(k + 3, own_f, halo_f);
    const long long base = plane * wrap(k, nz);
    const long long g = own_off + base;
    double prev[3];
    load_prev(g, prev);
    const double(*Rm)[RK3D_PL] = ring[(k - k0) & 3];
    const double(*R0)[RK3D_PL] = ring[(k - k0 + 1) & 3];
    const double(*Rp)[RK3D_PL] = ring[(k - k0 + 2) & 3];
    const RK3Cell r = rk3_cell<RK3D_PL, RK3D_HX>(Rm, R0, Rp, own_slot, A, prev);
    if (k < kend && active) {
      if (WRITE_AD) {
        A.ad[g] = r.ad[0];
        A.ad[g + N] = r.ad[1];
        A.ad[g + 2 * N] = r.ad[2];
      }
      A.star[g] = r.star[0];
      A.star[g + N] = r.star[1];
      A.star[g + 2 * N] = r.star[2];
      if (CORRECT) A.p_out[g] = R0[3][own_slot];
    }
    if (k > k0 && active) {                 // divergence of plane k - 1
      const int b = (k - 1 - k0) & 1;
      const double du = xu[b][ty][tx + 1] - xu[b][ty][tx];
      const double dv = xv[b][ty + 1][tx] - xv[b][ty][tx];
      const double dw = r.star[2] - star_below[2];
      rhs[g - base + plane * (k - 1)] = (du * A.idx + dv * A.idy + dw * A.idz) * inv_gdt;
    }
    if (k < kend) {
      const int b = (k - k0) & 1;
      xu[b][ty][tx] = r.star[0];
      xv[b][ty][tx] = r.star[1];
      if (edge_slot >= 0) {
        double eprev[3];
        load_prev(edge_off + base, eprev);
        const RK3Cell e = rk3_cell<RK3D_PL, RK3D_HX>(Rm, R0, Rp, edge_slot, A, eprev);
        if (t < RK3_TX) xv[b][RK3_TY][t] = e.star[1];
        else xu[b][t - RK3_TX][RK3_TX] = e.star[0];
      }
    }
    star_below[0] = r.star[0];
    star_below[1] = r.star[1];
    star_below[2] = r.star[2];
    if (k + 2 <= kend + 1) put(k + 2, own_n, halo_n);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      own_n[f] = own_f[f];
      halo_n[f] = halo_f[f];
    }
    __syncthreads();
  }
}

}  // namespace poisson_dev
