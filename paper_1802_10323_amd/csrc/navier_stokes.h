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
// One thread per cell computes the three faces that cell owns; neighbours
// along x come from the adjacent lanes' lines, along y and z from the
// caches.  Traffic per cell: velocity 24 B, p 8 B, AD_prev 24 B (read
// when beta_k != 0), AD 24 B (written when the next substep needs it),
// u* 24 B.
#pragma once
#include "refine_kernels.h"

namespace poisson_dev {

struct RK3Args {
  const double* vel;       // u, v, w (3 npts)
  const double* p;         // npts
  const double* ad_prev;   // 3 npts, read when READ_PREV
  double* ad;              // 3 npts, written when WRITE_AD
  double* star;            // 3 npts: the prediction u*
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

}  // namespace poisson_dev
