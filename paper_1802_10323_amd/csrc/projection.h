// projection.h - the pressure-correction steps on either side of the
// Poisson solve (Sec. 2: the right-hand side of Eq. (poi_ns) and the two
// updates that follow it), on the staggered grid.
//
// Layout: Phi, p and the right-hand side at cell centres (nx*ny*nz, x
// fastest).  The velocity component along an axis on the faces normal to
// it: n faces along a periodic axis (face f between cells f-1, cyclically,
// and f), n + 1 along a walled one (face 0 the low wall, face n the high
// wall); the other two extents are those of the cells.
//
// Face gradient of a cell field: (Phi_f - Phi_{f-1}) / dc_f, dc_f the
// distance of the two centres.  Walls use the ghost cells of the solve's
// boundary rule: a Neumann wall has zero gradient (the projection leaves
// its velocity untouched), a Dirichlet wall (Phi = 0 on it) has
// 2 Phi_edge / h_edge towards the inside.  The divergence of the gradient
// is then the solve's seven-point operator row for row, so the projected
// velocity is divergence-free up to rounding.
//
// Both kernels are one HBM sweep over the cells (x fastest across the
// threads): the right-hand side reads three face arrays and writes one
// cell array (32 B per cell), the update reads Phi, the three face arrays
// and p and writes the face arrays (in place or into a second set) and p
// (72 B per cell).
#pragma once
#include "refine_kernels.h"

namespace poisson_dev {

// One axis of the projection: n cells; walled (n + 1 faces) or periodic;
// wall kinds (0 Neumann, 1 Dirichlet); inv_h[n] = 1 / cell width;
// inv_dc[faces] = 1 / centre distance (at a wall: 1 / edge width).
struct ProjAxis {
  const double* inv_h;
  const double* inv_dc;
  int n;
  int walled;
  int lo_dirichlet;
  int hi_dirichlet;
};

struct ProjGeom {
  ProjAxis ax[3];
  long long npts;
};

static constexpr int PROJ_NT = 256;
static constexpr int PROJ_BLOCKS = 8192;   // grid-stride blocks of the right-hand side

// rhs = div(u, v, w) * inv_gdt at every cell.
__global__ __launch_bounds__(PROJ_NT) void proj_rhs_kernel(const double* __restrict__ u,
                                                           const double* __restrict__ v,
                                                           const double* __restrict__ w,
                                                           double inv_gdt, double* __restrict__ rhs,
                                                           ProjGeom G) {
  const int nx = G.ax[0].n, ny = G.ax[1].n, nz = G.ax[2].n;
  const int ux = nx + G.ax[0].walled;          // faces along x
  const int vy = ny + G.ax[1].walled;          // faces along y
  const long long step = (long long)gridDim.x * PROJ_NT;
  const long long first = blockIdx.x * (long long)PROJ_NT + threadIdx.x;
  GridWalk at(first, step, nx, ny);
  for (long long c = first; c < G.npts; c += step, at.advance()) {
    const int i = at.i, j = at.j, k = at.k;
    // x: faces i and i + 1 of row (j, k)
    const long long ur = (long long)ux * (j + (long long)ny * k);
    const double du = u[ur + (G.ax[0].walled || i + 1 < nx ? i + 1 : 0)] - u[ur + i];
    // y: faces j and j + 1 of column (i, k)
    const long long vb = i + (long long)nx * vy * k;
    const double dv = v[vb + (long long)nx * (G.ax[1].walled || j + 1 < ny ? j + 1 : 0)] -
                      v[vb + (long long)nx * j];
    // z: faces k and k + 1 of column (i, j)
    const long long wb = i + (long long)nx * j;
    const long long plane = (long long)nx * ny;
    const double dw = w[wb + plane * (G.ax[2].walled || k + 1 < nz ? k + 1 : 0)] -
                      w[wb + plane * k];
    rhs[c] = (du * G.ax[0].inv_h[i] + dv * G.ax[1].inv_h[j] + dw * G.ax[2].inv_h[k]) * inv_gdt;
  }
}

// Gradient of phi on the low face of the cell at offset `c`, whose index
// along the axis (stride s) is f; `apply` is false on a Neumann wall face,
// whose velocity the projection leaves as it is.
__device__ __forceinline__ double proj_low_grad(const double* __restrict__ phi, long long c,
                                                long long s, int f, const ProjAxis& A,
                                                bool& apply) {
  const double p0 = phi[c];
  apply = true;
  if (f > 0) return (p0 - phi[c - s]) * A.inv_dc[f];
  if (!A.walled) return (p0 - phi[c + s * (A.n - 1)]) * A.inv_dc[0];   // wrap face
  if (!A.lo_dirichlet) {                                               // Neumann wall
    apply = false;
    return 0.0;
  }
  return 2.0 * p0 * A.inv_dc[0];                                       // Dirichlet wall
}

// u = u_in - gdt grad(phi) on every face, p += phi at every cell; in place
// when u_in == u (each face is read before it is written, by the same
// thread, and by no other).  z-marching: a block owns a 64 x 4 tile of
// (i, j) columns and PROJ_KC consecutive planes; each thread walks its
// column upward with Phi of the cell below in a register, so the z
// gradient reads no other plane (the x and y neighbours come from the
// lines the adjacent lanes and rows load).
static constexpr int PROJ_TX = 64, PROJ_TY = 4, PROJ_KC = 32;

__global__ __launch_bounds__(PROJ_NT) void proj_update_zmarch_kernel(
    const double* __restrict__ phi, double gdt, const double* u_in, const double* v_in,
    const double* w_in, double* u, double* v, double* w, double* __restrict__ p, ProjGeom G) {
  const int nx = G.ax[0].n, ny = G.ax[1].n, nz = G.ax[2].n;
  const int ux = nx + G.ax[0].walled;
  const int vy = ny + G.ax[1].walled;
  const long long plane = (long long)nx * ny;
  const int i = blockIdx.x * PROJ_TX + (threadIdx.x & (PROJ_TX - 1));
  const int j = blockIdx.y * PROJ_TY + threadIdx.x / PROJ_TX;
  const int k0 = blockIdx.z * PROJ_KC;
  const int kend = min(k0 + PROJ_KC, nz);
  if (i >= nx || j >= ny) return;
  const ProjAxis& Z = G.ax[2];
  const long long col = i + (long long)nx * j;
  // Phi below the first plane: the plane under it, the periodic wrap, or none (a wall)
  double below = 0.0;
  if (k0 > 0) below = phi[col + plane * (k0 - 1)];
  else if (!Z.walled) below = phi[col + plane * (nz - 1)];
  for (int k = k0; k < kend; ++k) {
    const long long c = col + plane * k;
    bool ax_, ay_;
    const double gx = proj_low_grad(phi, c, 1, i, G.ax[0], ax_);
    const double gy = proj_low_grad(phi, c, nx, j, G.ax[1], ay_);
    const double ph = phi[c];
    bool az_ = true;
    double gz;
    if (k > 0 || !Z.walled) gz = (ph - below) * Z.inv_dc[k];
    else if (!Z.lo_dirichlet) { az_ = false; gz = 0.0; }
    else gz = 2.0 * ph * Z.inv_dc[0];
    const long long fu = (long long)ux * (j + (long long)ny * k) + i;
    const long long fv = i + (long long)nx * (j + (long long)vy * k);
    const long long fw = col + plane * k;
    const double u0 = u_in[fu], v0 = v_in[fv], w0 = w_in[fw], p0 = p[c];
    const bool xh = G.ax[0].walled && i == nx - 1;
    const bool yh = G.ax[1].walled && j == ny - 1;
    const bool zh = Z.walled && k == nz - 1;
    const double uh = xh ? u_in[fu + 1] : 0.0;
    const double vh = yh ? v_in[fv + nx] : 0.0;
    const double wh = zh ? w_in[fw + plane] : 0.0;
    u[fu] = ax_ ? u0 - gdt * gx : u0;
    v[fv] = ay_ ? v0 - gdt * gy : v0;
    w[fw] = az_ ? w0 - gdt * gz : w0;
    if (xh) u[fu + 1] = G.ax[0].hi_dirichlet ? uh - gdt * (-2.0 * ph * G.ax[0].inv_dc[nx]) : uh;
    if (yh) v[fv + nx] = G.ax[1].hi_dirichlet ? vh - gdt * (-2.0 * ph * G.ax[1].inv_dc[ny]) : vh;
    if (zh) w[fw + plane] = Z.hi_dirichlet ? wh - gdt * (-2.0 * ph * Z.inv_dc[nz]) : wh;
    p[c] = p0 + ph;
    below = ph;
  }
}

}  // namespace poisson_dev
