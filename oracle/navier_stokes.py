"""Oracle: one time step of the incompressible Navier-Stokes integration the
Poisson solve serves (Sec. 2): the low-storage three-substep Runge-Kutta
scheme with a pressure correction at every substep (Eq. (up), Eq. (poi_ns)
and the two updates after it), on a tri-periodic uniform staggered grid,
the setting of the Taylor-Green validation case (Sec. 4.1, Table 3).

Test infrastructure only (see ``oracle/__init__.py``).

Readings (the paper states the scheme in semi-discrete form only):

* Grid and layout.  Periodic along every axis, n cells of uniform width
  per axis (the widths of the three axes may differ).  Scalars (p, Phi) at
  cell centres; the velocity component along an axis on the faces normal
  to it, face i of an axis between cells i-1 (cyclically) and i, i.e. the
  low face of cell i, stored at the cell's index: u[k, j, i] lives at
  (i dx, (j + 1/2) dy, (k + 1/2) dz).  This is the periodic case of
  ``projection``'s layout.
* AD = -(u . grad) u + nu lap(u) is discretised with second-order central
  differences in divergence (conservative) form, -div(u u): each product
  is formed where its derivative needs it (the square of a velocity
  component at cell centres, the cross products on the cell edges), from
  arithmetic means of the two nearest stored values.  For a discretely
  divergence-free field this equals the advective form to second order and
  conserves the discrete kinetic energy and momentum exactly.  The viscous
  term is the three-point second difference along each axis.
* The pressure gradient in the prediction is the face gradient of
  ``projection`` (difference of the two neighbouring cell values over the
  spacing), the same operator that projects with Phi.
* p^{k-1/2} before the first substep is an input; AD^{k-1} is not read in
  the first substep (beta_1 = 0), so the previous step's AD is never needed.
* The Poisson solve of each substep is ``poisson.solve`` with (P, P, P):
  singular, so Phi has zero mean (the gauge of the pressure).
"""
import numpy as np

from . import poisson as ps
from . import projection as pj

ALPHA = (8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0)
BETA = (0.0, -17.0 / 60.0, -5.0 / 12.0)
GAMMA = tuple(a + b for a, b in zip(ALPHA, BETA))

PERIODIC = ("P", "P", "P")
X, Y, Z = 2, 1, 0      # array axes of f[k, j, i]


def _fwd(a, ax):
    """Value at index + 1 along array axis ax (cyclic)."""
    return np.roll(a, -1, axis=ax)


def _bwd(a, ax):
    """Value at index - 1 along array axis ax (cyclic)."""
    return np.roll(a, 1, axis=ax)


def _mean_bwd(a, ax):
    """Mean of the value at the index and at index - 1 along ax."""
    return 0.5 * (a + _bwd(a, ax))


def advection(u, v, w, dx, dy, dz):
    """-div(u u) for each component, at that component's faces.

    Products and where they live (cell (i, j, k) spans [i, i+1] dx etc.):
      uu, vv, ww  at cell centres: square of the mean of the component's
                  two faces of that cell (index and index + 1);
      uv          on the x-y edge at (i dx, j dy, .): mean of u over j-1, j
                  times mean of v over i-1, i;  uw, vw likewise.
    A face's derivative of a product is the difference of its values on
    the two sides of the face over the spacing."""
    u, v, w = (np.asarray(a, dtype=np.float64) for a in (u, v, w))
    uu = (0.5 * (u + _fwd(u, X))) ** 2          # centre of cell i
    vv = (0.5 * (v + _fwd(v, Y))) ** 2
    ww = (0.5 * (w + _fwd(w, Z))) ** 2
    uv = _mean_bwd(u, Y) * _mean_bwd(v, X)      # edge (i dx, j dy)
    uw = _mean_bwd(u, Z) * _mean_bwd(w, X)      # edge (i dx, k dz)
    vw = _mean_bwd(v, Z) * _mean_bwd(w, Y)      # edge (j dy, k dz)
    # u face i: centres i-1 and i along x; edges j and j+1 along y; k and k+1 along z
    au = -((uu - _bwd(uu, X)) / dx + (_fwd(uv, Y) - uv) / dy + (_fwd(uw, Z) - uw) / dz)
    av = -((_fwd(uv, X) - uv) / dx + (vv - _bwd(vv, Y)) / dy + (_fwd(vw, Z) - vw) / dz)
    aw = -((_fwd(uw, X) - uw) / dx + (_fwd(vw, Y) - vw) / dy + (ww - _bwd(ww, Z)) / dz)
    return au, av, aw


def laplacian(a, dx, dy, dz):
    """Three-point second difference along each axis (periodic)."""
    a = np.asarray(a, dtype=np.float64)
    return ((_fwd(a, X) - 2.0 * a + _bwd(a, X)) / dx ** 2
            + (_fwd(a, Y) - 2.0 * a + _bwd(a, Y)) / dy ** 2
            + (_fwd(a, Z) - 2.0 * a + _bwd(a, Z)) / dz ** 2)


def advection_diffusion(u, v, w, dx, dy, dz, nu):
    """AD = -(u . grad) u + nu lap(u) (Sec. 2, after the substep equations),
    per component at its faces."""
    au, av, aw = advection(u, v, w, dx, dy, dz)
    return (au + nu * laplacian(u, dx, dy, dz), av + nu * laplacian(v, dx, dy, dz),
            aw + nu * laplacian(w, dx, dy, dz))


def widths(n, d):
    return np.full(n, float(d))


def prediction(k, u, v, w, p, ad_prev, dt, nu, dx, dy, dz):
    """Eq. (up) for substep k: u* = u + dt (alpha_k AD(u) + beta_k AD_prev
    - gamma_k grad p).  Returns ((u*, v*, w*), ad), ad = AD(u)."""
    a, b, g = ALPHA[k - 1], BETA[k - 1], GAMMA[k - 1]
    nz, ny, nx = np.shape(u)
    ad = advection_diffusion(u, v, w, dx, dy, dz, nu)
    gp = pj.gradient(p, widths(nx, dx), widths(ny, dy), widths(nz, dz), PERIODIC)
    star = []
    for c in range(3):
        prev = b * ad_prev[c] if k > 1 else 0.0
        star.append(np.asarray((u, v, w)[c], float) + dt * (a * ad[c] + prev - g * gp[c]))
    return tuple(star), ad


def rk3_substep(k, u, v, w, p, ad_prev, dt, nu, dx, dy, dz):
    """Substep k (1, 2 or 3) of Eq. (up) and the pressure correction:

      u* = u + dt (alpha_k AD(u) + beta_k AD_prev - gamma_k grad p)
      lap Phi = div(u*) / (gamma_k dt)
      u  = u* - gamma_k dt grad Phi,   p = p + Phi

    ``ad_prev``: the AD of the previous substep (ignored for k = 1).
    Returns (u, v, w, p, ad, phi) with ad = AD(u) of this substep's input."""
    g = GAMMA[k - 1]
    nz, ny, nx = np.shape(u)
    hx, hy, hz = widths(nx, dx), widths(ny, dy), widths(nz, dz)
    (us, vs, ws), ad = prediction(k, u, v, w, p, ad_prev, dt, nu, dx, dy, dz)
    rhs = pj.projection_rhs(us, vs, ws, g * dt, hx, hy, hz, PERIODIC)
    phi = ps.solve(rhs, hx, hy, hz, *PERIODIC)
    u1, v1, w1, p1 = pj.project(us, vs, ws, p, phi, g * dt, hx, hy, hz, PERIODIC)
    return u1, v1, w1, p1, ad, phi


def rk3_step(u, v, w, p, dt, nu, dx, dy, dz):
    """One time step: the three substeps in order (gamma_1 + gamma_2 +
    gamma_3 = 1, so the step advances time by dt).  Returns (u, v, w, p)."""
    ad = None
    for k in (1, 2, 3):
        u, v, w, p, ad, _ = rk3_substep(k, u, v, w, p, ad, dt, nu, dx, dy, dz)
    return u, v, w, p


def stable_dt(u, v, w, dx, dy, dz, nu):
    """The sufficient stability bound on dt quoted in Sec. 2:
    min(1.65 dr^2 / nu, sqrt(3) dr / max(|u| + |v| + |w|)), dr the smallest
    spacing; the maximum is taken over cells, each cell pairing the three
    components stored at its index (its low faces)."""
    dr = min(dx, dy, dz)
    vmax = float(np.max(np.abs(u) + np.abs(v) + np.abs(w)))
    visc = 1.65 * dr * dr / nu if nu > 0 else np.inf
    conv = np.sqrt(3.0) * dr / vmax if vmax > 0 else np.inf
    return min(visc, conv)
