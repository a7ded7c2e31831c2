"""Oracle: the pressure-correction steps on either side of the Poisson solve
(Sec. 2, the substep equations after Eq. (up)): the right-hand side
div(u*) / (gamma_k dt) (Eq. (poi_ns)), the projection u = u* - gamma_k dt
grad(Phi) and the pressure update p = p + Phi, on the staggered (marker and
cell) grid of Sec. 2.

Test infrastructure only (see ``oracle/__init__.py``).

Readings (the paper gives the equations in semi-discrete form only):

* Layout.  Phi and p live at cell centres, f[k, j, i] (x fastest).  The
  velocity component along an axis lives on the faces normal to that axis.
  Along a periodic axis of n cells there are n faces, face f between cells
  f-1 (cyclically) and f; along a walled axis there are n + 1, face 0 the
  low wall, face n the high wall.  So u has shape (nz, ny, nx + 1) when x
  is walled, (nz, ny, nx) when periodic, and likewise v along y, w along z.
* Divergence at a cell: the net outward flux over the cell volume, i.e. the
  difference of the two face values along each axis over that axis's cell
  width (finite-volume form; Eq. (poi)'s central differences when uniform).
* Gradient at a face: the difference of the two adjacent cell values over
  the distance of their centres (the mean of the two widths).  At a wall
  the ghost cell of the Poisson operator's boundary rule applies: a Neumann
  face has zero normal gradient (the projection leaves its velocity as it
  is, as the paper requires of prescribed velocities), a Dirichlet face
  (Phi = 0 on the face) has gradient 2 Phi_edge / h_edge pointing inward.
  With these rules the divergence of the gradient is the seven-point
  operator of the solve, row for row, so the projected velocity has zero
  divergence up to rounding.
"""
import numpy as np

from . import poisson as ps
from .poisson import AXIS
from .tridiagonal import HIGH, LOW

AXES = ("x", "y", "z")


def face_count(n, kind):
    """Faces along an axis of n cells: n if periodic, n + 1 if walled."""
    return n if kind == "P" else n + 1


def velocity_shape(comp, nx, ny, nz, bcs):
    """Shape (nz, ny, nx) order of velocity component `comp` ('x', 'y', 'z')."""
    dims = {"x": nx, "y": ny, "z": nz}
    kinds = dict(zip(AXES, bcs))
    dims[comp] = face_count(dims[comp], kinds[comp])
    return (dims["z"], dims["y"], dims["x"])


def _centre_distances(h, kind):
    """dc[f] for the faces of an axis: the distance between the centres of
    the two cells that share face f (for a wall face: the edge width, the
    distance to the mirrored ghost cell)."""
    h = np.asarray(h, dtype=np.float64)
    n = h.size
    if kind == "P":
        return 0.5 * (np.roll(h, 1) + h)                      # face f: cells f-1 (cyclic) and f
    dc = np.empty(n + 1)
    dc[1:n] = 0.5 * (h[:-1] + h[1:])
    dc[0] = h[0]
    dc[n] = h[-1]
    return dc


def divergence(u, v, w, hx, hy, hz, bcs):
    """Divergence at cell centres of the face velocities (u, v, w)."""
    out = 0.0
    for comp, vel, h, kind in zip(AXES, (u, v, w), (hx, hy, hz), bcs):
        ax = AXIS[comp]
        vel = np.asarray(vel, dtype=np.float64)
        h = np.asarray(h, dtype=np.float64)
        n = h.size
        if kind == "P":
            hi = np.roll(vel, -1, axis=ax)          # face f + 1 (cyclic) is the high face of cell f
            lo = vel
        else:
            hi = np.take(vel, np.arange(1, n + 1), axis=ax)
            lo = np.take(vel, np.arange(0, n), axis=ax)
        shape = [1, 1, 1]
        shape[ax] = n
        out = out + (hi - lo) / h.reshape(shape)
    return out


def gradient(phi, hx, hy, hz, bcs):
    """Gradient of the cell field phi on the faces: (gx, gy, gz), each in the
    shape of its velocity component."""
    phi = np.asarray(phi, dtype=np.float64)
    out = []
    for comp, h, kind in zip(AXES, (hx, hy, hz), bcs):
        ax = AXIS[comp]
        h = np.asarray(h, dtype=np.float64)
        n = h.size
        dc = _centre_distances(h, kind)
        shape = [1, 1, 1]
        shape[ax] = dc.size
        if kind == "P":
            diff = phi - np.roll(phi, 1, axis=ax)                 # Phi_f - Phi_{f-1}
        else:
            first = np.take(phi, [0], axis=ax)
            last = np.take(phi, [n - 1], axis=ax)
            # ghost cells: N face -> the edge value (zero gradient), D face -> minus it
            ghost_lo = first if LOW[kind] == "N" else -first
            ghost_hi = last if HIGH[kind] == "N" else -last
            ext = np.concatenate([ghost_lo, phi, ghost_hi], axis=ax)
            diff = np.diff(ext, axis=ax)                          # faces 0 .. n
        out.append(diff / dc.reshape(shape))
    return tuple(out)


def projection_rhs(u, v, w, gamma_dt, hx, hy, hz, bcs):
    """Right-hand side of Eq. (poi_ns): div(u*) / (gamma_k dt)."""
    return divergence(u, v, w, hx, hy, hz, bcs) / gamma_dt


def project(u, v, w, p, phi, gamma_dt, hx, hy, hz, bcs):
    """The two updates after the solve: u = u* - gamma_k dt grad(Phi) and
    p = p + Phi.  Returns new arrays (u, v, w, p)."""
    gx, gy, gz = gradient(phi, hx, hy, hz, bcs)
    return (np.asarray(u, float) - gamma_dt * gx, np.asarray(v, float) - gamma_dt * gy,
            np.asarray(w, float) - gamma_dt * gz, np.asarray(p, float) + phi)


def pressure_correction(u, v, w, p, gamma_dt, hx, hy, hz, bcs):
    """One pressure-correction step (Sec. 2): the right-hand side of
    Eq. (poi_ns), the solve, and the two updates.  Returns (u, v, w, p, phi)."""
    rhs = projection_rhs(u, v, w, gamma_dt, hx, hy, hz, bcs)
    phi = ps.solve(rhs, hx, hy, hz, *bcs)
    u1, v1, w1, p1 = project(u, v, w, p, phi, gamma_dt, hx, hy, hz, bcs)
    return u1, v1, w1, p1, phi
