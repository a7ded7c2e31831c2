"""Oracle: the FP64 direct solve of the staggered second-order Poisson
equation by eigenfunction expansion, taking the paper's steps in order
(Sec. 2.1, the three-step list after Table 2):

1. forward transforms of f along the two transformed axes, in turn;
2. Gauss elimination of the reduced tridiagonal system (Eq. (poi_reduced))
   of every column along the remaining axis;
3. backward transforms along the two transformed axes, in reverse order.

plus the seven-point operator itself (Eq. (poi), generalised to a
non-uniform solve axis), which defines what the solve must satisfy.

Test infrastructure only (see ``oracle/__init__.py``).

Arrays are indexed f[k, j, i] (z, y, x): x is the last, fastest axis.
"""
import numpy as np

from . import transforms as tr
from . import tridiagonal as td

AXIS = {"x": 2, "y": 1, "z": 0}


def is_singular(bcx, bcy, bcz, shift=0.0):
    """The operator has a null space (the constants) iff no face is Dirichlet,
    i.e. every axis is periodic or Neumann-Neumann (staggered or on nodes),
    and there is no Helmholtz shift."""
    return shift == 0.0 and all(k in ("P", "NN", "NNn") for k in (bcx, bcy, bcz))


def volume_weights(hx, hy, hz):
    """Cell volumes w[k, j, i] = hz_k hy_j hx_i (the left null vector of the
    operator in the singular case)."""
    return (np.asarray(hz, dtype=np.float64)[:, None, None]
            * np.asarray(hy, dtype=np.float64)[None, :, None]
            * np.asarray(hx, dtype=np.float64)[None, None, :])


def weighted_mean(f, hx, hy, hz):
    w = volume_weights(hx, hy, hz)
    return float((w * f).sum() / w.sum())


def apply_operator(phi, hx, hy, hz, bcx, bcy, bcz, shift=0.0):
    """(A phi)[k, j, i]: the seven-point operator of Eq. (poi), with the
    one-dimensional rows of ``tridiagonal.coefficients`` along each axis
    (uniform widths give exactly the central differences of Eq. (poi)),
    plus ``shift`` * phi (the Helmholtz operator of an implicit diffusion
    step, Sec. 2)."""
    phi = np.asarray(phi, dtype=np.float64)
    out = shift * phi
    for name, h, kind in (("x", hx, bcx), ("y", hy, bcy), ("z", hz, bcz)):
        ax = AXIS[name]
        a, b, c, periodic = td.coefficients(h, kind)
        n = phi.shape[ax]
        shape = [1, 1, 1]
        shape[ax] = n
        a = a.reshape(shape)
        b = b.reshape(shape)
        c = c.reshape(shape)
        lower = np.roll(phi, 1, axis=ax)    # x_{k-1} (wraps: only used if periodic)
        upper = np.roll(phi, -1, axis=ax)   # x_{k+1}
        out += b * phi + a * lower + c * upper   # a[0] = c[n-1] = 0 unless periodic
    return out


def residual(f, phi, hx, hy, hz, bcx, bcy, bcz, shift=0.0):
    """r = f - A phi (f projected first when the operator is singular)."""
    f = np.asarray(f, dtype=np.float64)
    if is_singular(bcx, bcy, bcz, shift):
        f = f - weighted_mean(f, hx, hy, hz)
    return f - apply_operator(phi, hx, hy, hz, bcx, bcy, bcz, shift)


def _uniform_spacing(h):
    h = np.asarray(h, dtype=np.float64)
    if not np.all(h == h[0]):
        raise ValueError("a transformed axis must be uniformly spaced (Sec. 2.1)")
    return float(h[0])


def tridiagonal_stage(fhat, s, hs, bcs, lam1, lam2, t1, t2, singular):
    """Step 2: for every column along axis ``s`` solve
    (lam1_i + lam2_j) x_k + (A_s x)_k = fhat_k, where lam1/lam2 are the
    eigenvalues of the two transformed axes already divided by their spacing
    squared (Eq. (poi_reduced)).  The zero-wavenumber column of a singular
    problem gets the pinned solve and the zero weighted mean (gauge)."""
    a, b, c, periodic = td.coefficients(hs, bcs)
    ax_s = AXIS[s]
    # bring the array to (n_s, n_t1, n_t2) so every column is a trailing index
    order = (ax_s, AXIS[t1], AXIS[t2])
    g = np.transpose(np.asarray(fhat, dtype=np.float64), order)
    ns, n1, n2 = g.shape
    shift = lam1[:, None] + lam2[None, :]               # (n1, n2)
    diag = b[:, None, None] + shift[None, :, :]         # (ns, n1, n2)
    d = g.reshape(ns, n1 * n2)
    diag = diag.reshape(ns, n1 * n2)
    x = np.empty_like(d)
    # wavenumber zero is storage index 0 for both P and NN (Table 1), so the
    # null-space column of a singular problem is column 0
    first = 1 if singular else 0
    if d.shape[1] > first:
        x[:, first:] = td.solve_columns(a, diag[:, first:], c, periodic, d[:, first:])
    if singular:
        x[:, 0] = td.solve_pinned(a, b, c, periodic, d[:, 0], hs)
    x = x.reshape(ns, n1, n2)
    inv = np.argsort(order)
    return np.ascontiguousarray(np.transpose(x, inv))


def solve(f, hx, hy, hz, bcx, bcy, bcz, roles=("x", "y", "z"), shift=0.0):
    """Phi with A Phi = f (f projected onto the range of A when A is
    singular; then Phi has zero volume-weighted mean).

    ``hx``, ``hy``, ``hz`` are the cell widths along each axis (arrays);
    ``roles`` = (t1, t2, s) names the two transformed axes, in the order they
    are transformed, and the Gauss-elimination axis.  Any role assignment
    gives the same Phi up to rounding, as long as t1 and t2 are uniform.

    ``shift`` (<= 0) solves the Helmholtz equation (A + shift) Phi = f of an
    implicit diffusion step instead (Sec. 2); it joins the eigenvalue shift
    of every reduced system.  Node pairs (DDn, NNn) are the non-staggered
    transforms such steps need (Sec. 2.1); a singular problem with a node
    pair has no volume-weighted gauge here and is refused."""
    f = np.asarray(f, dtype=np.float64)
    t1, t2, s = roles
    h = {"x": np.asarray(hx, float), "y": np.asarray(hy, float), "z": np.asarray(hz, float)}
    bc = {"x": bcx, "y": bcy, "z": bcz}
    singular = is_singular(bcx, bcy, bcz, shift)
    if singular and any(k in td.NODE_KINDS for k in (bcx, bcy, bcz)):
        raise ValueError("a singular problem with a node boundary pair is not supported")
    if singular:                                        # compatibility (projection)
        f = f - weighted_mean(f, hx, hy, hz)
    d1 = _uniform_spacing(h[t1])
    d2 = _uniform_spacing(h[t2])
    # step 1: forward transforms, t1 then t2
    g = tr.forward(f, AXIS[t1], bc[t1])
    g = tr.forward(g, AXIS[t2], bc[t2])
    # step 2: tridiagonal systems along s
    lam1 = tr.eigenvalues(bc[t1], f.shape[AXIS[t1]]) / d1 ** 2 + shift
    lam2 = tr.eigenvalues(bc[t2], f.shape[AXIS[t2]]) / d2 ** 2
    g = tridiagonal_stage(g, s, h[s], bc[s], lam1, lam2, t1, t2, singular)
    # step 3: backward transforms, t2 then t1
    g = tr.backward(g, AXIS[t2], bc[t2])
    g = tr.backward(g, AXIS[t1], bc[t1])
    return g


def solve_corrected(f, hx, hy, hz, bcx, bcy, bcz, roles=("x", "y", "z"), phi=None, shift=0.0):
    """``solve`` followed by one correction with its own FP64 residual:
    Phi1 = solve(f), Phi = Phi1 + solve(f - A Phi1).

    The direct method meets Eq. (poi) to rounding (Sec. 2.1), but the
    rounding of its steps reaches the solution through the near-singular
    lowest-wavenumber systems (condition near 1e5 for 512 cells), which
    leaves relative errors that grow like n^2: about 2e-13 at 256^3 and
    7e-13 at 512^3 for random right-hand sides.  The FP64 residual of Phi1
    is white rounding noise of size u |A| |Phi1|, which the inverse damps
    almost entirely, so after one correction the error is at the level of
    u (the correction itself carries the solve's relative error on a
    quantity 1e-13 times smaller).  The result is the plain definition of
    the solve (A Phi = f, gauge as in ``solve``) computed more exactly, for
    comparisons at the largest sizes.  ``phi``: the plain solve of the same
    problem (with the same roles), if already computed."""
    if phi is None:
        phi = solve(f, hx, hy, hz, bcx, bcy, bcz, roles=roles, shift=shift)
    r = residual(f, phi, hx, hy, hz, bcx, bcy, bcz, shift)
    return phi + solve(r, hx, hy, hz, bcx, bcy, bcz, roles=roles, shift=shift)
