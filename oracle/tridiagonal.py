"""Oracle: the second-order operator along one axis of a staggered,
cell-centred grid and the Gauss elimination of the reduced tridiagonal
systems (Sec. 2.1, Eq. (poi_reduced); Sec. 3 for the cyclic case).

Test infrastructure only (see ``oracle/__init__.py``).

Readings of the paper used here (each listed in the design notes):

* Non-uniform spacing (Sec. 2.1 footnote: the solver allows a non-uniform
  grid in the Gauss-elimination direction; the paper gives no formula).  The
  finite-volume form is used: with cell widths h_k and centre distances
  dc_k = (h_{k-1} + h_k)/2, row k reads
  a_k x_{k-1} + b_k x_k + c_k x_{k+1} with a_k = 1/(h_k dc_k),
  c_k = 1/(h_k dc_{k+1}), b_k = -(a_k + c_k).  At a wall the ghost cell is the
  mirror image of the edge cell (dc_0 = h_0, dc_n = h_{n-1}); across a periodic
  wrap dc_0 = dc_n = (h_{n-1} + h_0)/2.  With uniform h this is exactly the
  central difference of Eq. (poi).
* Staggered boundary conditions (Table 1 caption): a Neumann face sets the
  ghost value equal to the edge value, a Dirichlet face sets it to minus the
  edge value (the face value, their mean, is zero).  The first letter of a
  pair is the low face (index 0), the second the high face (index n-1).
* Pivoting: the paper calls LAPACK's partial-pivoting routine.  The reduced
  systems are weakly diagonally dominant (every eigenvalue of Table 1 is
  <= 0), so elimination without pivoting is used; it differs from the pivoted
  one only by rounding.
* Periodic solve axis (Sec. 3: the cyclic system is reduced to two
  tridiagonal problems): Sherman-Morrison with gamma = -b_0.
* Singular column (every axis periodic or Neumann-Neumann; the paper is
  silent): the last equation of the zero-wavenumber column is dropped and its
  unknown set to zero, the remaining system is solved, and the volume-weighted
  mean is then subtracted.
* Non-staggered (node) pairs, uniform spacing h only: DDn, the neighbours
  beyond the two ends are boundary nodes with value zero (no ghost term);
  NNn, the neighbour beyond an end node mirrors the node next to it
  (x_{-1} = x_1), so the end rows read 2 (x_1 - x_0) / h^2.
"""
import numpy as np

LOW = {"P": "P", "NN": "N", "DD": "D", "ND": "N", "DN": "D"}
HIGH = {"P": "P", "NN": "N", "DD": "D", "ND": "D", "DN": "N"}
NODE_KINDS = ("DDn", "NNn")


def coefficients(h, kind):
    """Rows (a, b, c) of the 1D operator for cell widths ``h`` and boundary
    pair ``kind``.  Returns a, b, c (each length n) and a flag ``periodic``.
    For a periodic axis a[0] couples x_0 to x_{n-1} and c[n-1] couples x_{n-1}
    to x_0; otherwise a[0] = c[n-1] = 0 and the ghost rule is folded into b."""
    h = np.asarray(h, dtype=np.float64)
    n = h.size
    if kind in NODE_KINDS:
        if not np.all(h == h[0]):
            raise ValueError("node boundary pairs need a uniform spacing")
        inv = 1.0 / (h[0] * h[0])
        a = np.full(n, inv)
        c = np.full(n, inv)
        b = np.full(n, -2.0 * inv)
        a[0] = 0.0
        c[n - 1] = 0.0
        if kind == "NNn" and n > 1:   # mirrored neighbours beyond the end nodes
            c[0] = 2.0 * inv
            a[n - 1] = 2.0 * inv
        return a, b, c, False
    periodic = kind == "P"
    dc = np.empty(n + 1)
    dc[1:n] = 0.5 * (h[:-1] + h[1:])
    if periodic:
        dc[0] = dc[n] = 0.5 * (h[-1] + h[0])
    else:
        dc[0] = h[0]
        dc[n] = h[-1]
    a = 1.0 / (h * dc[:n])
    c = 1.0 / (h * dc[1:])
    b = -(a + c)
    if not periodic:
        b[0] += a[0] if LOW[kind] == "N" else -a[0]
        b[n - 1] += c[n - 1] if HIGH[kind] == "N" else -c[n - 1]
        a = a.copy()
        c = c.copy()
        a[0] = 0.0
        c[n - 1] = 0.0
    return a, b, c, periodic


def thomas(a, b, c, d):
    """Gauss elimination without pivoting of
    a_k x_{k-1} + b_k x_k + c_k x_{k+1} = d_k, k = 0 .. n-1
    for many right-hand sides at once.  ``a`` and ``c`` have shape (n,) and
    a[0], c[n-1] are ignored; ``b`` and ``d`` have shape (n, ncol)."""
    n = d.shape[0]
    b = np.broadcast_to(b, d.shape)
    cp = np.empty_like(d)
    dp = np.empty_like(d)
    beta = b[0].copy()
    cp[0] = c[0] / beta if n > 1 else 0.0
    dp[0] = d[0] / beta
    for k in range(1, n):
        beta = b[k] - a[k] * cp[k - 1]
        cp[k] = c[k] / beta if k < n - 1 else 0.0
        dp[k] = (d[k] - a[k] * dp[k - 1]) / beta
    x = np.empty_like(d)
    x[n - 1] = dp[n - 1]
    for k in range(n - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


def cyclic_thomas(a, b, c, d):
    """Periodic tridiagonal system (a[0] couples to x_{n-1}, c[n-1] to x_0),
    reduced to two non-periodic solves by Sherman-Morrison, gamma = -b_0."""
    n = d.shape[0]
    if n < 3:
        raise ValueError("a periodic solve axis needs at least 3 cells")
    b = np.array(np.broadcast_to(b, d.shape), dtype=np.float64)
    alpha = a[0]          # row 0, column n-1
    beta_ = c[n - 1]      # row n-1, column 0
    gamma = -b[0]
    bb = b.copy()
    bb[0] = b[0] - gamma
    bb[n - 1] = b[n - 1] - alpha * beta_ / gamma
    y = thomas(a, bb, c, d)
    u = np.zeros_like(d)
    u[0] = gamma
    u[n - 1] = beta_
    z = thomas(a, bb, c, u)
    vy = y[0] + (alpha / gamma) * y[n - 1]
    vz = z[0] + (alpha / gamma) * z[n - 1]
    return y - (vy / (1.0 + vz)) * z


def solve_columns(a, b, c, periodic, d):
    """Dispatch to the plain or the cyclic elimination."""
    if periodic:
        return cyclic_thomas(a, b, c, d)
    return thomas(a, b, c, d)


def solve_pinned(a, b, c, periodic, d, weights):
    """The zero-wavenumber column of a singular problem: drop the last
    equation, set x_{n-1} = 0, solve the remaining (n-1) rows (plain
    tridiagonal also for a periodic axis, since the wrap couplings all involve
    x_{n-1}), then remove the mean weighted by ``weights`` (cell widths)."""
    n = d.shape[0]
    x = np.zeros_like(d)
    if n > 1:
        bb = np.broadcast_to(b, d.shape)[: n - 1]
        x[: n - 1] = thomas(a[: n - 1], bb, c[: n - 1], d[: n - 1])
    w = np.asarray(weights, dtype=np.float64).reshape((n,) + (1,) * (d.ndim - 1))
    return x - (w * x).sum(axis=0) / w.sum()
