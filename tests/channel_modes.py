"""Manufactured solutions on the channel grid from discrete eigenmodes
(test infrastructure: built from the oracle's operator rows).

The stretched Neumann-Neumann z operator of the solve, A = D^-1 S (D the
cell widths, S the symmetric matrix of face fluxes), is similar to the
symmetric tridiagonal D^1/2 A D^-1/2, whose eigenpairs scipy's
eigh_tridiagonal gives; x = D^-1/2 y are then eigenvectors of A.  A mode
(Fourier x) (Fourier y) (eigenvector s in z) is an eigenfunction of the
seven-point operator with eigenvalue lambda_x + lambda_y + mu_s, so a
right-hand side made of such modes has the exact discrete solution
sum c_m / (lambda_x + lambda_y + mu_s) mode_m (Sec. 2.1; Table 1 for the
Fourier eigenvalues 2 (cos(2 pi k / n) - 1) / h^2)."""
import math

import numpy as np
import scipy.linalg

from oracle import tridiagonal as td
from paper_1802_10323_amd import inputs


def z_eigenpairs(hz, kind="NN"):
    """(mu, X): eigenvalues of the 1D operator along a stretched axis, from
    0 (the constant) downward, and its eigenvectors (columns), so that the
    profile index grows with the wavenumber as the cosines' does."""
    h = np.asarray(hz, dtype=np.float64)
    a, b, c, periodic = td.coefficients(h, kind)
    assert not periodic
    off = c[:-1] * np.sqrt(h[:-1] / h[1:])
    mu, y = scipy.linalg.eigh_tridiagonal(b, off)
    mu, y = mu[::-1], y[:, ::-1]
    return mu, y / np.sqrt(h)[:, None]


def manufactured_channel(seed=0, nx=512, ny=256, nz=192, modes=64):
    """(problem, exact solution): the channel grid and modes of the
    benchmark's channel generator, z profiles replaced by the discrete
    eigenvectors, no noise."""
    hz = inputs.tanh_widths(nz, 2.0, 1.8)
    mu, X = z_eigenpairs(hz)
    drawn = []
    prob = inputs.channel(seed, nx, ny, nz, modes, noise=0.0, z_profiles=lambda s: X[:, s],
                          drawn=drawn)
    dx, dy = 4.0 * math.pi / nx, 2.0 * math.pi / ny
    xc, yc = inputs.centres(prob.hx), inputs.centres(prob.hy)
    phi = np.zeros((nz, ny * nx))
    for kx, ky, kz, px, py, amp in drawn:
        lam = (2.0 * (math.cos(2.0 * math.pi * kx / nx) - 1.0) / dx ** 2
               + 2.0 * (math.cos(2.0 * math.pi * ky / ny) - 1.0) / dy ** 2 + mu[kz])
        if kx == 0 and ky == 0 and kz == 0:
            continue                       # the constant: removed with the mean
        fx = np.cos(2.0 * math.pi * kx * xc / (4.0 * math.pi) - px)
        fy = np.cos(2.0 * math.pi * ky * yc / (2.0 * math.pi) - py)
        phi += np.outer(amp / lam * X[:, kz], np.outer(fy, fx).reshape(-1))
    return prob, phi.reshape(nz, ny, nx)
