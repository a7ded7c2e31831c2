"""CPU checks of the channel's manufactured solution (tests/channel_modes.py)
and of the oracle against it: the z eigenvectors satisfy A x = mu x for the
oracle's stretched rows, the smallest eigenvalue is the null space (0), and
the oracle's solve of the manufactured right-hand side is its exact
solution (Sec. 2.1)."""
import numpy as np

import oracle
from channel_modes import manufactured_channel, z_eigenpairs
from oracle import tridiagonal as td
from paper_1802_10323_amd import inputs


def test_z_eigenvectors_of_the_stretched_operator():
    hz = inputs.tanh_widths(48, 2.0, 1.8)
    mu, X = z_eigenpairs(hz)
    a, b, c, _ = td.coefficients(hz, "NN")
    A = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
    assert np.allclose(A @ X, X * mu[None, :], rtol=0, atol=1e-9 * np.abs(mu).max())
    assert abs(mu[0]) <= 1e-10 * np.abs(mu).max()
    assert np.allclose(X[:, 0], X[0, 0])              # the null vector is the constant
    # eigenvectors are orthogonal in the cell-width inner product
    G = X.T @ (hz[:, None] * X)
    assert np.allclose(G, np.eye(48), atol=1e-12)


def test_oracle_solves_the_manufactured_channel():
    prob, exact = manufactured_channel(seed=3, nx=32, ny=16, nz=24, modes=20)
    phi = oracle.solve(prob.rhs, prob.hx, prob.hy, prob.hz, *prob.bcs)
    err = np.linalg.norm(phi - exact) / np.linalg.norm(exact)
    assert err <= 1e-12, err
