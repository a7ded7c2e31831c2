"""Pins for the oracle's elimination code: LAPACK's dgtsv (the routine the
paper names for the reduced systems, Sec. 3), dense solves, and the
null-vector property of the staggered operator."""
import numpy as np
import pytest
from scipy.linalg import lapack

from oracle import tridiagonal as td
from paper_1802_10323_amd.inputs import tanh_widths, uniform_widths


def random_system(n, ncol, seed, shift=0.0):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 1.5, n)
    c = rng.uniform(0.5, 1.5, n)
    b = -(a + c)[:, None] - rng.uniform(0.0, 1.0, (n, ncol)) - shift
    d = rng.uniform(-1, 1, (n, ncol))
    return a, b, c, d


@pytest.mark.parametrize("n", [1, 2, 3, 8, 17, 64])
def test_thomas_equals_dgtsv(n):
    a, b, c, d = random_system(n, 5, n)
    x = td.thomas(a, b, c, d)
    if n == 1:                       # the LAPACK wrapper needs n >= 2
        np.testing.assert_allclose(x, d / b, rtol=1e-15)
        return
    for j in range(d.shape[1]):
        _, _, _, ref, info = lapack.dgtsv(a[1:].copy(), b[:, j].copy(), c[:-1].copy(),
                                          d[:, j].copy())
        assert info == 0
        np.testing.assert_allclose(x[:, j], ref, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("kind", ["NN", "DD", "ND", "DN"])
@pytest.mark.parametrize("stretched", [False, True])
def test_poisson_rows_equal_dgtsv(kind, stretched):
    """The actual reduced rows of Eq. (poi_reduced): operator rows plus a
    non-positive eigenvalue shift per column."""
    n = 40
    h = tanh_widths(n, 2.0, 1.8) if stretched else uniform_widths(n, 2.0)
    a, b, c, periodic = td.coefficients(h, kind)
    shifts = -np.array([1e-3, 0.5, 10.0, 1e4])
    bb = b[:, None] + shifts[None, :]
    d = np.random.default_rng(5).uniform(-1, 1, (n, shifts.size))
    x = td.thomas(a, bb, c, d)
    for j in range(shifts.size):
        _, _, _, ref, info = lapack.dgtsv(a[1:].copy(), bb[:, j].copy(), c[:-1].copy(),
                                          d[:, j].copy())
        assert info == 0
        np.testing.assert_allclose(x[:, j], ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())


def dense_from_rows(a, b, c, periodic):
    n = b.size
    A = np.diag(b).astype(float)
    for k in range(n):
        if k > 0:
            A[k, k - 1] += a[k]
        elif periodic:
            A[k, n - 1] += a[k]
        if k < n - 1:
            A[k, k + 1] += c[k]
        elif periodic:
            A[k, 0] += c[k]
    return A


@pytest.mark.parametrize("n", [3, 4, 9, 32])
@pytest.mark.parametrize("stretched", [False, True])
def test_cyclic_equals_dense(n, stretched):
    h = tanh_widths(n, 1.0, 1.8) if stretched else uniform_widths(n, 1.0)
    a, b, c, periodic = td.coefficients(h, "P")
    assert periodic
    for shift in (-1e-2, -3.0, -1e3):
        d = np.random.default_rng(n).uniform(-1, 1, (n, 2))
        x = td.cyclic_thomas(a, (b + shift)[:, None], c, d)
        ref = np.linalg.solve(dense_from_rows(a, b + shift, c, True), d)
        np.testing.assert_allclose(x, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("kind", ["P", "NN"])
@pytest.mark.parametrize("stretched", [False, True])
def test_width_weighted_columns_vanish(kind, stretched):
    """h^T A = 0 for the singular one-dimensional operators: the cell widths
    are the left null vector (so the weighted mean is the compatibility
    condition); the unweighted column sums do not vanish on a stretched grid."""
    n = 24
    h = tanh_widths(n, 2.0, 1.8) if stretched else uniform_widths(n, 2.0)
    a, b, c, periodic = td.coefficients(h, kind)
    A = dense_from_rows(a, b, c, periodic)
    scale = np.abs(A).max()
    assert np.abs(h @ A).max() < 1e-13 * scale
    np.testing.assert_allclose(A @ np.ones(n), 0.0, atol=1e-12 * scale)
    if stretched:
        assert np.abs(np.ones(n) @ A).max() > 1e-3 * scale


def test_uniform_rows_are_central_differences():
    h = uniform_widths(6, 3.0)          # h = 0.5
    for kind, lo, hi in (("NN", -1, -1), ("DD", -3, -3), ("ND", -1, -3), ("DN", -3, -1)):
        a, b, c, periodic = td.coefficients(h, kind)
        assert not periodic
        np.testing.assert_allclose(b * 0.25, [lo, -2, -2, -2, -2, hi])
        np.testing.assert_allclose(a * 0.25, [0, 1, 1, 1, 1, 1])
        np.testing.assert_allclose(c * 0.25, [1, 1, 1, 1, 1, 0])
    a, b, c, periodic = td.coefficients(h, "P")
    assert periodic
    np.testing.assert_allclose(a * 0.25, 1)
    np.testing.assert_allclose(b * 0.25, -2)
    np.testing.assert_allclose(c * 0.25, 1)


@pytest.mark.parametrize("kind", ["P", "NN"])
@pytest.mark.parametrize("stretched", [False, True])
def test_pinned_solve_solves_singular_system(kind, stretched):
    n = 20
    h = tanh_widths(n, 2.0, 1.8) if stretched else uniform_widths(n, 2.0)
    a, b, c, periodic = td.coefficients(h, kind)
    A = dense_from_rows(a, b, c, periodic)
    d = np.random.default_rng(1).uniform(-1, 1, n)
    d -= (h @ d) / h.sum()                      # compatible right-hand side
    x = td.solve_pinned(a, b, c, periodic, d, h)
    np.testing.assert_allclose(A @ x, d, atol=1e-11 * np.abs(d).max())
    assert abs(h @ x) < 1e-13 * h.sum() * np.abs(x).max()
    # the solution is unique in the gauge: compare with the bordered dense system
    M = np.zeros((n + 1, n + 1))
    M[:n, :n] = A
    M[:n, n] = 1.0 / np.sqrt(n)
    M[n, :n] = h
    ref = np.linalg.solve(M, np.concatenate([d, [0.0]]))[:n]
    np.testing.assert_allclose(x, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
