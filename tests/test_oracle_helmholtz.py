"""Pins for the oracle's Helmholtz solves with non-staggered (node) pairs:
the implicit-diffusion equations of Sec. 2, (A + shift) Phi = f, with the
DST-I / DCT-I transforms Sec. 2.1 says they need.

* The node transforms equal scipy's unnormalised DST-I and DCT-I, and the
  backward ones invert them.
* Their eigenvalues equal the spectrum of the dense node-rule matrices, and
  each transform row is a left eigenvector of its matrix with the eigenvalue
  of the same index (pins the pairing).
* Whole solves equal a dense solve of the assembled (A + shift) on small
  grids, node pairs on every axis, staggered pairs beside them, uniform and
  (staggered z only) stretched.
* A singular problem with a node pair is refused.
"""
import itertools

import numpy as np
import pytest
import scipy.fft

import oracle
from oracle import poisson as ps
from oracle import transforms as tr
from oracle import tridiagonal as td
from paper_1802_10323_amd.inputs import tanh_widths, uniform_widths

ALL = ("P", "NN", "DD", "ND", "DN", "DDn", "NNn")


@pytest.mark.parametrize("n", [2, 3, 5, 8, 15, 31, 64])
def test_node_transforms_are_dst1_and_dct1(n):
    rng = np.random.default_rng(n)
    a = rng.uniform(-1, 1, n)
    assert np.allclose(tr.forward_matrix("DDn", n) @ a, scipy.fft.dst(a, type=1), rtol=0, atol=1e-13)
    assert np.allclose(tr.forward_matrix("NNn", n) @ a, scipy.fft.dct(a, type=1), rtol=0, atol=1e-13)
    for kind in ("DDn", "NNn"):
        B = tr.backward_matrix(kind, n)
        assert np.allclose(B @ (tr.forward_matrix(kind, n) @ a), a, rtol=0, atol=1e-13)


def node_matrix(kind, n, h=1.0):
    a, b, c, _ = td.coefficients(np.full(n, h), kind)
    return np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)


@pytest.mark.parametrize("kind", ["DDn", "NNn"])
@pytest.mark.parametrize("n", [2, 4, 7, 16, 33])
def test_node_eigenvalues_and_diagonalisation(kind, n):
    A = node_matrix(kind, n)
    lam = tr.eigenvalues(kind, n)
    ev = np.sort(np.linalg.eigvals(A).real)
    assert np.allclose(np.sort(lam), ev, rtol=0, atol=1e-12)
    F = tr.forward_matrix(kind, n)
    assert np.allclose(F @ A, lam[:, None] * F, rtol=0, atol=1e-11)


def test_node_rows_closed_form():
    """DDn rows are the plain second difference with zero beyond the ends;
    NNn end rows are 2 (x_1 - x_0) / h^2 (mirrored neighbour)."""
    h = 0.25
    x = np.array([1.0, 3.0, 2.0, 5.0])
    A = node_matrix("DDn", 4, h)
    ref = np.array([(0 - 2 * 1 + 3), (1 - 6 + 2), (3 - 4 + 5), (2 - 10 + 0)]) / h ** 2
    assert np.allclose(A @ x, ref)
    A = node_matrix("NNn", 4, h)
    ref = np.array([2 * (3 - 1), (1 - 6 + 2), (3 - 4 + 5), 2 * (2 - 5)]) / h ** 2
    assert np.allclose(A @ x, ref)


def dense_helmholtz(hx, hy, hz, bcs, shift):
    mats = []
    for h, k in zip((hx, hy, hz), bcs):
        a, b, c, periodic = td.coefficients(h, k)
        n = len(h)
        M = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
        if periodic and n > 1:
            M[0, n - 1] += a[0]
            M[n - 1, 0] += c[n - 1]
        mats.append(M)
    Mx, My, Mz = mats
    nx, ny, nz = len(hx), len(hy), len(hz)
    I = np.eye
    return (np.kron(I(nz), np.kron(I(ny), Mx)) + np.kron(I(nz), np.kron(My, I(nx)))
            + np.kron(Mz, np.kron(I(ny), I(nx))) + shift * I(nx * ny * nz))


@pytest.mark.parametrize("shift", [-3.7, -250.0])
def test_helmholtz_solve_equals_dense(shift):
    rng = np.random.default_rng(11)
    worst = 0.0
    for t, bcs in enumerate(itertools.product(ALL, repeat=3)):
        if not any(k in ("DDn", "NNn") for k in bcs) and t % 5:
            continue    # the staggered-only triples are pinned elsewhere; keep a sample
        nx, ny, nz = 6, 4, 5
        stretched = bcs[2] not in ("P", "DDn", "NNn") and t % 2 == 0
        hx, hy = uniform_widths(nx, 1.0), uniform_widths(ny, 0.5)
        hz = tanh_widths(nz, 1.0, 1.8) if stretched else uniform_widths(nz, 1.0)
        f = rng.uniform(-1, 1, (nz, ny, nx))
        got = oracle.solve(f, hx, hy, hz, *bcs, shift=shift)
        ref = np.linalg.solve(dense_helmholtz(hx, hy, hz, bcs, shift), f.reshape(-1)).reshape(f.shape)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        worst = max(worst, err)
        assert err <= 1e-13, (bcs, shift, err)
        r = ps.residual(f, got, hx, hy, hz, *bcs, shift=shift)
        assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(f)


def test_non_singular_node_problem_without_shift():
    rng = np.random.default_rng(12)
    hx, hy, hz = uniform_widths(6), uniform_widths(4), uniform_widths(4)
    for bcs in (("DDn", "P", "NN"), ("NNn", "DD", "P"), ("DDn", "NNn", "DDn")):
        f = rng.uniform(-1, 1, (4, 4, 6))
        got = oracle.solve(f, hx, hy, hz, *bcs)
        ref = np.linalg.solve(dense_helmholtz(hx, hy, hz, bcs, 0.0), f.reshape(-1)).reshape(f.shape)
        assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref), bcs


def test_singular_node_problem_refused():
    f = np.zeros((4, 4, 4))
    h = uniform_widths(4)
    with pytest.raises(ValueError):
        oracle.solve(f, h, h, h, "NNn", "P", "NN")
    assert not ps.is_singular("NNn", "P", "NN", shift=-1.0)
