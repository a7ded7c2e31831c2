"""Pins for the oracle's Table 1 / Table 2 code, against things other than
itself: scipy's and numpy's transforms (the Table 2 sums are exactly their
unnormalised DCT/DST types 2, 3, 4 and the real DFT), exact closed forms, and
eigen-decompositions of one-dimensional operator matrices that these tests
build from the staggered ghost-cell rules."""
import math
import os

import numpy as np
import pytest
import scipy.fft as sf

from oracle import transforms as tr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SIZES = [2, 4, 6, 8, 10, 12, 16, 30, 32, 48]
ODD = [1, 3, 5, 7, 9, 15]


def interleaved_rfft(a):
    """Table 2's DFT storage from numpy's rfft (sine sums = -Im)."""
    n = a.size
    m = n // 2
    X = np.fft.rfft(a)
    A = np.empty(n)
    A[0] = X[0].real
    A[n - 1] = X[m].real
    for l in range(1, m):
        A[2 * l - 1] = X[l].real
        A[2 * l] = -X[l].imag
    return A


def deinterleave_irfft(A):
    n = A.size
    m = n // 2
    X = np.zeros(m + 1, dtype=complex)
    X[0] = A[0]
    X[m] = A[n - 1]
    for l in range(1, m):
        X[l] = A[2 * l - 1] - 1j * A[2 * l]
    return np.fft.irfft(X, n)


LIB_FORWARD = {
    "NN": lambda a: sf.dct(a, 2),
    "DD": lambda a: sf.dst(a, 2),
    "ND": lambda a: sf.dct(a, 4),
    "DN": lambda a: sf.dst(a, 4),
}
LIB_BACKWARD = {
    "NN": lambda A: sf.dct(A, 3) / (2 * A.size),
    "DD": lambda A: sf.dst(A, 3) / (2 * A.size),
    "ND": lambda A: sf.dct(A, 4) / (2 * A.size),
    "DN": lambda A: sf.dst(A, 4) / (2 * A.size),
}


@pytest.mark.parametrize("n", SIZES + ODD)
@pytest.mark.parametrize("kind", ["NN", "DD", "ND", "DN"])
def test_forward_equals_library(kind, n):
    a = np.random.default_rng(n).uniform(-1, 1, n)
    np.testing.assert_allclose(tr.forward_matrix(kind, n) @ a, LIB_FORWARD[kind](a),
                               rtol=0, atol=1e-13 * n)


@pytest.mark.parametrize("n", SIZES + ODD)
@pytest.mark.parametrize("kind", ["NN", "DD", "ND", "DN"])
def test_backward_equals_library(kind, n):
    A = np.random.default_rng(100 + n).uniform(-1, 1, n)
    np.testing.assert_allclose(tr.backward_matrix(kind, n) @ A, LIB_BACKWARD[kind](A),
                               rtol=0, atol=1e-14 * n)


@pytest.mark.parametrize("n", SIZES)
def test_dft_equals_numpy_rfft(n):
    a = np.random.default_rng(7 * n).uniform(-1, 1, n)
    np.testing.assert_allclose(tr.forward_matrix("P", n) @ a, interleaved_rfft(a),
                               rtol=0, atol=1e-13 * n)
    A = np.random.default_rng(9 * n).uniform(-1, 1, n)
    np.testing.assert_allclose(tr.backward_matrix("P", n) @ A, deinterleave_irfft(A),
                               rtol=0, atol=1e-14 * n)


def test_periodic_needs_even_n():
    with pytest.raises(ValueError):
        tr.forward_matrix("P", 7)
    with pytest.raises(ValueError):
        tr.eigenvalues("P", 5)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("kind", tr.KINDS)
def test_round_trip_is_identity(kind, n):
    I = tr.backward_matrix(kind, n) @ tr.forward_matrix(kind, n)
    np.testing.assert_allclose(I, np.eye(n), rtol=0, atol=1e-13)


def operator_1d(kind, n):
    """Dense 1D second-difference matrix on n unit cells, built here from the
    staggered ghost rules: periodic wraps; a Neumann face copies the edge
    value into the ghost; a Dirichlet face puts minus the edge value there."""
    A = np.zeros((n, n))
    for p in range(n):
        A[p, p] -= 2.0
        for q in (p - 1, p + 1):
            if 0 <= q < n:
                A[p, q] += 1.0
            elif kind == "P":
                A[p, q % n] += 1.0
            else:
                face = kind[0] if q < 0 else kind[1]
                A[p, p] += 1.0 if face == "N" else -1.0
    return A


@pytest.mark.parametrize("n", [4, 6, 8, 16, 18, 32])
@pytest.mark.parametrize("kind", tr.KINDS)
def test_eigenvalues_are_operator_spectrum(kind, n):
    lam = np.sort(tr.eigenvalues(kind, n))
    ref = np.sort(np.linalg.eigvalsh(operator_1d(kind, n)))
    np.testing.assert_allclose(lam, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("n", [4, 6, 8, 12, 16, 32])
@pytest.mark.parametrize("kind", tr.KINDS)
def test_transform_diagonalises_operator(kind, n):
    """F A = diag(lambda) F: row q of the forward transform is a left
    eigenvector with eigenvalue lambda_q, which pins the pairing between the
    storage order of Table 2 and the angles of Table 1."""
    T = tr.forward_matrix(kind, n)
    A = operator_1d(kind, n)
    lam = tr.eigenvalues(kind, n)
    np.testing.assert_allclose(T @ A, lam[:, None] * T, rtol=0, atol=1e-12 * n)


def test_eigenvalues_golden_closed_forms():
    r2 = math.sqrt(2.0)
    basis = (1.0, r2, math.sqrt(2.0 + r2), math.sqrt(2.0 - r2))
    rows = {}
    with open(os.path.join(GOLDEN, "table1_eigenvalues_n4.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            kind, q, *coef = line.split()
            rows.setdefault(kind, {})[int(q)] = sum(int(c) * b for c, b in zip(coef, basis))
    assert set(rows) == set(tr.KINDS)
    for kind, vals in rows.items():
        exp = np.array([vals[q] for q in range(4)])
        np.testing.assert_allclose(tr.eigenvalues(kind, 4), exp, rtol=0, atol=1e-15)


@pytest.mark.parametrize("kind", tr.KINDS)
def test_apply_along_every_axis(kind):
    f = np.random.default_rng(3).uniform(-1, 1, (4, 6, 8))
    for axis in range(3):
        n = f.shape[axis]
        T = tr.forward_matrix(kind, n)
        ref = np.einsum("qp,...p->...q", T, np.moveaxis(f, axis, -1))
        np.testing.assert_allclose(tr.forward(f, axis, kind), np.moveaxis(ref, -1, axis),
                                   rtol=0, atol=1e-13)
        np.testing.assert_allclose(tr.backward(tr.forward(f, axis, kind), axis, kind), f,
                                   rtol=0, atol=1e-13)
