"""Pins for the oracle's whole solve and its seven-point operator.

* exact rational Gauss elimination of Eq. (poi) (built here, in Fractions)
  on tiny grids, including stretched and periodic solve axes;
* dense solves of the operator on 8^3 grids for all 125 boundary triples,
  uniform and stretched z (the direct method must reach the plain linear
  solution to round-off);
* closed-form discrete eigenfunctions (manufactured solutions exact to
  round-off);
* consistency (at least first order, pointwise) of the stretched operator with the continuous
  Laplacian;
* invariants: residual, zero weighted mean, role independence, axis
  reversal (N-D <-> D-N), linearity.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import poisson as op
from paper_1802_10323_amd.inputs import tanh_widths, uniform_widths

KINDS = ("P", "NN", "DD", "ND", "DN")


# ---------------------------------------------------------------- exact

def exact_operator_rows(h, kind):
    """Rows of the 1D staggered operator in exact arithmetic, written from
    the finite-volume reading: flux through each face divided by the cell
    width; centre distances are the mean of the two widths; a wall face sees
    a mirrored ghost cell (N: same value, D: opposite value)."""
    n = len(h)
    rows = []
    for k in range(n):
        row = {}
        for side in (-1, +1):
            nb = k + side
            if 0 <= nb < n:
                dist = (h[k] + h[nb]) / 2
                coef = 1 / (h[k] * dist)
                row[nb] = row.get(nb, 0) + coef
                row[k] = row.get(k, 0) - coef
            elif kind == "P":
                nb %= n
                dist = (h[k] + h[nb]) / 2
                coef = 1 / (h[k] * dist)
                row[nb] = row.get(nb, 0) + coef
                row[k] = row.get(k, 0) - coef
            else:
                face = kind[0] if side < 0 else kind[1]
                coef = 1 / (h[k] * h[k])
                row[k] = row.get(k, 0) - coef + (coef if face == "N" else -coef)
        rows.append(row)
    return rows


def exact_solve(f, hx, hy, hz, bcs):
    """Exact Gauss-Jordan elimination in Fractions of the full system (the
    bordered system with the weighted-mean gauge when it is singular)."""
    nz, ny, nx = f.shape
    hs = (hx, hy, hz)
    rows1d = [exact_operator_rows(h, k) for h, k in zip(hs, bcs)]
    N = nx * ny * nz
    idx = lambda i, j, k: i + nx * (j + ny * k)
    A = [[Fraction(0)] * N for _ in range(N)]
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                r = idx(i, j, k)
                for q, v in rows1d[0][i].items():
                    A[r][idx(q, j, k)] += v
                for q, v in rows1d[1][j].items():
                    A[r][idx(i, q, k)] += v
                for q, v in rows1d[2][k].items():
                    A[r][idx(i, j, q)] += v
    rhs = [Fraction(float(f[k, j, i])) for k in range(nz) for j in range(ny) for i in range(nx)]
    singular = all(b in ("P", "NN") for b in bcs)
    w = [hx[i] * hy[j] * hz[k] for k in range(nz) for j in range(ny) for i in range(nx)]
    if singular:
        mean = sum(wi * fi for wi, fi in zip(w, rhs)) / sum(w)
        rhs = [fi - mean for fi in rhs]
        for r in range(N):
            A[r].append(Fraction(1))
        A.append(list(w) + [Fraction(0)])
        rhs.append(Fraction(0))
        N += 1
    M = [A[r] + [rhs[r]] for r in range(N)]
    for col in range(N):
        piv = next(r for r in range(col, N) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        pv = M[col][col]
        M[col] = [v / pv for v in M[col]]
        for r in range(N):
            if r != col and M[r][col] != 0:
                fac = M[r][col]
                M[r] = [vr - fac * vc for vr, vc in zip(M[r], M[col])]
    x = [float(M[r][N]) for r in range(nx * ny * nz)]
    return np.array(x).reshape(nz, ny, nx)


EXACT_CASES = [
    ((4, 2, 3), ("P", "P", "NN"), False),
    ((2, 4, 3), ("NN", "P", "NN"), True),
    ((2, 2, 4), ("DD", "ND", "DN"), True),
    ((4, 2, 3), ("P", "DD", "P"), False),
    ((2, 2, 5), ("NN", "NN", "P"), True),
    ((2, 4, 3), ("DN", "P", "DD"), True),
    ((4, 4, 2), ("ND", "NN", "NN"), False),
]


@pytest.mark.parametrize("shape,bcs,stretched", EXACT_CASES)
def test_solve_equals_exact_rational_elimination(shape, bcs, stretched):
    nx, ny, nz = shape
    hx = [Fraction(1, nx)] * nx
    hy = [Fraction(2, ny)] * ny
    if stretched:
        hz = [Fraction(k + 1, 1) for k in range(nz)]
        tot = sum(hz)
        hz = [v / tot for v in hz]
    else:
        hz = [Fraction(1, nz)] * nz
    f = np.random.default_rng(nx * 100 + ny * 10 + nz).uniform(-1, 1, (nz, ny, nx))
    ref = exact_solve(f, hx, hy, hz, bcs)
    got = oracle.solve(f, np.array(hx, float), np.array(hy, float), np.array(hz, float), *bcs)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


# ---------------------------------------------------------------- dense 8^3

def dense_operator(hx, hy, hz, bcs):
    """Dense N x N operator assembled as a Kronecker sum of 1D matrices built
    from the exact rows above (evaluated in floating point)."""
    mats = []
    for h, kind in zip((hx, hy, hz), bcs):
        rows = exact_operator_rows([Fraction(float(v)) for v in h], kind)
        n = len(h)
        M = np.zeros((n, n))
        for r, row in enumerate(rows):
            for q, v in row.items():
                M[r, q] += float(v)
        mats.append(M)
    Mx, My, Mz = mats
    Ix, Iy, Iz = (np.eye(m.shape[0]) for m in mats)
    # flattened index i + nx*(j + ny*k): kron order (z, y, x)
    return (np.kron(Iz, np.kron(Iy, Mx)) + np.kron(Iz, np.kron(My, Ix))
            + np.kron(Mz, np.kron(Iy, Ix)))


def dense_solve(f, hx, hy, hz, bcs):
    A = dense_operator(hx, hy, hz, bcs)
    b = f.reshape(-1)
    N = b.size
    if all(k in ("P", "NN") for k in bcs):
        w = np.kron(hz, np.kron(hy, hx))
        b = b - (w @ b) / w.sum()
        M = np.zeros((N + 1, N + 1))
        M[:N, :N] = A
        M[:N, N] = 1.0
        M[N, :N] = w
        x = np.linalg.solve(M, np.concatenate([b, [0.0]]))[:N]
    else:
        x = np.linalg.solve(A, b)
    return x.reshape(f.shape)


@pytest.mark.parametrize("stretched", [False, True])
def test_solve_equals_dense_all_125_triples(stretched):
    n = 8
    hx = uniform_widths(n, 1.0)
    hy = uniform_widths(n, 2.0)
    worst = 0.0
    for t, bcs in enumerate(itertools.product(KINDS, repeat=3)):
        hz = tanh_widths(n, 1.5, 1.8) if stretched else uniform_widths(n, 1.5)
        f = np.random.default_rng(t).uniform(-1, 1, (n, n, n))
        ref = dense_solve(f, hx, hy, hz, bcs)
        got = oracle.solve(f, hx, hy, hz, *bcs)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        worst = max(worst, err)
        assert err <= 1e-13, (bcs, err)
    assert worst > 0.0


# ---------------------------------------------------------------- eigenfunctions

def eigvec(kind, n, q):
    """Closed-form eigenvectors of the 1D staggered operator, sampled at the
    cell centres x_p = p + 1/2 (unit cells): cosines/sines whose wavenumber
    makes the ghost rule hold at each face."""
    x = np.arange(n) + 0.5
    if kind == "P":
        l = (q + 1) // 2
        if q == 0:
            return np.ones(n)
        if q == n - 1:
            return np.cos(np.pi * (x - 0.5))
        return np.cos(2 * np.pi * l * x / n) if q % 2 else np.sin(2 * np.pi * l * x / n)
    if kind == "NN":
        return np.cos(np.pi * q * x / n)
    if kind == "DD":
        return np.sin(np.pi * (q + 1) * x / n)
    if kind == "ND":
        return np.cos(np.pi * (q + 0.5) * x / n)
    if kind == "DN":
        return np.sin(np.pi * (q + 0.5) * x / n)


def rayleigh(kind, n, v):
    """Eigenvalue of v for the 1D operator, measured (not from Table 1)."""
    rows = exact_operator_rows([Fraction(1)] * n, kind)
    Av = np.array([sum(float(c) * v[q] for q, c in row.items()) for row in rows])
    return float(v @ Av / (v @ v)), Av


@pytest.mark.parametrize("bcs", [("P", "P", "NN"), ("DD", "ND", "P"), ("NN", "DN", "DD"),
                                 ("P", "NN", "ND"), ("DN", "P", "P")])
def test_manufactured_eigenfunction_solutions(bcs):
    nx, ny, nz = 24, 16, 20
    dx, dy, dz = 0.5, 0.25, 0.1
    rng = np.random.default_rng(11)
    phi = np.zeros((nz, ny, nx))
    f = np.zeros_like(phi)
    for _ in range(6):
        qs = [int(rng.integers(0 if b not in ("P", "NN") else 1, n)) for b, n in
              zip(bcs, (nx, ny, nz))]
        vs, lams = [], []
        for kind, n, q, d in zip(bcs, (nx, ny, nz), qs, (dx, dy, dz)):
            v = eigvec(kind, n, q)
            lam, Av = rayleigh(kind, n, v)
            np.testing.assert_allclose(Av, lam * v, atol=1e-12)     # it is an eigenvector
            vs.append(v)
            lams.append(lam / d ** 2)
        mode = vs[2][:, None, None] * vs[1][None, :, None] * vs[0][None, None, :]
        c = rng.uniform(-1, 1)
        phi += c * mode
        f += c * sum(lams) * mode
    hx, hy, hz = np.full(nx, dx), np.full(ny, dy), np.full(nz, dz)
    got = oracle.solve(f, hx, hy, hz, *bcs)
    assert np.linalg.norm(got - phi) <= 1e-13 * np.linalg.norm(phi)


# ---------------------------------------------------------------- operator

def test_operator_matches_dense_kron():
    rng = np.random.default_rng(2)
    for bcs in [("P", "DD", "NN"), ("ND", "P", "P"), ("DN", "NN", "DD")]:
        hx, hy = uniform_widths(6, 1.0), uniform_widths(4, 3.0)
        hz = tanh_widths(5, 2.0, 1.8)
        phi = rng.uniform(-1, 1, (5, 4, 6))
        A = dense_operator(hx, hy, hz, bcs)
        np.testing.assert_allclose(op.apply_operator(phi, hx, hy, hz, *bcs).reshape(-1),
                                   A @ phi.reshape(-1), rtol=1e-13, atol=1e-12)


def test_stretched_operator_is_consistent():
    """On a tanh grid with Neumann walls the operator applied to cos(pi z/L)
    tends to -(pi/L)^2 cos(pi z/L) as the grid is refined."""
    L = 2.0
    errs = []
    for n in (32, 64, 128, 256):
        hz = tanh_widths(n, L, 1.8)
        zc = np.cumsum(hz) - 0.5 * hz
        phi = np.cos(np.pi * zc / L)[:, None, None] * np.ones((1, 1, 2))
        Aphi = op.apply_operator(phi, np.ones(2), np.ones(1), hz, "P", "NN", "NN")
        errs.append(np.abs(Aphi[:, 0, 0] + (np.pi / L) ** 2 * phi[:, 0, 0]).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(rates) > 0.9, (errs, rates)
    assert errs[-1] < 0.01 * (np.pi / L) ** 2


# ---------------------------------------------------------------- invariants

def test_residual_small_at_moderate_size():
    rng = np.random.default_rng(4)
    for bcs, stretched in ((("P", "P", "NN"), True), (("DD", "ND", "P"), False),
                           (("NN", "NN", "NN"), False), (("P", "P", "P"), True)):
        nx, ny, nz = 48, 40, 36
        hx, hy = uniform_widths(nx, 4 * math.pi), uniform_widths(ny, 2 * math.pi)
        hz = tanh_widths(nz, 2.0, 1.8) if stretched else uniform_widths(nz, 2.0)
        f = rng.uniform(-1, 1, (nz, ny, nx))
        phi = oracle.solve(f, hx, hy, hz, *bcs)
        r = op.residual(f, phi, hx, hy, hz, *bcs)
        assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(f), bcs
        if op.is_singular(*bcs):
            assert abs(op.weighted_mean(phi, hx, hy, hz)) <= 1e-14 * np.abs(phi).max()


def test_roles_do_not_change_the_result():
    rng = np.random.default_rng(6)
    h = {a: uniform_widths(n, 1.0) for a, n in (("x", 12), ("y", 10), ("z", 8))}
    for bcs in [("DD", "ND", "P"), ("P", "P", "NN"), ("NN", "NN", "NN"), ("P", "P", "P")]:
        f = rng.uniform(-1, 1, (8, 10, 12))
        ref = oracle.solve(f, h["x"], h["y"], h["z"], *bcs)
        for roles in [("y", "z", "x"), ("z", "x", "y"), ("y", "x", "z"), ("x", "z", "y")]:
            got = oracle.solve(f, h["x"], h["y"], h["z"], *bcs, roles=roles)
            assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref), (bcs, roles)


def test_axis_reversal_swaps_nd_and_dn():
    rng = np.random.default_rng(8)
    f = rng.uniform(-1, 1, (6, 8, 10))
    hx, hy, hz = uniform_widths(10, 1.0), uniform_widths(8, 1.0), tanh_widths(6, 1.0, 1.8)
    a = oracle.solve(f, hx, hy, hz, "ND", "P", "DD")
    b = oracle.solve(f[:, :, ::-1], hx, hy, hz, "DN", "P", "DD")[:, :, ::-1]
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(a)
    c = oracle.solve(f, hx, hy, hz, "P", "DD", "ND")
    d = oracle.solve(f[::-1], hx, hy, hz[::-1], "P", "DD", "DN")[::-1]
    assert np.linalg.norm(c - d) <= 1e-13 * np.linalg.norm(c)


def test_linearity():
    rng = np.random.default_rng(9)
    h = uniform_widths(8, 1.0)
    f, g = rng.uniform(-1, 1, (2, 8, 8, 8))
    bcs = ("DN", "DD", "NN")
    lhs = oracle.solve(2.5 * f - g, h, h, h, *bcs)
    rhs = 2.5 * oracle.solve(f, h, h, h, *bcs) - oracle.solve(g, h, h, h, *bcs)
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(lhs)


def test_non_uniform_transformed_axis_rejected():
    f = np.zeros((4, 4, 4))
    with pytest.raises(ValueError):
        oracle.solve(f, tanh_widths(4, 1.0, 1.8), uniform_widths(4), uniform_widths(4),
                     "NN", "NN", "NN")


# ---------------------------------------------------------------- corrected solve

def operator_longdouble(phi, hs, kinds):
    """A phi with the oracle's FP64 operator rows (the stored system that
    every solve here approximates; the rows are pinned above against exact
    rational arithmetic and a dense Kronecker sum) applied in extended
    precision (numpy longdouble, 64-bit significand on x86)."""
    from oracle import tridiagonal as td
    phi = phi.astype(np.longdouble)
    out = np.zeros_like(phi)
    for ax, h, kind in zip((2, 1, 0), hs, kinds):
        a, b, c, _ = td.coefficients(h, kind)
        shape = [1, 1, 1]
        shape[ax] = phi.shape[ax]
        a, b, c = (v.astype(np.longdouble).reshape(shape) for v in (a, b, c))
        out += b * phi + a * np.roll(phi, 1, axis=ax) + c * np.roll(phi, -1, axis=ax)
    return out


@pytest.mark.parametrize("bcs,stretched", [(("DD", "ND", "P"), False), (("P", "P", "NN"), True),
                                           (("NN", "DN", "DD"), True)])
def test_corrected_solve_reaches_the_exact_solution(bcs, stretched):
    """At 128 x 96 x 112 the plain solve's rounding is visible (near 1e-14
    to 1e-13); the corrected solve agrees with a correction made from the
    residual in extended precision (whose own error is below 1e-20
    relative, so that it is the exact solution of the stored system to
    FP64 rounding) at the FP64 rounding level (measured: 1.5e-16 uniform,
    6e-16 stretched), and the plain solve is the less accurate one."""
    nx, ny, nz = 128, 96, 112
    hx, hy = uniform_widths(nx, 1.0), uniform_widths(ny, 1.0)
    hz = tanh_widths(nz, 1.0, 1.8) if stretched else uniform_widths(nz, 1.0)
    f = np.random.default_rng(12).uniform(-1, 1, (nz, ny, nx))
    if op.is_singular(*bcs):
        f = f - op.weighted_mean(f, hx, hy, hz)
    plain = oracle.solve(f, hx, hy, hz, *bcs)
    r = (f.astype(np.longdouble) - operator_longdouble(plain, (hx, hy, hz), bcs)).astype(np.float64)
    exact = plain + oracle.solve(r, hx, hy, hz, *bcs)
    got = oracle.solve_corrected(f, hx, hy, hz, *bcs)
    err = np.linalg.norm(got - exact) / np.linalg.norm(exact)
    err_plain = np.linalg.norm(plain - exact) / np.linalg.norm(exact)
    assert err <= 2e-15, (bcs, err, err_plain)
    assert err <= err_plain, (bcs, err, err_plain)
