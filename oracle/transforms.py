"""Oracle: the one-dimensional discrete transforms of Table 2 and the
eigenvalues of Table 1, written as plain O(n)-per-output sums in FP64.

Test infrastructure only (see ``oracle/__init__.py``).

Every angle that appears in Table 2 is an integer multiple of pi/(4n), so the
sums below evaluate cos/sin of pi*M/(4n) from an exact integer M reduced
modulo 8n (one full turn) instead of from a rounded floating-point product.

Readings of the paper used here (each listed in the design notes):

* DFT ordering (Table 2, first row): coefficient 0 is the plain sum,
  coefficients 2l-1 and 2l (l = 1 .. n/2-1) are the cosine and sine sums of
  wavenumber l, coefficient n-1 is the alternating sum.  The printed row
  labels the wavenumber one off from the eigenvalue row of Table 1; the
  wavenumber used here is the one that makes the pair share the eigenvalue.
* IDFT (Table 2, second row): the interior cosine/sine terms carry a factor 2
  and wavenumber l, so that (1/n) IDFT inverts the DFT (Table 1).
* D-N (Dirichlet at the low face, Neumann at the high face) is not listed in
  Table 1; it is the DST-IV, with the same angles as N-D.
* Non-staggered pairs (Sec. 2.1 says they are needed when diffusion is
  integrated implicitly; the paper gives no table).  The unknowns sit on
  grid nodes: "DDn" has m interior nodes between two boundary nodes where
  the value is zero (DST-I), "NNn" has m nodes whose end nodes carry a zero
  gradient through a mirrored neighbour, x_{-1} = x_1 (DCT-I).  The sums
  are the textbook DST-I and DCT-I; the eigenvalues of the second
  difference with those end rules are -4 sin^2 of pi (q+1) / (2(m+1)) and of
  pi q / (2(m-1)).
"""
import numpy as np

KINDS = ("P", "NN", "DD", "ND", "DN")
NODE_KINDS = ("DDn", "NNn")


def _cos_sin(n, M):
    """cos and sin of pi*M/(4n) for an integer array M (reduced mod 8n)."""
    M = np.mod(np.asarray(M, dtype=np.int64), 8 * n)
    ang = np.pi * M.astype(np.float64) / (4.0 * n)
    return np.cos(ang), np.sin(ang)


def forward_matrix(kind, n):
    """Matrix T with T @ a = F(a) for the forward transform of Table 2.

    P  -> DFT (interleaved real storage), NN -> DCT-II, DD -> DST-II,
    ND -> DCT-IV, DN -> DST-IV.  Unnormalised, exactly as printed.
    """
    p = np.arange(n)[None, :]
    q = np.arange(n)[:, None]
    if kind == "P":
        if n % 2:
            raise ValueError("the DFT of Table 2 needs an even n")
        m = n // 2
        T = np.zeros((n, n))
        T[0, :] = 1.0
        for l in range(1, m):
            c, s = _cos_sin(n, 8 * l * np.arange(n))   # angle 2*pi*p*l/n
            T[2 * l - 1, :] = c
            T[2 * l, :] = s
        T[n - 1, :] = (-1.0) ** np.arange(n)
        return T
    if kind == "NN":   # 2 sum a_p cos(pi (p+1/2) q / n)
        c, _ = _cos_sin(n, 2 * (2 * p + 1) * q)
        return 2.0 * c
    if kind == "DD":   # 2 sum a_p sin(pi (p+1/2) (q+1) / n)
        _, s = _cos_sin(n, 2 * (2 * p + 1) * (q + 1))
        return 2.0 * s
    if kind == "ND":   # 2 sum a_p cos(pi (p+1/2) (q+1/2) / n)
        c, _ = _cos_sin(n, (2 * p + 1) * (2 * q + 1))
        return 2.0 * c
    if kind == "DN":   # 2 sum a_p sin(pi (p+1/2) (q+1/2) / n)
        _, s = _cos_sin(n, (2 * p + 1) * (2 * q + 1))
        return 2.0 * s
    if kind == "DDn":  # DST-I: 2 sum a_p sin(pi (p+1)(q+1) / (n+1)); angle = pi*M/(4(n+1))
        _, s = _cos_sin(n + 1, 4 * (p + 1) * (q + 1))
        return 2.0 * s
    if kind == "NNn":  # DCT-I: a_0 + (-1)^q a_{n-1} + 2 sum_{p=1}^{n-2} a_p cos(pi p q / (n-1))
        if n < 2:
            raise ValueError("a DCT-I needs at least 2 nodes")
        c, _ = _cos_sin(n - 1, 4 * p * q)
        T = 2.0 * c
        T[:, 0] = 1.0
        T[:, n - 1] = (-1.0) ** np.arange(n)
        return T
    raise ValueError(f"unknown boundary pair {kind!r}")


def backward_matrix(kind, n):
    """Matrix B with B @ F(a) = a: the backward operator of Table 1
    ((1/n) IDFT, (1/2n) DCT-III, (1/2n) DST-III, (1/2n) DCT-IV, (1/2n) DST-IV),
    each written from its Table 2 sum."""
    q = np.arange(n)[:, None]      # output index
    p = np.arange(n)[None, :]      # coefficient index
    if kind == "P":
        if n % 2:
            raise ValueError("the IDFT of Table 2 needs an even n")
        m = n // 2
        B = np.zeros((n, n))
        B[:, 0] = 1.0
        for l in range(1, m):
            c, s = _cos_sin(n, 8 * l * np.arange(n))   # angle 2*pi*l*q/n
            B[:, 2 * l - 1] = 2.0 * c
            B[:, 2 * l] = 2.0 * s
        B[:, n - 1] = (-1.0) ** np.arange(n)
        return B / n
    if kind == "NN":   # DCT-III: a_0 + 2 sum_{p>=1} a_p cos(pi p (q+1/2) / n)
        c, _ = _cos_sin(n, 2 * p * (2 * q + 1))
        B = 2.0 * c
        B[:, 0] = 1.0
        return B / (2.0 * n)
    if kind == "DD":   # DST-III: 2 sum_{p<=n-2} a_p sin(pi (p+1)(q+1/2)/n) + (-1)^q a_{n-1}
        _, s = _cos_sin(n, 2 * (p + 1) * (2 * q + 1))
        B = 2.0 * s
        B[:, n - 1] = (-1.0) ** np.arange(n)
        return B / (2.0 * n)
    if kind in ("ND", "DN"):   # DCT-IV and DST-IV are their own inverses up to 2n
        return forward_matrix(kind, n) / (2.0 * n)
    if kind == "DDn":          # DST-I is its own inverse up to 2(n+1)
        return forward_matrix(kind, n) / (2.0 * (n + 1))
    if kind == "NNn":          # DCT-I is its own inverse up to 2(n-1)
        return forward_matrix(kind, n) / (2.0 * (n - 1))
    raise ValueError(f"unknown boundary pair {kind!r}")


def eigenvalues(kind, n):
    """lambda_q = -4 sin^2(theta_q), q = 0 .. n-1, with theta_q from Table 1.

    P: theta_0 = 0, theta_{2l-1} = theta_{2l} = l*pi/n, theta_{n-1} = pi/2.
    NN: q*pi/(2n).  DD: (q+1)*pi/(2n).  ND and DN: (2q+1)*pi/(4n).
    Each theta is pi*M/(4n) with the integer M below.  Node pairs: DDn
    (q+1)*pi/(2(n+1)), NNn q*pi/(2(n-1)).
    """
    q = np.arange(n)
    if kind == "DDn":
        _, s = _cos_sin(n + 1, 2 * (q + 1))
        return -4.0 * s * s
    if kind == "NNn":
        _, s = _cos_sin(n - 1, 2 * q)
        return -4.0 * s * s
    if kind == "P":
        if n % 2:
            raise ValueError("periodic transforms need an even n")
        wavenumber = (q + 1) // 2          # 0, 1, 1, 2, 2, ..., n/2
        M = 4 * wavenumber
    elif kind == "NN":
        M = 2 * q
    elif kind == "DD":
        M = 2 * (q + 1)
    elif kind in ("ND", "DN"):
        M = 2 * q + 1
    else:
        raise ValueError(f"unknown boundary pair {kind!r}")
    _, s = _cos_sin(n, M)
    return -4.0 * s * s


def apply_along(T, f, axis):
    """Apply an (n x n) matrix to every line of ``f`` along ``axis``:
    out[..., q, ...] = sum_p T[q, p] f[..., p, ...]."""
    f = np.moveaxis(np.asarray(f, dtype=np.float64), axis, -1)
    out = f @ T.T
    return np.ascontiguousarray(np.moveaxis(out, -1, axis))


def forward(f, axis, kind):
    """Forward transform F of Table 2 along one array axis."""
    return apply_along(forward_matrix(kind, f.shape[axis]), f, axis)


def backward(f, axis, kind):
    """Backward transform F^-1 of Table 1 along one array axis."""
    return apply_along(backward_matrix(kind, f.shape[axis]), f, axis)
