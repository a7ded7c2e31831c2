"""Seeded synthetic inputs: grids and right-hand sides for the Poisson
workloads.  This module holds no part of the solver's arithmetic (no
transforms, eigenvalues, tridiagonal rows or operator); it only builds cell
widths and random fields, so that the GPU tests, the benchmark and the CPU
oracle all see the same bytes.

All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64), in FP64.

Workloads (sizes and boundary pairs follow the shapes of the paper's cases,
Table 3, and of the benchmark definitions):

* ``small``   32^3, unit box, periodic x and y, Neumann-Neumann z, uniform;
              f ~ U[-1, 1] with the volume-weighted mean removed.
* ``channel`` 512 x 256 x 192 channel-like grid, Lx = 4 pi, Ly = 2 pi, Lz = 2,
              periodic x/y, Neumann z stretched by tanh clustering (beta 1.8)
              toward both walls; f = sum of 64 random separable modes plus
              1e-3 uniform noise, volume-weighted mean removed.
* ``cube``    512^3 unit cube, Dirichlet-Dirichlet x, Neumann-Dirichlet y,
              periodic z; f ~ U[-1, 1].
* ``batch``   many independent instances with per-axis sizes from
              {64, 96, 128, 192, 256} and random boundary pairs.
* ``served``  a stream of requests with per-axis sizes log-uniform in
              [32, 512] snapped to even 2^a 3^b 5^c.
"""
import math

import numpy as np

BC_NAMES = ("P", "NN", "DD", "ND", "DN")


def uniform_widths(n, length=1.0):
    return np.full(n, length / n, dtype=np.float64)


def tanh_widths(n, length, beta):
    """Cell widths of a grid clustered toward both walls:
    faces z_k = (L/2) (1 + tanh(beta (2k/n - 1)) / tanh(beta)), k = 0..n."""
    k = np.arange(n + 1, dtype=np.float64)
    faces = 0.5 * length * (1.0 + np.tanh(beta * (2.0 * k / n - 1.0)) / math.tanh(beta))
    faces[0] = 0.0
    faces[-1] = length
    return np.diff(faces)


def has_null_space(bcx, bcy, bcz):
    """True when no face is Dirichlet (all axes periodic or Neumann-Neumann):
    then only right-hand sides with zero volume-weighted mean are solvable."""
    return all(b in ("P", "NN") for b in (bcx, bcy, bcz))


def remove_weighted_mean(f, hx, hy, hz):
    w = hz[:, None, None] * hy[None, :, None] * hx[None, None, :]
    return f - (w * f).sum() / w.sum()


def centres(h):
    return np.cumsum(h) - 0.5 * h


class Problem:
    """One Poisson instance: sizes, widths, boundary pairs and an FP64 rhs
    laid out f[k, j, i] (z, y, x), x fastest."""

    def __init__(self, hx, hy, hz, bcx, bcy, bcz, rhs, name=""):
        self.hx = np.asarray(hx, dtype=np.float64)
        self.hy = np.asarray(hy, dtype=np.float64)
        self.hz = np.asarray(hz, dtype=np.float64)
        self.bcx, self.bcy, self.bcz = bcx, bcy, bcz
        self.rhs = None if rhs is None else np.ascontiguousarray(rhs, dtype=np.float64)
        self.name = name

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def nx(self):
        return self.hx.size

    @property
    def ny(self):
        return self.hy.size

    @property
    def nz(self):
        return self.hz.size

    @property
    def points(self):
        return self.nx * self.ny * self.nz

    @property
    def bcs(self):
        return (self.bcx, self.bcy, self.bcz)

    @property
    def dx(self):
        return float(self.hx[0])

    @property
    def dy(self):
        return float(self.hy[0])

    def __repr__(self):
        return (f"Problem({self.name!r}, {self.nx}x{self.ny}x{self.nz}, "
                f"bc={self.bcs})")


def random_field(rng, nx, ny, nz):
    return rng.uniform(-1.0, 1.0, size=(nz, ny, nx))


def make_uniform(nx, ny, nz, bcs, seed, lengths=(1.0, 1.0, 1.0), stretch_z=None,
                 name="", with_rhs=True):
    """f ~ U[-1, 1] on a box; z optionally tanh-stretched with factor
    ``stretch_z``; weighted mean removed when the problem has a null space.
    ``with_rhs=False`` builds the grid only (rhs None), for callers that
    fill the field on the device themselves."""
    rng = np.random.default_rng(seed)
    hx = uniform_widths(nx, lengths[0])
    hy = uniform_widths(ny, lengths[1])
    hz = (tanh_widths(nz, lengths[2], stretch_z) if stretch_z
          else uniform_widths(nz, lengths[2]))
    if not with_rhs:
        return Problem(hx, hy, hz, *bcs, None, name=name)
    f = random_field(rng, nx, ny, nz)
    if has_null_space(*bcs):
        f = remove_weighted_mean(f, hx, hy, hz)
    return Problem(hx, hy, hz, *bcs, f, name=name)


def small(seed=0):
    """32^3, periodic x/y, Neumann-Neumann z, uniform unit box."""
    return make_uniform(32, 32, 32, ("P", "P", "NN"), seed, name="small")


def channel(seed=0, nx=512, ny=256, nz=192, modes=64, noise=1e-3, z_profiles=None, drawn=None):
    """Channel-like grid: Lx = 4 pi, Ly = 2 pi, Lz = 2, periodic x/y, Neumann z
    clustered toward both walls (tanh, beta = 1.8).  The right-hand side is a
    seeded sum of ``modes`` separable modes with U[-1, 1] amplitudes: Fourier
    modes exp(2 pi i k x / L) (real or imaginary part) in x and y, and in z
    profile number kz (0 <= kz < nz), by default cos(pi kz (z / Lz)) at the
    stretched cell centres; plus ``noise`` * U[-1, 1]; the volume-weighted
    mean is removed.

    ``z_profiles``: optional callable kz -> nz values replacing the cosines
    (the tests pass the discrete eigenvectors of the stretched z operator,
    which they build from the oracle, to make a manufactured solution);
    ``drawn``: optional list that receives (kx, ky, kz, px, py, amp) per mode."""
    rng = np.random.default_rng(seed)
    Lx, Ly, Lz = 4.0 * math.pi, 2.0 * math.pi, 2.0
    hx = uniform_widths(nx, Lx)
    hy = uniform_widths(ny, Ly)
    hz = tanh_widths(nz, Lz, 1.8)
    xc, yc, zc = centres(hx), centres(hy), centres(hz)
    FZ = np.empty((modes, nz))
    FYX = np.empty((modes, ny * nx))
    for m in range(modes):
        kx = int(rng.integers(0, nx // 2 + 1))
        ky = int(rng.integers(0, ny // 2 + 1))
        kz = int(rng.integers(0, nz))
        px = rng.integers(0, 2) * 0.5 * math.pi    # cos or sin
        py = rng.integers(0, 2) * 0.5 * math.pi
        amp = rng.uniform(-1.0, 1.0)
        if drawn is not None:
            drawn.append((kx, ky, kz, px, py, amp))
        fx = np.cos(2.0 * math.pi * kx * xc / Lx - px)
        fy = np.cos(2.0 * math.pi * ky * yc / Ly - py)
        prof = np.cos(math.pi * kz * zc / Lz) if z_profiles is None else np.asarray(z_profiles(kz))
        FZ[m] = amp * prof
        FYX[m] = np.outer(fy, fx).reshape(-1)
    f = (FZ.T @ FYX).reshape(nz, ny, nx)              # sum of the separable modes
    f += noise * rng.uniform(-1.0, 1.0, size=f.shape)
    f = remove_weighted_mean(f, hx, hy, hz)
    return Problem(hx, hy, hz, "P", "P", "NN", f, name="channel")


def cube(seed=0, n=512):
    """512^3 unit cube: Dirichlet-Dirichlet x, Neumann-Dirichlet y, periodic
    z, f ~ U[-1, 1] (non-singular)."""
    return make_uniform(n, n, n, ("DD", "ND", "P"), seed, name="cube")


BATCH_SIZES = (64, 96, 128, 192, 256)


def batch(seed=0, count=64, sizes=BATCH_SIZES, beta=1.8):
    """``count`` independent instances: each axis size drawn from ``sizes``,
    each boundary pair uniform over P/NN/DD/ND/DN, z tanh-stretched with
    probability 1/2 when its pair is not periodic; unit lengths; per-instance
    seeds seed*1000 + i."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed * 1000 + i)
        nx, ny, nz = (int(rng.choice(sizes)) for _ in range(3))
        bcs = tuple(BC_NAMES[int(rng.integers(0, 5))] for _ in range(3))
        stretch = beta if (bcs[2] != "P" and rng.uniform() < 0.5) else None
        out.append(make_uniform(nx, ny, nz, bcs, seed * 1000 + i + 1,
                                stretch_z=stretch, name=f"batch{i}"))
    return out


def smooth_sizes(lo=32, hi=512):
    """Even sizes 2^a 3^b 5^c in [lo, hi]."""
    out = []
    for n in range(lo, hi + 1, 2):
        m = n
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            out.append(n)
    return out


def snap_size(x, sizes):
    return min(sizes, key=lambda s: (abs(s - x), s))


def served_request(seed, i, lo=32, hi=512, beta=1.8, max_points=None, with_rhs=True):
    """One request of the served stream: per-axis size log-uniform in
    [lo, hi] snapped to an even 2^a 3^b 5^c, random boundary pairs, z
    stretched with probability 1/2 when not periodic, precision FP64 or
    FP32 + refinement with probability 1/2."""
    rng = np.random.default_rng(seed * 1000 + i)
    sizes = smooth_sizes(lo, hi)
    while True:
        dims = [snap_size(math.exp(rng.uniform(math.log(lo), math.log(hi))), sizes)
                for _ in range(3)]
        if max_points is None or dims[0] * dims[1] * dims[2] <= max_points:
            break
    bcs = tuple(BC_NAMES[int(rng.integers(0, 5))] for _ in range(3))
    stretch = beta if (bcs[2] != "P" and rng.uniform() < 0.5) else None
    mixed = bool(rng.uniform() < 0.5)
    p = make_uniform(dims[0], dims[1], dims[2], bcs, seed * 1000 + i + 500000,
                     stretch_z=stretch, name=f"req{i}", with_rhs=with_rhs)
    p.mixed = mixed
    return p


def face_shape(comp, nx, ny, nz, bcs):
    """(nz, ny, nx)-order shape of the face array of velocity component comp
    ('x', 'y' or 'z'): n faces along a periodic axis of n cells, n + 1 along
    a walled one."""
    dims = {"x": nx, "y": ny, "z": nz}
    kind = dict(zip("xyz", bcs))[comp]
    dims[comp] += 0 if kind == "P" else 1
    return (dims["z"], dims["y"], dims["x"])


def prediction_velocity(prob, seed, amplitude=1.0):
    """Seeded face velocities (u, v, w) ~ amplitude * U[-1, 1] on the faces
    of `prob`'s grid, zero on the faces of impermeable walls (the Neumann
    letter of a boundary pair), so that the net flux through the walls is
    zero."""
    rng = np.random.default_rng(seed)
    out = []
    for comp, ax in (("x", 2), ("y", 1), ("z", 0)):
        shape = face_shape(comp, prob.nx, prob.ny, prob.nz, prob.bcs)
        vel = amplitude * rng.uniform(-1.0, 1.0, size=shape)
        kind = dict(zip("xyz", prob.bcs))[comp]
        if kind != "P":
            if kind[0] == "N":
                np.moveaxis(vel, ax, 0)[0] = 0.0
            if kind[1] == "N":
                np.moveaxis(vel, ax, 0)[-1] = 0.0
        out.append(vel)
    return out


def taylor_green(n=512, U=1.0, L=1.0, with_pressure=True):
    """The Taylor-Green vortex initial condition (Sec. 4.1, Table 3) on the
    tri-periodic box [0, 2 pi L]^3 with n cells per axis:
    u = U sin(x/L) cos(y/L) cos(z/L), v = -U cos(x/L) sin(y/L) cos(z/L),
    w = 0, sampled where each component is stored (u[k, j, i] at
    (i dx, (j + 1/2) dx, (k + 1/2) dx), v and w likewise on their own faces).

    The pressure is not part of the stated condition; with_pressure gives
    the one of the inviscid Taylor-Green flow at t = 0,
    p = (U^2 / 16) (cos(2x/L) + cos(2y/L)) (cos(2z/L) + 2), at cell centres,
    else zero.  Returns (u, v, w, p, dx), arrays indexed [k, j, i]."""
    d = 2.0 * math.pi * L / n
    face = np.arange(n, dtype=np.float64) * d / L
    centre = (np.arange(n, dtype=np.float64) + 0.5) * d / L
    X = (None, None, slice(None))                # broadcast along the last axis (x)
    Y = (None, slice(None), None)
    Z = (slice(None), None, None)
    u = U * np.sin(face)[X] * np.cos(centre)[Y] * np.cos(centre)[Z]
    v = -U * np.cos(centre)[X] * np.sin(face)[Y] * np.cos(centre)[Z]
    w = np.zeros((n, n, n))
    if with_pressure:
        p = ((U * U / 16.0) * (np.cos(2 * centre)[X] + np.cos(2 * centre)[Y])
             * (np.cos(2 * centre)[Z] + 2.0))
    else:
        p = np.zeros((n, n, n))
    return u, v, w, p, d
