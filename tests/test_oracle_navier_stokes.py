"""Pins for the oracle's Navier-Stokes step (oracle/navier_stokes.py; Sec. 2,
Eq. (up) with the pressure correction, on the tri-periodic staggered grid of
the Taylor-Green case, Sec. 4.1).

* Conservation: the divergence-form advection sums to zero per component
  (momentum) for any field, and u . adv(u) sums to zero (kinetic energy)
  for a discretely divergence-free field, not for others.
* Consistency: the discrete AD converges at second order to the analytic
  -(u . grad) u + nu lap(u) of the ABC (Beltrami) flow, where it is
  -grad(|u|^2 / 2) - nu u, and of the Taylor-Green initial condition, on
  boxes with three different spacings.  A dropped or mis-signed term does
  not converge; a half-cell offset converges at first order only.
* A shear mode u = sin(m y) has no advection and its diffusion is the
  exact discrete eigenvalue nu (2 cos(m dy) - 2) / dy^2.
* One step of that mode multiplies it by 1 + z + z^2/2 + z^3/6, z = dt nu
  lambda: the stability polynomial of every three-stage third-order
  Runge-Kutta scheme, reached only with the stated alpha, beta, gamma.
* A fluid at rest under any pressure stays at rest and the pressure drops
  to its mean after one substep: pins the sign and the gamma_k of the
  pressure gradient in the prediction against those of the projection.
* Every substep leaves a divergence-free velocity; one step of the 2D
  Taylor-Green flow (an exact Navier-Stokes solution) converges to it.
"""
import math

import numpy as np
import pytest

from oracle import navier_stokes as ns
from oracle import projection as pj
from paper_1802_10323_amd import inputs

P3 = ("P", "P", "P")


def faces(n, d):
    return np.arange(n) * d


def centres(n, d):
    return (np.arange(n) + 0.5) * d


def grid_coords(comp, nx, ny, nz, dx, dy, dz):
    """Broadcastable (z, y, x) coordinates where component comp is stored
    (comp 'p' for cell centres)."""
    x = faces(nx, dx) if comp == "u" else centres(nx, dx)
    y = faces(ny, dy) if comp == "v" else centres(ny, dy)
    z = faces(nz, dz) if comp == "w" else centres(nz, dz)
    return z[:, None, None], y[None, :, None], x[None, None, :]


def div(u, v, w, dx, dy, dz):
    nz, ny, nx = u.shape
    return pj.divergence(u, v, w, ns.widths(nx, dx), ns.widths(ny, dy), ns.widths(nz, dz), P3)


def projected_random(rng, nx, ny, nz, dx, dy, dz):
    u, v, w = (rng.uniform(-1, 1, (nz, ny, nx)) for _ in range(3))
    p = np.zeros((nz, ny, nx))
    hx, hy, hz = ns.widths(nx, dx), ns.widths(ny, dy), ns.widths(nz, dz)
    u, v, w, _, _ = pj.pressure_correction(u, v, w, p, 1.0, hx, hy, hz, P3)
    return u, v, w


def test_advection_conserves_momentum():
    rng = np.random.default_rng(1)
    u, v, w = (rng.uniform(-1, 1, (5, 6, 7)) for _ in range(3))
    for a in ns.advection(u, v, w, 0.3, 0.2, 0.7):
        assert abs(a.sum()) <= 1e-12 * np.abs(a).sum()


def test_advection_conserves_energy_only_when_divergence_free():
    rng = np.random.default_rng(2)
    dx, dy, dz = 0.3, 0.2, 0.45
    u, v, w = projected_random(rng, 8, 6, 10, dx, dy, dz)
    assert np.linalg.norm(div(u, v, w, dx, dy, dz)) <= 1e-12 * np.linalg.norm(u) / dx
    au, av, aw = ns.advection(u, v, w, dx, dy, dz)
    e = (u * au).sum() + (v * av).sum() + (w * aw).sum()
    scale = np.abs(u * au).sum() + np.abs(v * av).sum() + np.abs(w * aw).sum()
    assert abs(e) <= 1e-13 * scale
    # a field with divergence changes the energy
    u2 = u + 0.1 * rng.uniform(-1, 1, u.shape)
    au, av, aw = ns.advection(u2, v, w, dx, dy, dz)
    e = (u2 * au).sum() + (v * av).sum() + (w * aw).sum()
    assert abs(e) >= 1e-4 * scale


def abc_flow(nx, ny, nz, A=1.0, B=0.7, C=0.4):
    """ABC flow on [0, 2 pi]^3 at the stored positions, with its exact
    (u . grad) u = grad(|u|^2 / 2) (a Beltrami flow, curl u = u) and
    lap u = -u."""
    dx, dy, dz = (2 * math.pi / n for n in (nx, ny, nz))
    out, conv = [], []
    for comp in "uvw":
        z, y, x = grid_coords(comp, nx, ny, nz, dx, dy, dz)
        uu = A * np.sin(z) + C * np.cos(y)
        vv = B * np.sin(x) + A * np.cos(z)
        ww = C * np.sin(y) + B * np.cos(x)
        val = {"u": uu, "v": vv, "w": ww}[comp]
        g = {"u": vv * B * np.cos(x) - ww * B * np.sin(x),
             "v": -uu * C * np.sin(y) + ww * C * np.cos(y),
             "w": uu * A * np.cos(z) - vv * A * np.sin(z)}[comp]
        out.append(np.broadcast_to(val, (nz, ny, nx)).copy())
        conv.append(np.broadcast_to(g, (nz, ny, nx)).copy())
    return out, conv, (dx, dy, dz)


def taylor_green_exact(nx, ny, nz):
    """The Taylor-Green initial field (U = L = 1) and its exact (u . grad) u
    = (sin 2x cos^2 z / 2, sin 2y cos^2 z / 2, 0) and lap u = -3 u."""
    dx, dy, dz = (2 * math.pi / n for n in (nx, ny, nz))
    vel, conv = [], []
    for comp in "uvw":
        z, y, x = grid_coords(comp, nx, ny, nz, dx, dy, dz)
        val = {"u": np.sin(x) * np.cos(y) * np.cos(z),
               "v": -np.cos(x) * np.sin(y) * np.cos(z), "w": 0 * x * y * z}[comp]
        g = {"u": 0.5 * np.sin(2 * x) * np.cos(z) ** 2,
             "v": 0.5 * np.sin(2 * y) * np.cos(z) ** 2, "w": 0 * x * y * z}[comp]
        vel.append(np.broadcast_to(val, (nz, ny, nx)).copy())
        conv.append(np.broadcast_to(g, (nz, ny, nx)).copy())
    return vel, conv, (dx, dy, dz), 3.0


@pytest.mark.parametrize("flow", ["abc", "taylor_green"])
def test_ad_converges_at_second_order(flow):
    nu = 0.05
    errs = []
    for s in (2, 4, 8):
        nx, ny, nz = 12 * s, 16 * s, 10 * s
        if flow == "abc":
            vel, conv, d = abc_flow(nx, ny, nz)
            lap_factor = 1.0
        else:
            vel, conv, d, lap_factor = taylor_green_exact(nx, ny, nz)
        ad = ns.advection_diffusion(*vel, *d, nu)
        exact = [-g - nu * lap_factor * a for g, a in zip(conv, vel)]
        errs.append(max(np.max(np.abs(a - e)) for a, e in zip(ad, exact)))
    assert errs[0] > 1e-3                     # the test resolves the truncation error
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.6 <= e0 / e1 <= 4.4, errs


def test_shear_mode_is_exact():
    nx, ny, nz, m = 6, 20, 4, 3
    dx, dy, dz = 0.5, 2 * math.pi / ny, 0.25
    nu = 0.3
    y = centres(ny, dy)[None, :, None]
    u = np.broadcast_to(np.sin(m * y), (nz, ny, nx)).copy()
    zero = np.zeros_like(u)
    au, av, aw = ns.advection(u, zero, zero, dx, dy, dz)
    assert max(np.abs(a).max() for a in (au, av, aw)) == 0.0
    lam = (2 * math.cos(m * dy) - 2) / dy ** 2
    adu, adv, adw = ns.advection_diffusion(u, zero, zero, dx, dy, dz, nu)
    assert np.allclose(adu, nu * lam * u, rtol=0, atol=1e-14 * nu * abs(lam))
    assert np.abs(adv).max() == 0.0 and np.abs(adw).max() == 0.0


@pytest.mark.parametrize("dt", [0.01, 0.05, 0.2])
def test_rk3_step_is_the_third_order_taylor_polynomial(dt):
    nx, ny, nz, m = 4, 16, 6, 2
    dx, dy, dz = 0.5, 2 * math.pi / ny, 0.3
    nu = 0.4
    z_ = np.arange(nz)[:, None, None]
    x_ = np.arange(nx)[None, None, :]
    y = centres(ny, dy)[None, :, None]
    u = np.broadcast_to(np.cos(m * y) + 0 * z_ + 0 * x_, (nz, ny, nx)).copy()
    zero = np.zeros_like(u)
    z = dt * nu * (2 * math.cos(m * dy) - 2) / dy ** 2
    u1, v1, w1, p1 = ns.rk3_step(u, zero, zero, zero, dt, nu, dx, dy, dz)
    assert np.allclose(u1, u * (1 + z + z * z / 2 + z ** 3 / 6), rtol=0, atol=1e-14)
    assert max(np.abs(a).max() for a in (v1, w1, p1)) <= 1e-14


@pytest.mark.parametrize("k", [1, 2, 3])
def test_rest_stays_at_rest_and_pressure_drops_to_its_mean(k):
    rng = np.random.default_rng(3 + k)
    nx, ny, nz = 8, 6, 10
    dx, dy, dz = 0.3, 0.5, 0.2
    p = rng.uniform(-1, 1, (nz, ny, nx))
    zero = np.zeros_like(p)
    u1, v1, w1, p1, ad, phi = ns.rk3_substep(k, zero, zero, zero, p, (zero,) * 3, 0.07, 0.1,
                                             dx, dy, dz)
    assert max(np.abs(a).max() for a in (u1, v1, w1)) <= 1e-12
    assert np.allclose(p1, p.mean(), rtol=0, atol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_substeps_are_divergence_free(k):
    rng = np.random.default_rng(10 + k)
    nx, ny, nz = 10, 8, 6
    dx, dy, dz = 0.3, 0.5, 0.2
    vel = [rng.uniform(-1, 1, (nz, ny, nx)) for _ in range(3)]
    ad_prev = [rng.uniform(-1, 1, (nz, ny, nx)) for _ in range(3)]
    p = rng.uniform(-1, 1, (nz, ny, nx))
    u1, v1, w1, p1, ad, phi = ns.rk3_substep(k, *vel, p, ad_prev, 0.05, 0.01, dx, dy, dz)
    d0 = div(*vel, dx, dy, dz)
    assert np.linalg.norm(div(u1, v1, w1, dx, dy, dz)) <= 1e-13 * np.linalg.norm(d0)
    assert np.array_equal(p1, p + phi)


def taylor_green_2d(n, nz, t, nu):
    """The decaying 2D Taylor-Green flow, an exact Navier-Stokes solution:
    u = sin x cos y F, v = -cos x sin y F, p = (cos 2x + cos 2y) F^2 / 4,
    F = exp(-2 nu t), independent of z."""
    d = 2 * math.pi / n
    F = math.exp(-2 * nu * t)
    zu, yu, xu = grid_coords("u", n, n, nz, d, d, 1.0)
    zv, yv, xv = grid_coords("v", n, n, nz, d, d, 1.0)
    zp, yp, xp = grid_coords("p", n, n, nz, d, d, 1.0)
    shape = (nz, n, n)
    u = np.broadcast_to(np.sin(xu) * np.cos(yu) * F, shape).copy()
    v = np.broadcast_to(-np.cos(xv) * np.sin(yv) * F, shape).copy()
    p = np.broadcast_to((np.cos(2 * xp) + np.cos(2 * yp)) * F * F / 4, shape).copy()
    return u, v, np.zeros(shape), p, d


def test_taylor_green_2d_step_converges():
    nu = 0.05
    errs = []
    for n in (16, 32, 64):
        u, v, w, p, d = taylor_green_2d(n, 4, 0.0, nu)
        dt = 0.4 * d
        u1, v1, w1, _ = ns.rk3_step(u, v, w, p, dt, nu, d, d, 1.0)
        ue, ve, _, _, _ = taylor_green_2d(n, 4, dt, nu)
        errs.append(max(np.abs(u1 - ue).max(), np.abs(v1 - ve).max()))
        assert np.abs(w1).max() <= 1e-14
    for e0, e1 in zip(errs, errs[1:]):
        assert e0 / e1 >= 6.0, errs        # one step: dt h^2 + dt^3, dt ~ h


def test_stable_dt_of_the_taylor_green_start():
    u, v, w, p, d = inputs.taylor_green(32)
    nu = 1.0 / 1600
    vmax = np.max(np.abs(u) + np.abs(v) + np.abs(w))
    # co-located, |sin x cos y| + |cos x sin y| = max |sin(x +- y)| <= 1; the
    # staggered pairing of u and v at one index moves each by half a cell
    assert 0.9 < vmax <= 1.0 + d
    assert ns.stable_dt(u, v, w, d, d, d, nu) == pytest.approx(math.sqrt(3) * d / vmax, rel=1e-15)
    # viscous limit wins at low Reynolds number
    assert ns.stable_dt(u, v, w, d, d, d, 10.0) == pytest.approx(1.65 * d * d / 10.0, rel=1e-15)


def test_taylor_green_input_is_divergence_free():
    u, v, w, p, d = inputs.taylor_green(24)
    dv = div(u, v, w, d, d, d)
    assert np.abs(dv).max() <= 1e-13
    assert p.shape == u.shape and abs(p.mean()) <= 1e-15 + 1e-12 * np.abs(p).max()
