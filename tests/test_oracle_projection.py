"""Pins for the oracle's projection steps (oracle/projection.py; Sec. 2, the
pressure-correction substep).

* The divergence of the gradient is the seven-point operator of the solve
  (itself pinned by tests/test_oracle_poisson.py), for all 125 boundary
  triples, uniform and stretched z (periodic z included).
* Discrete integration by parts: sum over cells of V Phi div(u) = - sum
  over faces of W u grad(Phi), with the face volumes W written here from
  the geometry (centre distance times face area, half a cell at a wall),
  for velocities with no flux through Neumann walls.  A sign, an index
  offset or a wrong distance in either operator breaks it.
* Closed forms: the gradient of the cell-centre coordinate is 1 on every
  interior face, the divergence of the face coordinate is 1 in every cell,
  for stretched widths.
* After the projection the divergence vanishes to rounding, also for a
  singular problem with a compatible prediction, and p gains Phi.
"""
import itertools

import numpy as np
import pytest

from oracle import poisson as ps
from oracle import projection as pj
from paper_1802_10323_amd.inputs import tanh_widths, uniform_widths

KINDS = ("P", "NN", "DD", "ND", "DN")


def widths(nx, ny, nz, stretched):
    hx, hy = uniform_widths(nx, 1.0), uniform_widths(ny, 2.0)
    hz = tanh_widths(nz, 1.5, 1.8) if stretched else uniform_widths(nz, 1.5)
    return hx, hy, hz


def random_velocity(rng, nx, ny, nz, bcs, no_wall_flux=True):
    """Random face velocities; Neumann wall faces carry no flux."""
    out = []
    for comp in ("x", "y", "z"):
        shape = pj.velocity_shape(comp, nx, ny, nz, bcs)
        vel = rng.uniform(-1, 1, shape)
        kind = dict(zip("xyz", bcs))[comp]
        ax = pj.AXIS[comp]
        if kind != "P" and no_wall_flux:
            n = shape[ax]
            idx_lo = [slice(None)] * 3
            idx_lo[ax] = 0
            idx_hi = [slice(None)] * 3
            idx_hi[ax] = n - 1
            if kind[0] == "N":
                vel[tuple(idx_lo)] = 0.0
            if kind[1] == "N":
                vel[tuple(idx_hi)] = 0.0
        out.append(vel)
    return out


@pytest.mark.parametrize("stretched", [False, True])
def test_divergence_of_gradient_is_the_operator(stretched):
    rng = np.random.default_rng(1)
    nx, ny, nz = 6, 5, 7
    hx, hy, hz = widths(nx, ny, nz, stretched)
    for bcs in itertools.product(KINDS, repeat=3):     # stretched periodic z included
        phi = rng.uniform(-1, 1, (nz, ny, nx))
        g = pj.gradient(phi, hx, hy, hz, bcs)
        for comp, gi in zip("xyz", g):
            assert gi.shape == pj.velocity_shape(comp, nx, ny, nz, bcs)
        dg = pj.divergence(*g, hx, hy, hz, bcs)
        a = ps.apply_operator(phi, hx, hy, hz, *bcs)
        assert np.linalg.norm(dg - a) <= 1e-13 * np.linalg.norm(a), bcs


def face_volumes(comp, nx, ny, nz, hx, hy, hz, bcs):
    """Volume attached to each face of component comp: centre distance (half
    a cell at a wall) times the face area."""
    h = {"x": np.asarray(hx), "y": np.asarray(hy), "z": np.asarray(hz)}
    kind = dict(zip("xyz", bcs))[comp]
    hc = h[comp]
    n = hc.size
    if kind == "P":
        d = np.array([(hc[f - 1] + hc[f]) / 2 for f in range(n)])
    else:
        d = np.array([hc[0] / 2] + [(hc[f - 1] + hc[f]) / 2 for f in range(1, n)] + [hc[-1] / 2])
    parts = {a: h[a] for a in "xyz"}
    parts[comp] = d
    return parts["z"][:, None, None] * parts["y"][None, :, None] * parts["x"][None, None, :]


@pytest.mark.parametrize("stretched", [False, True])
def test_discrete_integration_by_parts(stretched):
    rng = np.random.default_rng(2)
    nx, ny, nz = 5, 6, 4
    hx, hy, hz = widths(nx, ny, nz, stretched)
    for bcs in itertools.product(KINDS, repeat=3):
        phi = rng.uniform(-1, 1, (nz, ny, nx))
        u, v, w = random_velocity(rng, nx, ny, nz, bcs)
        vol = hz[:, None, None] * hy[None, :, None] * hx[None, None, :]
        lhs = np.sum(vol * phi * pj.divergence(u, v, w, hx, hy, hz, bcs))
        g = pj.gradient(phi, hx, hy, hz, bcs)
        rhs = -sum(np.sum(face_volumes(c, nx, ny, nz, hx, hy, hz, bcs) * vel * gi)
                   for c, vel, gi in zip("xyz", (u, v, w), g))
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0), (bcs, lhs, rhs)


def test_closed_forms_on_stretched_widths():
    nx, ny, nz = 7, 5, 9
    hx, hy, hz = uniform_widths(nx, 1.0), uniform_widths(ny, 1.0), tanh_widths(nz, 2.0, 1.8)
    bcs = ("NN", "DD", "ND")
    zc = np.cumsum(hz) - hz / 2                     # cell centres along z
    zf = np.concatenate([[0.0], np.cumsum(hz)])     # faces along z
    phi = np.broadcast_to(zc[:, None, None], (nz, ny, nx)).copy()
    _, _, gz = pj.gradient(phi, np.full(nx, 1.0 / nx), np.full(ny, 1.0 / ny), hz, bcs)
    assert np.allclose(gz[1:nz], 1.0, rtol=0, atol=1e-13)          # interior faces
    w = np.broadcast_to(zf[:, None, None], (nz + 1, ny, nx)).copy()
    u = np.zeros(pj.velocity_shape("x", nx, ny, nz, bcs))
    v = np.zeros(pj.velocity_shape("y", nx, ny, nz, bcs))
    d = pj.divergence(u, v, w, hx, hy, hz, bcs)
    assert np.allclose(d, 1.0, rtol=0, atol=1e-12)
    # a periodic axis: the wrap face joins cell n-1 and cell 0
    phi = np.zeros((3, 3, 4))
    phi[:, :, 0] = 1.0
    gx, _, _ = pj.gradient(phi, np.full(4, 0.5), np.ones(3), np.ones(3), ("P", "P", "P"))
    assert np.allclose(gx[:, :, 0], 2.0) and np.allclose(gx[:, :, 1], -2.0)
    assert np.allclose(gx[:, :, 2:], 0.0)


@pytest.mark.parametrize("bcs,stretched", [(("P", "P", "NN"), True), (("DD", "ND", "P"), False),
                                           (("NN", "NN", "NN"), False), (("P", "P", "P"), False),
                                           (("DN", "P", "DD"), True)])
def test_projection_removes_the_divergence(bcs, stretched):
    rng = np.random.default_rng(3)
    nx, ny, nz = 12, 10, 8
    hx, hy, hz = widths(nx, ny, nz, stretched)
    u, v, w = random_velocity(rng, nx, ny, nz, bcs)
    p = rng.uniform(-1, 1, (nz, ny, nx))
    gdt = 0.37
    u1, v1, w1, p1, phi = pj.pressure_correction(u, v, w, p, gdt, hx, hy, hz, bcs)
    d0 = pj.divergence(u, v, w, hx, hy, hz, bcs)
    d1 = pj.divergence(u1, v1, w1, hx, hy, hz, bcs)
    assert np.linalg.norm(d1) <= 1e-12 * np.linalg.norm(d0), bcs
    assert np.array_equal(p1, p + phi)
    # Neumann walls keep their (prescribed) velocity
    for comp, a, b in zip("xyz", (u, v, w), (u1, v1, w1)):
        kind = dict(zip("xyz", bcs))[comp]
        ax = pj.AXIS[comp]
        if kind != "P" and kind[0] == "N":
            assert np.array_equal(np.take(a, 0, axis=ax), np.take(b, 0, axis=ax))
        if kind != "P" and kind[1] == "N":
            assert np.array_equal(np.take(a, -1, axis=ax), np.take(b, -1, axis=ax))
