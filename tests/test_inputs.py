"""The seeded input generators: deterministic, the stated shapes, grids that
sum to the box length, and right-hand sides that are compatible when the
problem has a null space."""
import math

import numpy as np

from paper_1802_10323_amd import inputs


def test_tanh_widths_cluster_at_walls():
    h = inputs.tanh_widths(192, 2.0, 1.8)
    assert h.size == 192
    assert abs(h.sum() - 2.0) < 1e-14
    assert np.all(h > 0)
    np.testing.assert_allclose(h, h[::-1], rtol=1e-12)       # symmetric
    assert h.max() / h.min() > 9.0
    assert abs(h[0] - h.min()) < 1e-12 * h.min()


def test_generators_are_deterministic():
    a, b = inputs.small(3), inputs.small(3)
    np.testing.assert_array_equal(a.rhs, b.rhs)
    assert not np.array_equal(a.rhs, inputs.small(4).rhs)
    c = inputs.channel(1, nx=32, ny=16, nz=12, modes=8)
    d = inputs.channel(1, nx=32, ny=16, nz=12, modes=8)
    np.testing.assert_array_equal(c.rhs, d.rhs)


def test_small_and_channel_shapes():
    p = inputs.small(0)
    assert p.shape == (32, 32, 32) and p.bcs == ("P", "P", "NN")
    c = inputs.channel(0, nx=64, ny=32, nz=24, modes=16)
    assert c.shape == (24, 32, 64) and c.bcs == ("P", "P", "NN")
    assert abs(c.dx - 4 * math.pi / 64) < 1e-15
    for prob in (p, c):
        w = prob.hz[:, None, None] * prob.hy[None, :, None] * prob.hx[None, None, :]
        assert abs((w * prob.rhs).sum()) < 1e-12 * np.abs(w * prob.rhs).sum()


def test_batch_and_served_draws():
    insts = inputs.batch(0, count=12)
    assert len(insts) == 12
    for p in insts:
        assert p.nx in inputs.BATCH_SIZES and p.ny in inputs.BATCH_SIZES
        assert p.nz in inputs.BATCH_SIZES
        assert all(b in inputs.BC_NAMES for b in p.bcs)
        if p.bcz == "P":
            assert np.all(p.hz == p.hz[0])
    sizes = inputs.smooth_sizes()
    assert 32 in sizes and 512 in sizes and 96 in sizes and 250 in sizes
    assert all(s % 2 == 0 for s in sizes)
    for i in range(6):
        r = inputs.served_request(0, i, max_points=64 ** 3)
        assert r.points <= 64 ** 3
        assert all(n in sizes for n in (r.nx, r.ny, r.nz))
