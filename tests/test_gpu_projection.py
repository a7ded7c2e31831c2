"""GPU parity of the pressure-correction steps (Sec. 2: the right-hand side
of Eq. (poi_ns), the solve, u = u* - gamma dt grad(Phi), p += Phi) against
the oracle (oracle/projection.py) on the same seeded inputs, through the C
ABI: every array within 1e-12 relative L2 (the right-hand side and the
updates are one FP64 stencil each, the solve is bound by 1e-12), and the
divergence of the projected velocity, computed by the GPU, at rounding
level.  Shapes span several blocks with ragged rows; every boundary triple
class, stretched and uniform z, singular and regular."""
import itertools

import numpy as np
import pytest

from gpu_util import rel_l2, to_dev, to_host
from paper_1802_10323_amd import inputs

pytestmark = pytest.mark.gpu

KINDS = ("P", "NN", "DD", "ND", "DN")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_10323_amd import lib
    lib()


def _run(prob, seed, gdt, whole=True):
    import torch
    from oracle import projection as pj
    from paper_1802_10323_amd import Plan
    u, v, w = inputs.prediction_velocity(prob, seed)
    pres = np.random.default_rng(seed + 1).uniform(-1, 1, prob.shape)
    plan = Plan.from_problem(prob)
    du, dv, dw, dp = (to_dev(a) for a in (u, v, w, pres))
    phi = torch.empty(prob.points, dtype=torch.float64, device="cuda")
    args = (prob.hx, prob.hy, prob.hz, prob.bcs)
    rhs_ref = pj.projection_rhs(u, v, w, gdt, *args)
    if whole:
        plan.pressure_correction(du, dv, dw, dp, gdt, phi)
    else:
        plan.projection_rhs(du, dv, dw, gdt, phi)
        assert rel_l2(to_host(phi).reshape(prob.shape), rhs_ref) <= 1e-14
        plan.solve(phi)
        plan.projection_update(phi, gdt, du, dv, dw, dp)
    ref = pj.pressure_correction(u, v, w, pres, gdt, *args)
    got = [to_host(t).reshape(r.shape) for t, r in zip((du, dv, dw, dp, phi), ref)]
    # divergence of the projected velocity, by the GPU
    div = torch.empty_like(phi)
    plan.projection_rhs(du, dv, dw, 1.0, div)
    d1 = np.linalg.norm(to_host(div))
    d0 = np.linalg.norm(pj.divergence(u, v, w, *args))
    plan.close()
    return got, ref, d1 / d0


CASES = [((24, 20, 18), ("P", "P", "NN"), True), ((33, 18, 20), ("DD", "ND", "P"), False),
         ((40, 36, 30), ("NN", "NN", "NN"), False), ((16, 12, 10), ("P", "P", "P"), False),
         ((20, 31, 16), ("P", "ND", "P"), False), ((45, 36, 20), ("DD", "P", "P"), False),
         ((50, 64, 47), ("NN", "DN", "DD"), True), ((300, 8, 5), ("DN", "NN", "DD"), True)]


@pytest.mark.parametrize("shape,bcs,stretched", CASES)
@pytest.mark.parametrize("whole", [True, False])
def test_projection_matches_oracle(shape, bcs, stretched, whole):
    prob = inputs.make_uniform(*shape, bcs, seed=sum(shape), stretch_z=1.8 if stretched else None,
                               with_rhs=False)
    got, ref, div_rel = _run(prob, seed=len(bcs[0]) + sum(shape), gdt=0.37, whole=whole)
    for name, g, r in zip(("u", "v", "w", "p", "phi"), got, ref):
        assert rel_l2(g, r) <= 1e-12, (shape, bcs, name, rel_l2(g, r))
    assert div_rel <= 1e-12, (shape, bcs, div_rel)


def test_projection_all_triples():
    worst = 0.0
    for t, bcs in enumerate(itertools.product(KINDS, repeat=3)):
        prob = inputs.make_uniform(12, 10, 9 if bcs[2] != "P" else 8, bcs, seed=t,
                                   stretch_z=1.8 if (t % 2 and bcs[2] != "P") else None,
                                   with_rhs=False)
        got, ref, div_rel = _run(prob, seed=t, gdt=0.5)
        for name, g, r in zip(("u", "v", "w", "p", "phi"), got, ref):
            err = rel_l2(g, r)
            worst = max(worst, err)
            assert err <= 1e-12, (bcs, name, err)
        assert div_rel <= 1e-12, (bcs, div_rel)
    print("projection, 125 triples: worst rel-L2", worst)


def test_projection_channel_full_size():
    """The channel grid (512 x 256 x 192, periodic x/y, walls in z
    stretched by tanh): one pressure-correction step."""
    prob = inputs.channel(0)
    prob.rhs = None
    got, ref, div_rel = _run(prob, seed=5, gdt=0.01)
    for name, g, r in zip(("u", "v", "w", "p", "phi"), got, ref):
        assert rel_l2(g, r) <= 1e-12, (name, rel_l2(g, r))
    print("channel projection: divergence after / before", div_rel)
    assert div_rel <= 1e-12
