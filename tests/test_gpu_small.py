"""Small grids (x and y transformed, each at most 48 points; z the
elimination axis): the two transforms of each direction run as one launch
that applies dense transform matrices to an x-y plane held in LDS, the
matrices made by the plan's own transform kernels; lines of 32 and 48
points use the 16-lane elimination.  Whole solves against the oracle
(<= 1e-12, Sec. 2.1) and against the same plan's FFT path (POISSON_PLANE=0,
<= 1e-13: the two differ by the rounding of a dense product against an
FFT), on every z boundary pair, uniform and stretched, singular and
regular, node pairs with a Helmholtz shift, FP64 and FP32 + refinement."""
import pytest

from gpu_util import oracle_solve, rel_l2, to_dev, to_host
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


def _solve(prob, monkeypatch, plane, mixed=False):
    from paper_1802_10323_amd import FP32_REFINED, Plan
    if plane:
        monkeypatch.delenv("POISSON_PLANE", raising=False)
    else:
        monkeypatch.setenv("POISSON_PLANE", "0")
    plan = Plan.from_problem(prob)
    if mixed:
        plan.set_precision(FP32_REFINED, 1e-10, 4)
    t = to_dev(prob.rhs)
    plan.solve(t)
    out = to_host(t)
    status = plan.status()
    plan.close()
    return out, status


def _roles(prob):
    from paper_1802_10323_amd import Plan
    plan = Plan.from_problem(prob)
    roles = plan.roles
    plan.close()
    return roles


SHAPES = [(32, 32, 32), (48, 40, 48), (24, 16, 32), (6, 10, 48), (48, 48, 20), (32, 8, 7)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("bz", KINDS)
def test_small_grid_vs_oracle_and_fft_path(shape, bz, monkeypatch):
    nx, ny, nz = shape
    bx, by = KINDS[(nx + nz) % 5], KINDS[(ny + 2 * nz) % 5]
    # a periodic z is the elimination axis only when stretched
    for stretched in ((True,) if bz == "P" else (False, True)):
        prob = inputs.make_uniform(nx, ny, nz, (bx, by, bz), seed=nx + ny + nz,
                                   stretch_z=1.8 if stretched else None)
        ref = oracle_solve(prob)
        got, _ = _solve(prob, monkeypatch, True)
        assert _roles(prob) == ("x", "y", "z")
        fft, _ = _solve(prob, monkeypatch, False)
        e_ref, e_fft = rel_l2(got, ref), rel_l2(got, fft)
        print(shape, (bx, by, bz), stretched, "vs oracle", e_ref, "vs FFT path", e_fft, flush=True)
        assert e_ref <= 1e-12, (shape, bz, stretched, e_ref)
        assert e_fft <= 1e-13, (shape, bz, stretched, e_fft)


@pytest.mark.parametrize("shape", [(32, 32, 32), (40, 48, 48)], ids=lambda s: "x".join(map(str, s)))
def test_small_grid_refined(shape, monkeypatch):
    prob = inputs.make_uniform(*shape, ("P", "DN", "NN"), seed=5, stretch_z=1.8)
    ref = oracle_solve(prob)
    got, (iters, rel, conv) = _solve(prob, monkeypatch, True, mixed=True)
    err = rel_l2(got, ref)
    print(shape, "FP32 + refinement", iters, err, flush=True)
    assert conv and iters <= 4 and err <= 1e-10


def test_small_grid_helmholtz_node_pairs(monkeypatch):
    nx, ny, nz, shift = 31, 33, 32, -350.0
    prob = inputs.make_uniform(nx, ny, nz, ("DDn", "NNn", "DD"), seed=9)
    prob.shift = shift
    ref = oracle_solve(prob)
    got, _ = _solve(prob, monkeypatch, True)
    fft, _ = _solve(prob, monkeypatch, False)
    assert rel_l2(got, ref) <= 1e-12 and rel_l2(got, fft) <= 1e-13
    assert _roles(prob) == ("x", "y", "z")
