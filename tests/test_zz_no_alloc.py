"""The refined solve that allocates nothing (solve_refined_noalloc, for
callers that cannot allocate device memory) against the existing refined
entry point (solve() on a POISSON_FP32_REFINED plan, which runs on the
plan's own workspace): same kernels, same launch sequence, so the same bits
and the same refinement status; two calls in a row, the second on a
smaller grid (the static workspace keeps the first call's contents), and
within 1e-10 of the FP64 oracle (Sec. 2.1, Eq. (poi))."""
import numpy as np
import pytest

from gpu_util import oracle_solve, rel_l2, to_dev, to_host
from paper_1802_10323_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_10323_amd import lib
    lib()


def _existing(prob, tol, max_iters):
    from paper_1802_10323_amd import FP32_REFINED, Plan
    plan = Plan.from_problem(prob)
    plan.set_precision(FP32_REFINED, tol, max_iters)
    d = to_dev(prob.rhs)
    plan.solve(d)
    out = to_host(d)
    status = plan.status()
    plan.close()
    return out, status


def test_noalloc_equals_refined_solve_two_calls():
    import torch
    from paper_1802_10323_amd import Plan
    big = inputs.make_uniform(128, 96, 80, ("DD", "ND", "P"), seed=31)
    small = inputs.make_uniform(40, 36, 30, ("P", "P", "NN"), seed=32, stretch_z=1.8)
    cases = [(big, 1e-10, 6), (small, 1e-10, 6)]
    refs = [_existing(p, tol, it) for p, tol, it in cases]
    plans = [Plan.from_problem(p) for p, _, _ in cases]        # FP64 plans: no workspace
    status = torch.zeros(3, dtype=torch.float64, device="cuda")
    fields = [to_dev(p.rhs) for p, _, _ in cases]
    torch.cuda.synchronize()
    # two calls in a row on one stream, the second on the smaller grid
    outs = []
    for plan, field, (p, tol, it) in zip(plans, fields, cases):
        plan.solve_refined_noalloc(field, tol, it, status=status)
        outs.append((to_host(field), to_host(status).copy()))
    for (got, st), (ref, (iters, rel, conv)), (p, _, _) in zip(outs, refs, cases):
        assert np.array_equal(got, ref), p
        assert int(st[0]) == iters and bool(st[1]) == conv and st[2] == rel, (p, st, iters, rel, conv)
        assert conv and iters <= 4
        assert rel_l2(got, oracle_solve(p)) <= 1e-10, p
    # again, after other device work: no device memory is taken
    free0, _ = torch.cuda.mem_get_info()
    for plan, field, (p, tol, it), (got, _) in zip(plans, fields, cases, outs):
        field.copy_(torch.from_numpy(p.rhs))
        plan.solve_refined_noalloc(field, tol, it)
        assert np.array_equal(to_host(field), got), p
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0
    for pl in plans:
        pl.close()


def test_noalloc_rejects_grid_beyond_workspace():
    """A grid larger than the static workspace is refused before anything is
    enqueued (the raw C call with a small buffer: nothing touches it)."""
    import ctypes
    import torch
    from paper_1802_10323_amd import Plan, lib, refined_noalloc_max_points
    from paper_1802_10323_amd.poisson import EUNSUPPORTED
    cap = refined_noalloc_max_points()
    assert cap >= 256 ** 3       # a 256^3 grid fits
    plan = Plan(512, 512, 96, 1.0, 1.0, np.ones(96), ("DD", "ND", "P"))
    assert 512 * 512 * 96 > cap
    field = torch.zeros(8, dtype=torch.float64, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib().solve_refined_noalloc(plan.handle, ctypes.c_void_p(field.data_ptr()), 1e-10, 4,
                                     None, stream)
    assert rc == EUNSUPPORTED
    assert b"no-allocation workspace" in lib().last_error_message()
    torch.cuda.synchronize()
    assert torch.count_nonzero(field).item() == 0
    plan.close()
