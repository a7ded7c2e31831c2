"""The solve kernels move neighbouring points with 16-byte accesses, so the
C ABI refuses fields that are not 16-byte aligned (POISSON_EINVAL, before
anything is enqueued), and the same data at an aligned address solves as
usual.  The misaligned views are never handed to a kernel."""
import numpy as np
import pytest

from gpu_util import oracle_solve, rel_l2, to_host
from paper_1802_10323_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_10323_amd import lib
    lib()


def _offset_pair(a):
    """The same values at an aligned address and 8 bytes past one."""
    import torch
    flat = torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).cuda()
    buf = torch.zeros(flat.numel() + 2, dtype=torch.float64, device="cuda")
    assert buf.data_ptr() % 16 == 0
    odd = buf[1:1 + flat.numel()]
    odd.copy_(flat)
    return flat.clone(), odd


def _einval(fn):
    from paper_1802_10323_amd import PoissonError
    from paper_1802_10323_amd.poisson import EINVAL
    with pytest.raises(PoissonError) as e:
        fn()
    assert e.value.code == EINVAL and "16-byte aligned" in str(e.value)


def test_misaligned_fields_are_refused():
    import torch
    from paper_1802_10323_amd import FP32_REFINED, Batch, Plan
    prob = inputs.make_uniform(64, 6, 512, ("DD", "NN", "P"), seed=3)
    plan = Plan.from_problem(prob)
    good, odd = _offset_pair(prob.rhs)
    before = odd.clone()
    _einval(lambda: plan.solve(odd))
    _einval(lambda: plan.transform_stage(0, False, odd))
    _einval(lambda: plan.tridiag_stage(odd))
    _einval(lambda: plan.solve_refined_noalloc(odd))
    torch.cuda.synchronize()
    assert torch.equal(odd, before)            # nothing ran on it
    plan.set_precision(FP32_REFINED, 1e-10, 4)
    _einval(lambda: plan.solve(odd))
    plan.close()
    # a batch of plans the batched kernels take (specialised lengths)
    bprob = inputs.make_uniform(32, 64, 64, ("P", "DD", "NN"), seed=4)
    bplan = Plan.from_problem(bprob)
    _, bodd = _offset_pair(bprob.rhs)
    batch = Batch([bplan])
    _einval(lambda: batch.bind([bodd]))
    batch.close()
    bplan.close()


def test_aligned_copy_solves():
    prob = inputs.make_uniform(64, 6, 512, ("DD", "NN", "P"), seed=3)
    from paper_1802_10323_amd import Plan
    plan = Plan.from_problem(prob)
    good, _ = _offset_pair(prob.rhs)
    plan.solve(good)
    got = to_host(good).reshape(prob.shape)
    plan.close()
    assert rel_l2(got, oracle_solve(prob)) <= 1e-12


def test_time_step_and_server_refuse_misaligned():
    import torch
    from paper_1802_10323_amd import Plan, Server
    n = 16
    plan = Plan(n, n, n, 1.0 / n, 1.0 / n, [1.0 / n] * n, ("P", "P", "P"))
    N = n ** 3
    vel = torch.zeros(3 * N, dtype=torch.float64, device="cuda")
    work = torch.zeros_like(vel)
    ad = torch.zeros(6 * N, dtype=torch.float64, device="cuda")
    p = torch.zeros(N, dtype=torch.float64, device="cuda")
    buf = torch.zeros(2 * N + 2, dtype=torch.float64, device="cuda")
    _einval(lambda: plan.rk3_step(0.01, 0.01, vel, work, ad, p, buf[1:N + 1], buf[:2 * N]))
    _einval(lambda: plan.rk3_substep(1, 0.01, 0.01, vel, work, ad, p, buf[1:N + 1]))
    plan.close()
    prob = inputs.make_uniform(32, 32, 32, ("P", "P", "NN"), seed=1)
    _, odd = _offset_pair(prob.rhs)
    server = Server(slots=2)
    _einval(lambda: server.submit(prob, odd))
    server.close()
