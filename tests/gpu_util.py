"""Helpers for the GPU tests: run the HIP path through the C ABI on seeded
inputs and compare with the oracle."""
import numpy as np

AXIS = {"x": 2, "y": 1, "z": 0}


def rel_l2(a, b):
    d = np.linalg.norm(np.asarray(a) - np.asarray(b))
    r = np.linalg.norm(np.asarray(b))
    return d / r if r > 0 else d


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def gpu_solve(prob, mixed=False, tol=1e-10, max_iters=4):
    from paper_1802_10323_amd import FP32_REFINED, Plan
    plan = Plan.from_problem(prob)
    if mixed:
        plan.set_precision(FP32_REFINED, tol, max_iters)
    t = to_dev(prob.rhs)
    plan.solve(t)
    out = to_host(t)
    status = plan.status()
    plan.close()
    return out, status


def oracle_solve(prob, roles=("x", "y", "z")):
    import oracle
    return oracle.solve(prob.rhs, prob.hx, prob.hy, prob.hz, *prob.bcs, roles=roles)
