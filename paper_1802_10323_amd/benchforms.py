"""Measurements of the solver's further forms for the benchmark report
(each separate from the headline FP64 number):

* mixed  - 512^3 (DD, ND, P) cube: FP32 transforms/elimination + FP64
           refinement to 1e-10 against plain FP64 on the same shape.
* batch  - 64 uneven instances (sizes per axis from {64, 96, 128, 192, 256},
           random boundary pairs, half the walled z axes stretched) in one
           batched launch sequence against one solve at a time.
* serve  - continuous-batching server fed by Poisson arrivals at 80 % of its
           measured capacity: p50 / p99 latency and points/s.
"""
import time

import numpy as np


def _timed(fn, reps, torch):
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in evs]


def mixed(log, steps=6, warmup=2):
    import torch
    from . import FP32_REFINED, Plan, inputs
    prob = inputs.cube(0)
    N = prob.points
    src = torch.from_numpy(prob.rhs).cuda()
    work = torch.empty_like(src)
    p64 = Plan.from_problem(prob)
    p32 = Plan.from_problem(prob)
    p32.set_precision(FP32_REFINED, 1e-10, 4)

    def run(plan):
        work.copy_(src)
        plan.solve(work)

    for _ in range(warmup):
        run(p64)
        run(p32)
    # the copy is inside each event pair for both forms; subtract it
    copy_ms = float(np.median(_timed(lambda: work.copy_(src), steps, torch)))
    t64 = float(np.median(_timed(lambda: run(p64), steps, torch))) - copy_ms
    ref = work.clone()
    t32 = float(np.median(_timed(lambda: run(p32), steps, torch))) - copy_ms
    torch.cuda.synchronize()
    iters, upd, conv = p32.status()
    rel = float(torch.linalg.norm(work - ref) / torch.linalg.norm(ref))
    log(f"[forms] mixed 512^3: fp64 {t64:.3f} ms, fp32+refine {t32:.3f} ms ({iters} FP32 solves), "
        f"rel-L2 vs FP64 {rel:.2e}")
    p64.close()
    p32.close()
    return {"workload": "cube 512^3 (DD,ND,P)", "points": N,
            "fp64_ms": round(t64, 4), "fp64_points_per_s": N / (t64 * 1e-3),
            "mixed_ms": round(t32, 4), "mixed_points_per_s": N / (t32 * 1e-3),
            "speedup_vs_fp64": round(t64 / t32, 4), "fp32_solves": iters,
            "converged": bool(conv), "last_update_rel": upd,
            "rel_l2_vs_gpu_fp64": rel, "tolerance": 1e-10}


def run(wanted, log):
    out = {}
    if "mixed" in wanted:
        out["mixed"] = mixed(log)
    return out
