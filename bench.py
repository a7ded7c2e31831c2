#!/usr/bin/env python3
"""Benchmark of the MI355X Poisson solver: grid points solved per second.

One step = one complete FP64 solve (forward transforms t1, t2, elimination
along s, backward transforms t2, t1) of the 512^3 cube: unit box, uniform,
Dirichlet-Dirichlet x, Neumann-Dirichlet y, periodic z (so t1 = y, DCT-IV;
t2 = z, DFT; elimination along x), seeded synthetic right-hand side
U[-1, 1].  Inputs are resident in HBM before the timed region (one fresh
copy per step).  The timed region is K steps between two device
synchronisations; HIP events on the solver's stream separate the five
kernels of every step, giving each kernel's average duration for the
roofline.

Prints one JSON line.  Extra objects: `roofline` (dominant kernel:
algorithmic 16 B/point per launch over its measured duration, against the
8 TB/s HBM peak), `cpu_baseline` (the FP64 oracle on the host cores, on the
same field), `rel_l2_vs_oracle` (the solve() result against the oracle),
`kernels` (every kernel's duration and bandwidth), and `forms` (the FP32 +
refinement, channel, 32^3 latency, batched and served forms, each measured
separately and each with its own error against the oracle; not part of
`value`).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
BYTES_PER_POINT_FP64 = 16.0     # one sweep: read + write 8 B per point
STAGES = ("fwd_t1", "fwd_t2", "tridiag", "inv_t2", "inv_t1")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stored_traffic(workload, stage):
    """HBM bytes per launch of `stage` measured by rocprofv3 counters
    (profiles/traffic_<workload>.txt), or None when absent or taken on
    other kernel sources."""
    from paper_1802_10323_amd import profiling
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    src, per_stage = profiling.read_traffic(path)
    if src != profiling.kernel_source_hash():
        return None
    return per_stage.get(stage)


def make_problem(workload, seed=0):
    from paper_1802_10323_amd import inputs
    if workload == "channel":
        return inputs.channel(seed), "channel 512x256x192 (P,P,NN; tanh z beta 1.8; Lx=4pi Ly=2pi Lz=2)"
    if workload == "cube":
        return inputs.cube(seed), "cube 512^3 (DD,ND,P; uniform, unit box)"
    if workload == "small":
        return inputs.small(seed), "small 32^3 (P,P,NN; uniform, unit box)"
    raise SystemExit(f"unknown workload {workload!r}")


def time_fp64(plan, src, steps, warmup, torch):
    """K timed steps of the five stage kernels, with events between them."""
    N = src.numel()
    nbuf = max(1, min(steps, int(12e9 // (8 * N))))
    bufs = [torch.empty_like(src) for _ in range(nbuf)]
    stream = torch.cuda.current_stream()

    def step(buf, evs=None):
        if evs:
            evs[0].record(stream)
        plan.transform_stage(0, False, buf)
        if evs:
            evs[1].record(stream)
        plan.transform_stage(1, False, buf)
        if evs:
            evs[2].record(stream)
        plan.tridiag_stage(buf)
        if evs:
            evs[3].record(stream)
        plan.transform_stage(1, True, buf)
        if evs:
            evs[4].record(stream)
        plan.transform_stage(0, True, buf)
        if evs:
            evs[5].record(stream)

    for i in range(warmup):
        bufs[i % nbuf].copy_(src)
        step(bufs[i % nbuf])
    for b in bufs:
        b.copy_(src)
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        step(bufs[s % nbuf], events[s])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per_stage = [0.0] * 5
    for evs in events:
        for i in range(5):
            per_stage[i] += evs[i].elapsed_time(evs[i + 1])
    per_stage = [v / steps for v in per_stage]        # ms
    return t1 - t0, per_stage


def host_cpu():
    """(CPU model, logical CPUs usable by this process, BLAS threads)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = usable
    return model, usable, threads


def hbm_reference(src, torch, reps=10):
    """Bandwidth that plain sweeps of the field reach with the runtime's own
    kernels (medians over `reps`, events): a copy into a second buffer and an
    in-place scale, each reading and writing the field once (16 B per point,
    like a solver stage).  Context for the stage kernels, not a peak."""
    a = src.clone()
    b = torch.empty_like(src)
    stream = torch.cuda.current_stream()

    def timed(fn):
        out = []
        for _ in range(reps + 2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return float(sorted(out[2:])[reps // 2])

    nbytes = 2 * src.numel() * src.element_size()
    copy_ms = timed(lambda: b.copy_(a))
    scale_ms = timed(lambda: a.mul_(1.0))
    del a, b
    return {"bytes": nbytes, "copy_ms": round(copy_ms, 4),
            "copy_GBs": round(nbytes / (copy_ms * 1e-3) / 1e9, 1),
            "inplace_ms": round(scale_ms, 4),
            "inplace_GBs": round(nbytes / (scale_ms * 1e-3) / 1e9, 1)}


def cpu_baseline(prob, budget_s=12.0, max_reps=6):
    """The FP64 oracle on the host: plain solves of the full workload, as
    many as fit in about `budget_s` (at least one); returns the baseline
    object and the last plain solution."""
    import numpy as np
    import oracle
    model, usable, threads = host_cpu()
    times = []
    phi = None
    t_start = time.perf_counter()
    while not times or (len(times) < max_reps and (time.perf_counter() - t_start) < budget_s):
        t = time.perf_counter()
        phi = oracle.solve(prob.rhs, prob.hx, prob.hy, prob.hz, *prob.bcs)
        times.append(time.perf_counter() - t)
    med = float(np.median(times))
    return {"value": prob.points / med, "unit": "points/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"full workload ({prob.points} points), {len(times)} plain FP64 oracle "
                      f"solve(s) (numpy: dense Table-2 sums through BLAS, Gauss elimination "
                      f"vectorised over columns), median {med:.3f} s; {threads} BLAS threads "
                      f"on {usable} usable logical CPUs, {model}"}, phi


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cube", choices=["cube", "channel", "small"])
    ap.add_argument("--forms", default="all",
                    help="extra forms to measure: none, or a comma list of "
                         "mixed,channel,small,projection,helmholtz,batch,serve (all)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print("this build drives one GPU: multi-GPU runs are not part of it "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("RANK", "0")) != 0:
        return

    import numpy as np
    import torch

    from paper_1802_10323_amd import Plan, lib

    lib()
    torch.cuda.set_device(0)
    prob, workload_desc = make_problem(args.workload)
    log(f"[bench] workload {workload_desc}: {prob.points} points")
    plan = Plan.from_problem(prob)
    src = torch.from_numpy(prob.rhs).cuda()

    elapsed, per_stage = time_fp64(plan, src, args.steps, args.warmup, torch)
    N = prob.points
    value = N * args.steps / elapsed
    ms_per_step = elapsed / args.steps * 1e3
    log(f"[bench] {args.steps} steps in {elapsed:.4f} s: {value:.4e} points/s, {ms_per_step:.3f} ms/step")

    roles = plan.roles
    names = {"fwd_t1": f"r2r forward {roles[0]}", "fwd_t2": f"r2r forward {roles[1]}",
             "tridiag": f"tridiagonal along {roles[2]}", "inv_t2": f"r2r backward {roles[1]}",
             "inv_t1": f"r2r backward {roles[0]}"}
    alg_bytes = BYTES_PER_POINT_FP64 * N
    kernels = []
    for st, ms in zip(STAGES, per_stage):
        kernels.append({"stage": st, "kernel": names[st], "avg_ms": round(ms, 5),
                        "achieved_GBs": round(alg_bytes / (ms * 1e-3) / 1e9, 1),
                        "frac": round(alg_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
    dom = max(range(5), key=lambda i: per_stage[i])
    achieved = alg_bytes / (per_stage[dom] * 1e-3) / 1e9
    traffic = stored_traffic(args.workload, STAGES[dom])
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": names[STAGES[dom]], "algorithmic_bytes_per_launch": alg_bytes}

    # what plain sweeps of the same field reach on this GPU (runtime kernels,
    # no solver arithmetic): context for the stage kernels' bandwidth
    ref_bw = hbm_reference(src, torch)
    log(f"[bench] plain sweeps of the field: copy {ref_bw['copy_GBs']} GB/s, "
        f"in-place scale {ref_bw['inplace_GBs']} GB/s")

    # correctness of the product entry point on this workload
    check = src.clone()
    plan.solve(check)
    torch.cuda.synchronize()
    gpu_phi = check.cpu().numpy()
    del check

    cpu = None
    rel = None
    refs = {}
    if not args.no_cpu_baseline:
        import oracle
        cpu, phi = cpu_baseline(prob)
        corrected = oracle.solve_corrected(prob.rhs, prob.hx, prob.hy, prob.hz, *prob.bcs, phi=phi)
        rel = {"oracle": float(np.linalg.norm(gpu_phi - phi) / np.linalg.norm(phi)),
               "oracle_corrected": float(np.linalg.norm(gpu_phi - corrected)
                                         / np.linalg.norm(corrected)),
               "oracle_vs_corrected": float(np.linalg.norm(phi - corrected)
                                            / np.linalg.norm(corrected))}
        refs[args.workload] = (phi, corrected)
        log(f"[bench] oracle {cpu['value']:.3e} points/s on {cpu['cores']} threads; GPU rel-L2 "
            f"vs oracle {rel['oracle']:.3e}, vs corrected oracle {rel['oracle_corrected']:.3e}")
    del gpu_phi

    forms = {}
    wanted = set() if args.forms == "none" else (
        {"mixed", "channel", "small", "projection", "helmholtz", "taylor_green", "batch", "serve"}
        if args.forms == "all"
        else set(args.forms.split(",")))
    if wanted:
        from paper_1802_10323_amd import benchforms
        forms = benchforms.run(wanted, log, refs, with_oracle=not args.no_cpu_baseline)

    out = {
        "metric": "Poisson grid points solved/s (FP64 direct solve) + %HBM roofline",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload_desc, "points": N, "roles": "".join(roles),
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "hbm_effective": {"bytes_per_point": 5 * BYTES_PER_POINT_FP64,
                          "GBs": round(5 * alg_bytes / (ms_per_step * 1e-3) / 1e9, 1),
                          "frac": round(5 * alg_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "kernels": kernels,
        "hbm_reference": ref_bw,
        "rel_l2_vs_oracle": rel,
        "cpu_baseline": cpu,
        "forms": forms,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
