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


def batch(log, count=64, steps=5, warmup=2, seed=0):
    """64 uneven instances: one solve() per instance in turn, against the
    batched form (one persistent launch per stage) enqueued directly and as
    a replayed HIP graph.  Every form solves the same fields."""
    import torch
    from . import Batch, Plan, inputs
    probs = inputs.batch(seed, count=count)
    points = sum(p.points for p in probs)
    plans = [Plan.from_problem(p) for p in probs]
    src = [torch.from_numpy(p.rhs).cuda() for p in probs]
    work = [s.clone() for s in src]
    B = Batch(plans)
    B.bind(work)

    def refill():
        for w, s in zip(work, src):
            w.copy_(s)

    def singles():
        for pl, w in zip(plans, work):
            pl.solve(w)

    forms = {"single": singles, "batch": lambda: B.launch(graph=False),
             "graph": lambda: B.launch(graph=True)}
    ms = {}
    results = {}

    def measure(name, fn):
        for _ in range(warmup):
            refill()
            fn()
        times = []
        for _ in range(steps):
            refill()
            times += _timed(fn, 1, torch)
        ms[name] = float(np.median(times))
        refill()
        fn()
        torch.cuda.synchronize()
        results[name] = [w.clone() for w in work[:8]]

    for name, fn in forms.items():
        measure(name, fn)

    def max_rel(name, ref):
        return max(float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
                   for a, b in zip(results[name], results[ref]))

    # single solves use the staging transform where it is the default; the
    # batched kernels have the synchronous variants: equal to rounding
    diff = max(max_rel("batch", "single"), max_rel("graph", "single"))
    # autotuner: time every kernel variant on each instance's shape, keep the
    # fastest per length and layout, rebuild the job tables, measure again
    t0 = time.perf_counter()
    for pl, w in zip(plans, work):
        pl.autotune(w, reps=3)
    tune_s = time.perf_counter() - t0
    B.bind(work)
    measure("single_tuned", singles)
    measure("graph_table", lambda: B.launch(graph=True))
    # then the batch as a whole: per step, the per-length choices against one
    # variant for every job (the launch runs at its largest job's occupancy)
    t0 = time.perf_counter()
    steps_report = B.autotune(reps=5)
    tune_s += time.perf_counter() - t0
    B.bind(work)
    measure("graph_tuned", lambda: B.launch(graph=True))
    diff = max(diff, max_rel("graph_table", "single_tuned"), max_rel("graph_tuned", "single_tuned"))
    batch_choice = {s: ("table" if int(np.argmin(r)) == 0 else int(np.argmin(r)) - 1)
                    for s, r in ((s, [v if v > 0 else np.inf for v in r]) for s, r in steps_report.items())}
    from . import tuned_variant
    chosen = {}
    for n in (64, 96, 128, 192, 256):
        chosen[str(n)] = {"transform_strided": tuned_variant(0, n, 0),
                          "transform_contiguous": tuned_variant(0, n, 1),
                          "elimination_strided": tuned_variant(1, n, 0),
                          "elimination_contiguous": tuned_variant(1, n, 1)}
    log(f"[forms] batch {count} instances ({points / 1e6:.1f} M points): one by one "
        f"{ms['single']:.3f} ms, batched {ms['batch']:.3f} ms, graph {ms['graph']:.3f} ms; "
        f"autotuned ({tune_s:.1f} s): one by one {ms['single_tuned']:.3f} ms, graph with per-length "
        f"variants {ms['graph_table']:.3f} ms, graph tuned as a batch {ms['graph_tuned']:.3f} ms; "
        f"max relative difference to single solves {diff:.1e}")
    fp64_ref = results["single_tuned"]
    B.close()
    # the same instances in FP32 + refinement to 1e-10: one refined solve at
    # a time against the refined batch (each FP32 solve batched) as a graph
    from . import FP32_REFINED
    for pl in plans:
        pl.set_precision(FP32_REFINED, 1e-10, 6)
    B32 = Batch(plans)
    B32.bind(work)
    measure("single_fp32", singles)
    measure("graph_fp32", lambda: B32.launch(graph=True))
    diff32 = max_rel("graph_fp32", "single_fp32")
    err32 = max(float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
                for a, b in zip(results["graph_fp32"], fp64_ref))
    solves = [pl.status()[0] for pl in plans]
    log(f"[forms] batch FP32 + refinement: one by one {ms['single_fp32']:.3f} ms, graph "
        f"{ms['graph_fp32']:.3f} ms ({min(solves)}-{max(solves)} FP32 solves per instance); "
        f"max relative difference to refined single solves {diff32:.1e}, to FP64 {err32:.1e}")
    B32.close()
    for pl in plans:
        pl.close()
    return {"workload": f"{count} instances, per-axis n from {{64,96,128,192,256}}, random BC pairs",
            "points": points, "single_ms": round(ms["single"], 4), "batched_ms": round(ms["batch"], 4),
            "graph_ms": round(ms["graph"], 4),
            "graph_points_per_s": points / (ms["graph"] * 1e-3),
            "speedup_vs_single": round(ms["single"] / ms["graph"], 4),
            "autotune_s": round(tune_s, 2),
            "single_tuned_ms": round(ms["single_tuned"], 4),
            "graph_per_length_tuned_ms": round(ms["graph_table"], 4),
            "graph_tuned_ms": round(ms["graph_tuned"], 4),
            "graph_tuned_points_per_s": points / (ms["graph_tuned"] * 1e-3),
            "speedup_tuned_vs_single_tuned": round(ms["single_tuned"] / ms["graph_tuned"], 4),
            "tuned_variants": chosen,
            "batch_step_choice": batch_choice,
            "max_rel_diff_vs_single": diff,
            "fp32_refined": {"single_ms": round(ms["single_fp32"], 4),
                             "graph_ms": round(ms["graph_fp32"], 4),
                             "graph_points_per_s": points / (ms["graph_fp32"] * 1e-3),
                             "speedup_vs_single": round(ms["single_fp32"] / ms["graph_fp32"], 4),
                             "fp32_solves": [min(solves), max(solves)],
                             "max_rel_diff_vs_single": diff32,
                             "max_rel_l2_vs_fp64": err32, "tolerance": 1e-10}}


def serve(log, count=400, warmup=50, seed=0, slots=8, load=0.8, sample=12):
    """Served stream: per request, per-axis n log-uniform in [32, 512]
    (snapped to even 2^a 3^b 5^c), random boundary pairs, z stretched with
    probability 1/2 when walled, FP64 or FP32 + refinement (tol 1e-10) with
    probability 1/2.  Fields are filled on the device from a seeded
    generator.  Capacity = requests/s of a closed-loop run (all requests
    queued at once); then Poisson arrivals at `load` x capacity, latency =
    completion - submission per request."""
    import torch
    from . import FP32_REFINED, FP64, Plan, Server, inputs
    specs = [inputs.served_request(seed, i, with_rhs=False) for i in range(warmup + count)]
    gen = torch.Generator(device="cuda")
    fields = [torch.empty(sp.points, dtype=torch.float64, device="cuda") for sp in specs]

    def refill():
        gen.manual_seed(seed)
        for f in fields:
            f.uniform_(-1.0, 1.0, generator=gen)
        torch.cuda.synchronize()

    srv = Server(slots=slots)

    def submit(i):
        sp = specs[i]
        return srv.submit(sp, fields[i], FP32_REFINED if sp.mixed else FP64, 1e-10, 6)

    refill()
    for rid in [submit(i) for i in range(warmup)]:
        srv.wait(rid)
    timed = list(range(warmup, warmup + count))
    points = sum(specs[i].points for i in timed)

    # closed loop: everything queued at once
    refill()
    t0 = time.perf_counter()
    infos = [srv.wait(r) for r in [submit(i) for i in timed]]
    closed_s = time.perf_counter() - t0
    capacity = count / closed_s
    bad = sum(1 for x in infos if x["status"] != 0)

    # open loop: Poisson arrivals at load x capacity
    refill()
    rng = np.random.default_rng(seed + 1)
    arrivals = np.cumsum(rng.exponential(1.0 / (load * capacity), count))
    keep = set(timed[:: max(1, count // sample)])
    saved = {i: fields[i].clone() for i in keep}
    torch.cuda.synchronize()
    ids = []
    t0 = time.perf_counter()
    for k, i in enumerate(timed):
        while time.perf_counter() - t0 < arrivals[k]:
            pass
        ids.append(submit(i))
    infos = [srv.wait(r) for r in ids]
    lat = np.array([x["done_s"] - x["submit_s"] for x in infos]) * 1e3
    queue = np.array([x["start_s"] - x["submit_s"] for x in infos]) * 1e3
    span = max(x["done_s"] for x in infos) - min(x["submit_s"] for x in infos)
    bad += sum(1 for x in infos if x["status"] != 0)
    stats = srv.stats()
    srv.close()

    # the same requests alone (fresh plan, default stream)
    same = True
    for i in sorted(keep):
        sp = specs[i]
        plan = Plan.from_problem(sp)
        if sp.mixed:
            plan.set_precision(FP32_REFINED, 1e-10, 6)
        plan.solve(saved[i])
        torch.cuda.synchronize()
        same = same and bool(torch.equal(saved[i], fields[i]))
        plan.close()
    out = {"workload": "served stream, per-axis n log-uniform [32, 512], random BC pairs, "
                       "FP64 or FP32+IR (1e-10) with p = 1/2",
           "requests": count, "warmup": warmup, "slots": slots, "points": points,
           "closed_loop_req_per_s": capacity,
           "closed_loop_points_per_s": points / closed_s,
           "arrival_rate_req_per_s": load * capacity,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "mean_queue_ms": float(queue.mean()),
           "open_loop_points_per_s": points / span,
           "failed": bad, "plan_cache": stats,
           "sampled_equal_to_solo": same, "sampled": len(keep)}
    log(f"[forms] serve: capacity {capacity:.1f} req/s ({points / closed_s:.3e} points/s closed "
        f"loop); at {load:.0%}: p50 {out['p50_ms']:.3f} ms, p99 {out['p99_ms']:.3f} ms, "
        f"{out['open_loop_points_per_s']:.3e} points/s; {len(keep)} sampled results equal "
        f"to solo solves: {same}")
    return out


def run(wanted, log):
    out = {}
    if "mixed" in wanted:
        out["mixed"] = mixed(log)
    if "batch" in wanted:
        out["batch"] = batch(log)
    if "serve" in wanted:
        out["serve"] = serve(log)
    return out
