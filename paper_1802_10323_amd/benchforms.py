"""Measurements of the solver's further forms for the benchmark report
(each separate from the headline FP64 number), each with its relative L2
error against the FP64 oracle on the same seeded input (the oracle runs on
the host; it is the test reference, timed nowhere here):

* mixed   - 512^3 (DD, ND, P) cube: FP32 transforms (elimination
            recurrences in FP64 on FP32 data) + FP64 residual/update,
            refined to 1e-10, against plain FP64 on the same shape.
* channel - 512 x 256 x 192 channel (P, P, NN; tanh z), FP64.
* small   - 32^3 (P, P, NN), FP64: a latency-bound solve; host round-trip
            latency p50/p99 over 2000 solves and device time per solve.
* batch   - 64 uneven instances (sizes per axis from {64, 96, 128, 192,
            256}, random boundary pairs, half the walled z axes stretched) in
            one batched launch sequence against one solve at a time.
* projection - one pressure-correction step (right-hand side of
            Eq. (poi_ns), FP64 solve, velocity and pressure update) on the
            channel grid.
* helmholtz - Helmholtz solves (A + shift) Phi = f of an implicit
            diffusion step: the wall-normal velocity of a channel (node
            Dirichlet pair along z, 512 x 256 x 191 interior nodes) and a
            field whose x axis carries a node pair (DST-I of 255 nodes).
* taylor_green - one low-storage RK3 time step of the 512^3 Taylor-Green
            vortex (tri-periodic, Re 1600): per substep the prediction, the
            right-hand side, the FP64 solve and the update.
* serve   - continuous-batching server fed by Poisson arrivals at 80 % of
            its measured capacity: p50 / p99 latency and points/s, for 2, 4
            and 8 slots.
"""
import math
import threading
import time

import numpy as np

# low-storage RK3 coefficients of the time step (Sec. 2), for timing its parts
ALPHA = (8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0)
BETA = (0.0, -17.0 / 60.0, -5.0 / 12.0)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _oracle_pair(prob, refs=None, key=None):
    """(plain, corrected) oracle solutions of prob, from refs[key] if there."""
    import oracle
    if refs is not None and key in refs:
        return refs[key]
    args = (prob.rhs, prob.hx, prob.hy, prob.hz, *prob.bcs)
    plain = oracle.solve(*args)
    return plain, oracle.solve_corrected(*args, phi=plain)


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


def mixed(log, refs=None, with_oracle=True, steps=6, warmup=2):
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
    out = {"workload": "cube 512^3 (DD,ND,P)", "points": N,
           "arithmetic": "FP32 transforms, FP64 elimination recurrences on FP32 data, "
                         "FP64 residual/update/gauge",
           "fp64_ms": round(t64, 4), "fp64_points_per_s": N / (t64 * 1e-3),
           "mixed_ms": round(t32, 4), "mixed_points_per_s": N / (t32 * 1e-3),
           "speedup_vs_fp64": round(t64 / t32, 4), "fp32_solves": iters,
           "converged": bool(conv), "last_update_rel": upd,
           "rel_l2_vs_gpu_fp64": rel, "tolerance": 1e-10}
    if with_oracle:
        plain, corrected = _oracle_pair(prob, refs, "cube")
        got = work.cpu().numpy()
        out["rel_l2_vs_oracle"] = _rel(got, plain)
        out["rel_l2_vs_oracle_corrected"] = _rel(got, corrected)
        out["fp64_rel_l2_vs_oracle_corrected"] = _rel(ref.cpu().numpy(), corrected)
    log(f"[forms] mixed 512^3: fp64 {t64:.3f} ms, fp32+refine {t32:.3f} ms ({iters} FP32 solves), "
        f"rel-L2 vs FP64 {rel:.2e}, vs oracle {out.get('rel_l2_vs_oracle_corrected', float('nan')):.2e}")
    p64.close()
    p32.close()
    return out


def channel(log, refs=None, with_oracle=True, steps=20, warmup=3):
    """The 512 x 256 x 192 channel (P, P, NN; z tanh-stretched), FP64."""
    import torch
    from . import Plan, inputs
    prob = inputs.channel(0)
    N = prob.points
    src = torch.from_numpy(prob.rhs).cuda()
    work = torch.empty_like(src)
    plan = Plan.from_problem(prob)

    def run():
        work.copy_(src)
        plan.solve(work)

    for _ in range(warmup):
        run()
    copy_ms = float(np.median(_timed(lambda: work.copy_(src), steps, torch)))
    t = float(np.median(_timed(run, steps, torch))) - copy_ms
    run()
    torch.cuda.synchronize()
    out = {"workload": "channel 512x256x192 (P,P,NN; tanh z beta 1.8; Lx=4pi Ly=2pi Lz=2)",
           "points": N, "ms": round(t, 4), "points_per_s": N / (t * 1e-3),
           "hbm_effective_frac": round(80.0 * N / (t * 1e-3) / 8e12, 4),
           "note": "the FP64 field (201 MB) fits in the 256 MB Infinity Cache: part of each "
                   "sweep's traffic may be served there, not by HBM"}
    if with_oracle:
        plain, corrected = _oracle_pair(prob, refs, "channel")
        got = work.cpu().numpy()
        out["rel_l2_vs_oracle"] = _rel(got, plain)
        out["rel_l2_vs_oracle_corrected"] = _rel(got, corrected)
    plan.close()
    log(f"[forms] channel: {t:.4f} ms, {N / (t * 1e-3):.3e} points/s, rel-L2 vs oracle "
        f"{out.get('rel_l2_vs_oracle', float('nan')):.2e}")
    return out


def small(log, refs=None, with_oracle=True, count=2000, warmup=200):
    """32^3 (P, P, NN), FP64, latency-bound: per solve, the host round trip
    (enqueue the solve, wait for the stream) and the device time between
    events around it; the field is refilled (untimed) before each solve."""
    import torch
    from . import Plan, inputs
    prob = inputs.small(0)
    N = prob.points
    src = torch.from_numpy(prob.rhs).cuda()
    work = torch.empty_like(src)
    plan = Plan.from_problem(prob)
    stream = torch.cuda.current_stream()
    host_us, dev_us = [], []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for i in range(warmup + count):
        work.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        plan.solve(work)
        e1.record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if i >= warmup:
            host_us.append((t1 - t0) * 1e6)
            dev_us.append(e0.elapsed_time(e1) * 1e3)
    # throughput: solves enqueued back to back (each on its own refilled copy)
    bufs = [src.clone() for _ in range(64)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in bufs:
        plan.solve(b)
    torch.cuda.synchronize()
    back_to_back_us = (time.perf_counter() - t0) / len(bufs) * 1e6
    host_us, dev_us = np.array(host_us), np.array(dev_us)
    out = {"workload": "small 32^3 (P,P,NN; uniform, unit box)", "points": N, "solves": count,
           "latency_p50_us": float(np.percentile(host_us, 50)),
           "latency_p99_us": float(np.percentile(host_us, 99)),
           "device_p50_us": float(np.percentile(dev_us, 50)),
           "device_p99_us": float(np.percentile(dev_us, 99)),
           "back_to_back_us_per_solve": back_to_back_us,
           "points_per_s_latency": N / (np.percentile(host_us, 50) * 1e-6),
           "points_per_s_back_to_back": N / (back_to_back_us * 1e-6)}
    if with_oracle:
        plain, corrected = _oracle_pair(prob)
        got = bufs[0].cpu().numpy()
        out["rel_l2_vs_oracle"] = _rel(got, plain)
        out["rel_l2_vs_oracle_corrected"] = _rel(got, corrected)
    plan.close()
    log(f"[forms] small 32^3: latency p50 {out['latency_p50_us']:.1f} us, p99 "
        f"{out['latency_p99_us']:.1f} us (device {out['device_p50_us']:.1f} us), back to back "
        f"{back_to_back_us:.1f} us/solve")
    return out


def batch(log, refs=None, with_oracle=True, count=64, steps=5, warmup=2, seed=0, checked=4):
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
    # oracle check of the `checked` smallest of the instances kept above
    check_ids = sorted(range(len(results["graph_tuned"])), key=lambda i: probs[i].points)[:checked]
    oracle_rel = {}
    if with_oracle:
        for i in check_ids:
            plain, corrected = _oracle_pair(probs[i])
            oracle_rel[i] = (plain, corrected)
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
    rel64 = {i: _rel(results["graph_tuned"][i].cpu().numpy(), oracle_rel[i][1]) for i in oracle_rel}
    rel32 = {i: _rel(results["graph_fp32"][i].cpu().numpy(), oracle_rel[i][1]) for i in oracle_rel}
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
            "rel_l2_vs_oracle_corrected": {f"instance {i} {probs[i].nx}x{probs[i].ny}x{probs[i].nz} "
                                           f"{','.join(probs[i].bcs)}": v for i, v in rel64.items()},
            "fp32_refined": {"single_ms": round(ms["single_fp32"], 4),
                             "graph_ms": round(ms["graph_fp32"], 4),
                             "graph_points_per_s": points / (ms["graph_fp32"] * 1e-3),
                             "speedup_vs_single": round(ms["single_fp32"] / ms["graph_fp32"], 4),
                             "fp32_solves": [min(solves), max(solves)],
                             "max_rel_diff_vs_single": diff32,
                             "max_rel_l2_vs_fp64": err32, "tolerance": 1e-10,
                             "rel_l2_vs_oracle_corrected": {f"instance {i}": v for i, v in rel32.items()}}}


def projection(log, refs=None, with_oracle=True, steps=10, warmup=2):
    """One pressure-correction step on the channel grid (512 x 256 x 192,
    periodic x/y, walls in z): projection_rhs (32 B per cell: three face
    arrays read, the right-hand side written), the FP64 solve (80 B per
    cell) and projection_update (72 B per cell: Phi, the face arrays and p
    read, the face arrays and p written), timed with events on one stream."""
    import torch
    from . import Plan, inputs
    prob = inputs.channel(0)
    N = prob.points
    u, v, w = inputs.prediction_velocity(prob, 5)
    src = [torch.from_numpy(a).cuda() for a in (u, v, w)]
    p0 = torch.from_numpy(np.random.default_rng(6).uniform(-1, 1, prob.shape)).cuda()
    work = [a.clone() for a in src]
    pres = p0.clone()
    phi = torch.empty(N, dtype=torch.float64, device="cuda")
    plan = Plan.from_problem(prob)
    gdt = 0.01
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.pressure_correction(*work, pres, gdt, phi)
    times = {"rhs": [], "solve": [], "update": []}
    for _ in range(steps):
        for a, b in zip(work, src):
            a.copy_(b)
        pres.copy_(p0)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(stream)
        plan.projection_rhs(*work, gdt, phi)
        ev[1].record(stream)
        plan.solve(phi)
        ev[2].record(stream)
        plan.projection_update(phi, gdt, *work, pres)
        ev[3].record(stream)
        torch.cuda.synchronize()
        for k, name in enumerate(("rhs", "solve", "update")):
            times[name].append(ev[k].elapsed_time(ev[k + 1]))
    ms = {k: float(np.median(t)) for k, t in times.items()}
    total = sum(ms.values())
    out = {"workload": "pressure-correction step on the channel grid 512x256x192 (P,P,NN; tanh z)",
           "points": N, "rhs_ms": round(ms["rhs"], 4), "solve_ms": round(ms["solve"], 4),
           "update_ms": round(ms["update"], 4), "step_ms": round(total, 4),
           "points_per_s": N / (total * 1e-3),
           "rhs_GBs": round(32.0 * N / (ms["rhs"] * 1e-3) / 1e9, 1),
           "update_GBs": round(72.0 * N / (ms["update"] * 1e-3) / 1e9, 1),
           "fused": False}
    if with_oracle:
        from oracle import projection as pj
        ref = pj.pressure_correction(u, v, w, p0.cpu().numpy(), gdt, prob.hx, prob.hy, prob.hz,
                                     prob.bcs)
        got = [a.cpu().numpy() for a in work] + [pres.cpu().numpy()]
        out["rel_l2_vs_oracle"] = max(_rel(g.reshape(r.shape), r) for g, r in zip(got, ref[:4]))
        div = torch.empty_like(phi)
        plan.projection_rhs(*work, 1.0, div)
        out["divergence_after_over_before"] = float(
            np.linalg.norm(div.cpu().numpy())
            / np.linalg.norm(pj.divergence(u, v, w, prob.hx, prob.hy, prob.hz, prob.bcs)))
    plan.close()
    log(f"[forms] projection step (channel): rhs {ms['rhs']:.4f} ms, solve {ms['solve']:.4f} ms, "
        f"update {ms['update']:.4f} ms; rel-L2 vs oracle {out.get('rel_l2_vs_oracle', float('nan')):.2e}")
    return out


def helmholtz(log, refs=None, with_oracle=True, steps=10, warmup=2):
    """FP64 Helmholtz solves, shift -2/(nu dt) = -2e4 (a Crank-Nicolson
    step): (a) 512 x 256 x 191, periodic x/y, node Dirichlet pair along z
    (uniform, Lz = 2): the transforms are the channel's, the elimination
    runs on node rows; (b) 255 x 256 x 192, node Dirichlet pair along x
    (DST-I through the size-generic transform), periodic y, walls in z."""
    import torch
    from . import Plan, inputs
    out = {}
    for name, shape, bcs, lengths in (
            ("channel_w", (512, 256, 191), ("P", "P", "DDn"), (4 * np.pi, 2 * np.pi, 2.0 * 191 / 192)),
            ("node_x", (255, 256, 192), ("DDn", "P", "DD"), (1.0, 1.0, 1.0))):
        prob = inputs.make_uniform(*shape, bcs, seed=7, lengths=lengths)
        prob.shift = -2.0e4
        N = prob.points
        src = torch.from_numpy(prob.rhs).cuda()
        work = torch.empty_like(src)
        plan = Plan.from_problem(prob)

        def run():
            work.copy_(src)
            plan.solve(work)

        for _ in range(warmup):
            run()
        copy_ms = float(np.median(_timed(lambda: work.copy_(src), steps, torch)))
        t = float(np.median(_timed(run, steps, torch))) - copy_ms
        run()
        torch.cuda.synchronize()
        res = {"shape": list(shape), "bcs": list(bcs), "shift": prob.shift, "roles": "".join(plan.roles),
               "ms": round(t, 4), "points_per_s": N / (t * 1e-3),
               "hbm_effective_frac": round(80.0 * N / (t * 1e-3) / 8e12, 4)}
        if with_oracle:
            import oracle
            ref = oracle.solve(prob.rhs, prob.hx, prob.hy, prob.hz, *prob.bcs, shift=prob.shift)
            res["rel_l2_vs_oracle"] = _rel(work.cpu().numpy(), ref)
        plan.close()
        out[name] = res
        log(f"[forms] helmholtz {name} {shape} {bcs}: {t:.4f} ms, rel-L2 vs oracle "
            f"{res.get('rel_l2_vs_oracle', float('nan')):.2e}")
    return out


def taylor_green(log, refs=None, with_oracle=True, steps=5, warmup=1):
    """One Runge-Kutta time step of the 512^3 Taylor-Green vortex (Re 1600,
    tri-periodic 2 pi box, dt at 0.9 of the stability bound), FP64, timed
    with events on one stream: the step as rk3_step runs it (each
    projection applied by the next prediction), and substep by substep
    through the entry points for the split (prediction with the right-hand
    side, solve, update).  Checks: the energy budget of the start (dE/dt = -6 nu E)
    and the divergence after the step, at full size on the GPU's result,
    and one 64^3 step against the oracle."""
    import torch
    from . import Plan, inputs
    n = 512
    u, v, w, p, d = inputs.taylor_green(n)
    N = n ** 3
    nu = 1.0 / 1600
    vmax = float(np.max(np.abs(u) + np.abs(v)))          # w = 0 at the start
    dt = 0.9 * min(1.65 * d * d / nu, math.sqrt(3.0) * d / vmax)
    plan = Plan(n, n, n, d, d, d, ("P", "P", "P"))
    vel0 = torch.from_numpy(np.concatenate([u.reshape(-1), v.reshape(-1), w.reshape(-1)])).cuda()
    p0 = torch.from_numpy(p.reshape(-1)).cuda()
    e0 = 0.5 * float(torch.sum(vel0 * vel0))
    del u, v, w, p
    vel, pres = vel0.clone(), p0.clone()
    work = torch.empty_like(vel0)
    ad = torch.zeros(2 * vel0.numel(), dtype=torch.float64, device="cuda")   # two AD buffers
    phi = torch.empty_like(p0)
    scratch = torch.empty(2 * N, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    # the first step from the start, for the checks
    plan.rk3_step(dt, nu, vel, work, ad, pres, phi, scratch)
    torch.cuda.synchronize()
    e1 = 0.5 * float(torch.sum(vel * vel))
    plan.projection_rhs(vel[:N], vel[N:2 * N], vel[2 * N:], 1.0, phi)
    div_rel = float(torch.max(torch.abs(phi))) / (float(torch.max(torch.abs(vel))) / d)
    for _ in range(warmup):
        plan.rk3_step(dt, nu, vel, work, ad, pres, phi, scratch)
    fused = []
    for _ in range(steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        plan.rk3_step(dt, nu, vel, work, ad, pres, phi, scratch)
        ev[1].record(stream)
        torch.cuda.synchronize()
        fused.append(ev[0].elapsed_time(ev[1]))
    # substep by substep (each projection in a sweep of its own), for the split
    sub = {1: [], 2: [], 3: []}
    for _ in range(steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(stream)
        for k in (1, 2, 3):
            plan.rk3_substep(k, dt, nu, vel, work, ad, pres, phi)
            ev[k].record(stream)
        torch.cuda.synchronize()
        for k in (1, 2, 3):
            sub[k].append(ev[k - 1].elapsed_time(ev[k]))
    # the same substeps through the component entry points, one event per
    # kernel sweep: prediction (+ right-hand side), solve, update (in place
    # on u*, which then serves as the velocity: the same arithmetic)
    parts = {(k, name): [] for k in (1, 2, 3) for name in ("predict", "solve", "update")}
    for _ in range(steps):
        for k in (1, 2, 3):
            gdt = dt * (ALPHA[k - 1] + BETA[k - 1])
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            ev[0].record(stream)
            plan.rk3_predict(k, dt, nu, vel, work, ad, pres, phi)
            ev[1].record(stream)
            plan.solve(phi)
            ev[2].record(stream)
            plan.projection_update(phi, gdt, work[:N], work[N:2 * N], work[2 * N:], pres)
            ev[3].record(stream)
            vel, work = work, vel
            torch.cuda.synchronize()
            for i, name in enumerate(("predict", "solve", "update")):
                parts[(k, name)].append(ev[i].elapsed_time(ev[i + 1]))
    pm_ = {key: float(np.median(t)) for key, t in parts.items()}
    solve_ms = float(np.median([pm_[(k, "solve")] for k in (1, 2, 3)]))
    ms = {k: float(np.median(t)) for k, t in sub.items()}
    step = float(np.median(fused))
    predict_bytes = {1: 88.0, 2: 112.0, 3: 88.0}
    out = {"workload": "RK3 step, Taylor-Green vortex 512^3 (P,P,P), Re 1600, FP64",
           "points": N, "dt": dt, "step_ms": round(step, 4),
           "step": "rk3_step: the projections of substeps 1 and 2 applied by the next prediction",
           "substep_by_substep_ms": round(sum(ms.values()), 4),
           "substep_ms": [round(ms[k], 4) for k in (1, 2, 3)],
           "solve_ms": round(solve_ms, 4),
           "around_solve_ms": round(step - 3 * solve_ms, 4),
           "cell_steps_per_s": N / (step * 1e-3),
           "kernels": [{"substep": k, "predict_ms": round(pm_[(k, "predict")], 4),
                        "predict_GBs": round(predict_bytes[k] * N / (pm_[(k, "predict")] * 1e-3) / 1e9, 1),
                        "solve_ms": round(pm_[(k, "solve")], 4),
                        "solve_GBs": round(80.0 * N / (pm_[(k, "solve")] * 1e-3) / 1e9, 1),
                        "update_ms": round(pm_[(k, "update")], 4),
                        "update_GBs": round(72.0 * N / (pm_[(k, "update")] * 1e-3) / 1e9, 1)}
                       for k in (1, 2, 3)],
           "bytes_per_cell": "prediction + right-hand side 88 / 112 / 88 (substeps 1 / 2 / 3), "
                             "solve 80, update 72",
           "energy_rate_over_minus_6nu": (e1 - e0) / (dt * e0) / (-6 * nu),
           "divergence_after_step": div_rel}
    del vel, work, ad, pres, phi, vel0, p0
    plan.close()
    torch.cuda.empty_cache()
    if with_oracle:
        from oracle import navier_stokes as ns
        m = 64
        u, v, w, p, dm = inputs.taylor_green(m)
        dtm = 0.9 * ns.stable_dt(u, v, w, dm, dm, dm, nu)
        pm = Plan(m, m, m, dm, dm, dm, ("P", "P", "P"))
        dv = torch.from_numpy(np.concatenate([u.reshape(-1), v.reshape(-1), w.reshape(-1)])).cuda()
        dp = torch.from_numpy(p.reshape(-1).copy()).cuda()
        pm.rk3_step(dtm, nu, dv, torch.empty_like(dv), torch.zeros(2 * dv.numel(), dtype=dv.dtype,
                                                                    device="cuda"), dp,
                    torch.empty_like(dp), torch.empty(2 * m ** 3, dtype=dv.dtype, device="cuda"))
        ref = ns.rk3_step(u, v, w, p, dtm, nu, dm, dm, dm)
        got = dv.cpu().numpy().reshape(3, m, m, m)
        out["rel_l2_vs_oracle_64"] = max([_rel(got[c], ref[c]) for c in range(3)]
                                         + [_rel(dp.cpu().numpy().reshape(p.shape), ref[3])])
        pm.close()
    for kk in out["kernels"]:
        log(f"[forms]   substep {kk['substep']}: predict {kk['predict_ms']:.3f} ms "
            f"({kk['predict_GBs']} GB/s), solve {kk['solve_ms']:.3f} ms ({kk['solve_GBs']} GB/s), "
            f"update {kk['update_ms']:.3f} ms ({kk['update_GBs']} GB/s)")
    log(f"[forms] Taylor-Green 512^3 RK3 step: {step:.3f} ms (substep by substep "
        f"{ms[1]:.3f}/{ms[2]:.3f}/{ms[3]:.3f} ms, solve {solve_ms:.3f} ms each); energy rate "
        f"{out['energy_rate_over_minus_6nu']:.6f} x (-6 nu); divergence {div_rel:.1e}; "
        f"64^3 rel-L2 vs oracle {out.get('rel_l2_vs_oracle_64', float('nan')):.2e}")
    return out


def _serve_once(log, specs, order, slots, load, seed, window):
    """One server with `slots` streams: warm-up (every spec of the catalogue
    once, so every plan is cached), a closed loop over the timed requests
    (at most `window` outstanding) for the capacity, then the same requests
    as Poisson arrivals at `load` x capacity.  Each request's field is
    written (seeded uniform values) on the caller's stream just before it is
    submitted, and released when it completes."""
    import torch
    from . import FP32_REFINED, FP64, Server
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    srv = Server(slots=slots)

    def submit(k, fields):
        sp = specs[k]
        f = torch.empty(sp.points, dtype=torch.float64, device="cuda")
        f.uniform_(-1.0, 1.0, generator=gen)
        rid = srv.submit(sp, f, FP32_REFINED if sp.mixed else FP64, 1e-10, 6)
        fields[rid] = f
        return rid

    fields = {}
    warm = [submit(k, fields) for k in range(len(specs))]
    for rid in warm:
        srv.wait(rid)
        fields.pop(rid)
    st0 = srv.stats()
    points = sum(specs[k].points for k in order)
    count = len(order)

    # closed loop: `window` requests outstanding
    t0 = time.perf_counter()
    pending = []
    infos = []
    for k in order:
        if len(pending) >= window:
            rid = pending.pop(0)
            infos.append(srv.wait(rid))
            fields.pop(rid)
        pending.append(submit(k, fields))
    for rid in pending:
        infos.append(srv.wait(rid))
        fields.pop(rid)
    closed_s = time.perf_counter() - t0
    capacity = count / closed_s
    bad = sum(1 for x in infos if x["status"] != 0)

    # open loop: Poisson arrivals; a second thread waits for completions
    rng = np.random.default_rng(seed + 1)
    arrivals = np.cumsum(rng.exponential(1.0 / (load * capacity), count))
    ids = []
    done = []
    lock = threading.Lock()
    ready = threading.Semaphore(0)

    def waiter():
        for _ in range(count):
            ready.acquire()
            with lock:
                rid = ids[len(done)]
            info = srv.wait(rid)
            with lock:
                done.append(info)
                fields.pop(rid, None)

    th = threading.Thread(target=waiter)
    th.start()
    t0 = time.perf_counter()
    for a, k in zip(arrivals, order):
        while time.perf_counter() - t0 < a:
            pass
        rid = submit(k, fields)
        with lock:
            ids.append(rid)
        ready.release()
    th.join()
    lat = np.array([x["done_s"] - x["submit_s"] for x in done]) * 1e3
    queue = np.array([x["start_s"] - x["submit_s"] for x in done]) * 1e3
    span = max(x["done_s"] for x in done) - min(x["submit_s"] for x in done)
    bad += sum(1 for x in done if x["status"] != 0)
    st1 = srv.stats()
    use = srv.usage()
    srv.close()
    out = {"slots": slots, "requests": count, "warmup": len(specs), "points": points,
           "closed_loop_window": window,
           "closed_loop_req_per_s": capacity, "closed_loop_points_per_s": points / closed_s,
           "arrival_rate_req_per_s": load * capacity,
           "achieved_req_per_s": count / span, "achieved_load": count / span / capacity,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "mean_queue_ms": float(queue.mean()), "open_loop_points_per_s": points / span,
           "failed": bad,
           "plan_misses_warmup": st0["plan_misses"],
           "plan_misses_timed": st1["plan_misses"] - st0["plan_misses"],
           "plans_resident": st1["plans_resident"], "hbm_budget": st1["hbm_budget"],
           "server_peak_bytes": use["peak_bytes"]}
    log(f"[forms] serve, {slots} slots: capacity {capacity:.1f} req/s ({points / closed_s:.3e} "
        f"points/s); at {out['achieved_load']:.0%} of it: p50 {out['p50_ms']:.3f} ms, p99 "
        f"{out['p99_ms']:.3f} ms; plan misses {out['plan_misses_warmup']} warm-up, "
        f"{out['plan_misses_timed']} timed")
    return out


def serve(log, refs=None, with_oracle=True, count=2000, catalogue=200, seed=0,
          slot_counts=(2, 4, 8), load=0.8, sample=8):
    """Served stream: a catalogue of `catalogue` request kinds (per-axis n
    log-uniform in [32, 512] snapped to even 2^a 3^b 5^c, random boundary
    pairs, z stretched with probability 1/2 when walled, FP64 or FP32 +
    refinement to 1e-10 with probability 1/2); `count` timed requests drawn
    from it at random after a warm-up of one request per kind.  Measured for
    each slot count.  Then `sample` small requests with host-generated
    fields are served in the middle of a burst of others and compared with
    the oracle and with solo solves."""
    import torch
    from . import FP32_REFINED, FP64, Plan, Server, inputs
    specs = [inputs.served_request(seed, i, with_rhs=False) for i in range(catalogue)]
    order = np.random.default_rng(seed + 7).integers(0, catalogue, count).tolist()
    runs = [_serve_once(log, specs, order, s, load, seed, window=2 * s) for s in slot_counts]

    # correctness: sampled requests (host fields) inside a burst of others
    small_specs = [i for i in range(catalogue) if specs[i].points <= 400_000][:sample]
    probs = [inputs.served_request(seed, i) for i in small_specs]
    srv = Server(slots=max(slot_counts))
    burst = []
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed + 3)
    for k in range(16):
        sp = specs[order[k]]
        f = torch.empty(sp.points, dtype=torch.float64, device="cuda").uniform_(-1, 1, generator=gen)
        burst.append((srv.submit(sp, f, FP32_REFINED if sp.mixed else FP64, 1e-10, 6), f))
    fields = [torch.from_numpy(p.rhs).cuda() for p in probs]
    ids = [srv.submit(p, f, FP32_REFINED if p.mixed else FP64, 1e-10, 6)
           for p, f in zip(probs, fields)]
    for rid, _ in burst:
        srv.wait(rid)
    infos = [srv.wait(r) for r in ids]
    srv.close()
    same, rel_max = True, {"fp64": 0.0, "fp32_refined": 0.0}
    for p, f, info in zip(probs, fields, infos):
        got = f.cpu().numpy()
        plan = Plan.from_problem(p)
        if p.mixed:
            plan.set_precision(FP32_REFINED, 1e-10, 6)
        solo = torch.from_numpy(p.rhs).cuda()
        plan.solve(solo)
        torch.cuda.synchronize()
        same = same and np.array_equal(solo.cpu().numpy(), got) and info["status"] == 0
        plan.close()
        if with_oracle:
            _, corrected = _oracle_pair(p)
            key = "fp32_refined" if p.mixed else "fp64"
            rel_max[key] = max(rel_max[key], _rel(got, corrected))
    out = {"workload": f"served stream, {catalogue} request kinds (per-axis n log-uniform "
                       "[32, 512], random BC pairs, FP64 or FP32+IR (1e-10) with p = 1/2), "
                       f"{count} timed requests drawn from them after one warm-up request "
                       "per kind; each field written on the caller's stream just before "
                       "submission",
           "runs": runs, "sampled": len(probs), "sampled_equal_to_solo": bool(same)}
    if with_oracle:
        out["sampled_max_rel_l2_vs_oracle_corrected"] = rel_max
    log(f"[forms] serve: {len(probs)} sampled requests equal to solo solves: {same}; "
        f"max rel-L2 vs oracle {rel_max}")
    return out


def run(wanted, log, refs=None, with_oracle=True):
    out = {}
    for name, fn in (("mixed", mixed), ("channel", channel), ("small", small),
                     ("projection", projection), ("helmholtz", helmholtz),
                     ("taylor_green", taylor_green), ("batch", batch), ("serve", serve)):
        if name in wanted:
            out[name] = fn(log, refs, with_oracle)
    return out
