"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs.  Tolerance: relative L2 <= 1e-12 for the plain FP64
solve, <= 1e-10 for FP32 + FP64 refinement; transform and elimination stages
<= 1e-13 relative.  Shapes span several tiles and ragged tails; edge cases
cover n = 1/2/3, singular problems with an incompatible right-hand side,
zero input, and the largest supported lengths."""
import itertools
import sys

import numpy as np
import pytest

from gpu_util import AXIS, check_elimination, gpu_solve, oracle_solve, rel_l2, to_dev, to_host
from paper_1802_10323_amd import inputs

pytestmark = pytest.mark.gpu

KINDS = ("P", "NN", "DD", "ND", "DN")
TOL64 = 1e-12
FAST_M = [16, 32, 48, 64, 72, 80, 96, 128, 144, 160, 192, 256]
ELIM_LENGTHS = [64, 96, 128, 192, 256, 384, 512]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_10323_amd import lib
    lib()


# --------------------------------------------------------------- stages

STAGE_CASES = [
    ((48, 40, 30), ("P", "P", "NN"), True),
    ((64, 36, 20), ("NN", "DD", "ND"), False),
    ((40, 50, 24), ("DN", "ND", "P"), False),     # z periodic uniform: s = x
    ((33, 24, 20), ("DD", "P", "P"), False),      # s = x with odd length
    ((20, 31, 16), ("P", "ND", "P"), False),      # s = y
    ((16, 12, 10), ("P", "P", "P"), False),       # all periodic: cyclic s = x
    ((16, 12, 10), ("P", "P", "P"), True),        # cyclic s = z, stretched
    ((16, 12, 14), ("P", "P", "P"), False),       # z has no DFT (n/2 = 7): cyclic s = z
]


@pytest.mark.parametrize("shape,bcs,stretched", STAGE_CASES)
def test_stages_match_oracle(shape, bcs, stretched):
    import oracle
    from oracle import transforms as tr
    from oracle.poisson import tridiagonal_stage
    from paper_1802_10323_amd import Plan
    nx, ny, nz = shape
    say("stages", shape, bcs, stretched)
    prob = inputs.make_uniform(nx, ny, nz, bcs, seed=sum(shape), stretch_z=1.8 if stretched else None)
    plan = Plan.from_problem(prob)
    t1, t2, s = plan.roles
    h = {"x": prob.hx, "y": prob.hy, "z": prob.hz}
    bc = dict(zip("xyz", bcs))
    f = prob.rhs
    # forward t1
    ref1 = tr.forward(f, AXIS[t1], bc[t1])
    d = to_dev(f)
    plan.transform_stage(0, False, d)
    g1 = to_host(d)
    assert rel_l2(g1, ref1) <= 1e-13
    # forward t2 (applied to the oracle's t1 output)
    ref2 = tr.forward(ref1, AXIS[t2], bc[t2])
    d = to_dev(ref1)
    plan.transform_stage(1, False, d)
    assert rel_l2(to_host(d), ref2) <= 1e-13
    # elimination
    lam1 = tr.eigenvalues(bc[t1], f.shape[AXIS[t1]]) / h[t1][0] ** 2
    lam2 = tr.eigenvalues(bc[t2], f.shape[AXIS[t2]]) / h[t2][0] ** 2
    singular = oracle.is_singular(*bcs)
    ref3 = tridiagonal_stage(ref2, s, h[s], bc[s], lam1, lam2, t1, t2, singular)
    d = to_dev(ref2)
    plan.tridiag_stage(d)
    assert rel_l2(to_host(d), ref3) <= 1e-12
    # backward t2 then t1
    ref4 = tr.backward(ref3, AXIS[t2], bc[t2])
    d = to_dev(ref3)
    plan.transform_stage(1, True, d)
    assert rel_l2(to_host(d), ref4) <= 1e-13
    ref5 = tr.backward(ref4, AXIS[t1], bc[t1])
    d = to_dev(ref4)
    plan.transform_stage(0, True, d)
    assert rel_l2(to_host(d), ref5) <= 1e-13
    plan.close()


@pytest.mark.parametrize("path", ["specialised", "generic"])
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", [2, 4, 6, 10, 18, 30, 32, 50, 64, 96, 128, 144, 160, 192, 240, 250,
                               256, 288, 320, 384, 480, 512, 1024])
def test_transform_lengths(kind, n, path, monkeypatch):
    """Every supported transform length class on the contiguous (x) and the
    strided (y) axis, against the Table 2 sums; round trip is the identity.
    Lengths 2M with M in {16, 32, 48, 64, 72, 80, 96, 128, 144, 160, 192,
    256} have size-specialised kernels; the generic kernel is run on them
    too."""
    from oracle import transforms as tr
    from paper_1802_10323_amd import Plan
    if path == "generic":
        monkeypatch.setenv("POISSON_GENERIC_R2R", "1")
    rng = np.random.default_rng(n)
    # walls on z make z the elimination axis, so x is role 0 and y role 1
    for axis_name, shape in (("x", (3, 6, n)), ("y", (3, n, 8))):
        f = rng.uniform(-1, 1, shape)
        nz, ny, nx = shape
        bcx, bcy = (kind, "P") if axis_name == "x" else ("P", kind)
        plan = Plan(nx, ny, nz, 1.0, 1.0, np.ones(nz), (bcx, bcy, "DD"))
        assert plan.roles == ("x", "y", "z")
        role = 0 if axis_name == "x" else 1
        d = to_dev(f)
        plan.transform_stage(role, False, d)
        got = to_host(d)
        ref = tr.forward(f, AXIS[axis_name], kind)
        assert rel_l2(got, ref) <= 1e-13, (axis_name, kind, n)
        plan.transform_stage(role, True, d)
        assert rel_l2(to_host(d), f) <= 1e-13
        plan.close()


@pytest.mark.parametrize("path", ["specialised", "generic"])
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", ELIM_LENGTHS)
def test_elimination_lengths(n, kind, path, monkeypatch):
    if path == "generic":
        monkeypatch.setenv("POISSON_GENERIC_TRI", "1")
    check_elimination(n, kind)


# --------------------------------------------------------------- whole solve

@pytest.mark.parametrize("stretched", [False, True])
def test_all_125_triples(stretched):
    worst = 0.0
    for t, bcs in enumerate(itertools.product(KINDS, repeat=3)):
        prob = inputs.make_uniform(12, 10, 9 if bcs[2] != "P" else 8, bcs, seed=t,
                                   stretch_z=1.8 if (stretched and bcs[2] != "P") else None)
        got, _ = gpu_solve(prob)
        ref = oracle_solve(prob)
        err = rel_l2(got, ref)
        worst = max(worst, err)
        assert err <= TOL64, (bcs, err)
    say("125 triples worst rel-L2", worst)


RAGGED = [
    ((96, 40, 33), ("P", "P", "NN"), True),
    ((50, 64, 47), ("NN", "DN", "DD"), True),
    ((34, 30, 40), ("DD", "ND", "P"), False),
    ((45, 36, 20), ("DD", "P", "P"), False),
    ((40, 60, 36), ("P", "P", "P"), False),
    ((160, 20, 4), ("P", "NN", "P"), False),
    ((4, 6, 3), ("P", "P", "P"), False),
    ((24, 18, 1), ("NN", "NN", "NN"), False),
    ((20, 2, 2), ("P", "P", "DN"), False),
    ((2, 2, 6), ("NN", "NN", "P"), False),
]


@pytest.mark.parametrize("shape,bcs,stretched", RAGGED)
def test_solve_ragged_shapes(shape, bcs, stretched):
    say("ragged", shape, bcs)
    prob = inputs.make_uniform(*shape, bcs, seed=7, stretch_z=1.8 if stretched else None)
    got, _ = gpu_solve(prob)
    assert rel_l2(got, oracle_solve(prob)) <= TOL64


def test_small_config():
    prob = inputs.small(0)
    got, _ = gpu_solve(prob)
    err = rel_l2(got, oracle_solve(prob))
    say("small 32^3 rel-L2", err)
    assert err <= TOL64


def test_singular_projection_and_gauge():
    """An incompatible right-hand side (nonzero weighted mean) is projected:
    the result equals the oracle's and has zero weighted mean."""
    import oracle
    prob = inputs.make_uniform(24, 20, 18, ("P", "NN", "NN"), seed=3, stretch_z=1.8)
    prob.rhs = prob.rhs + 0.75
    got, _ = gpu_solve(prob)
    assert rel_l2(got, oracle_solve(prob)) <= TOL64
    assert abs(oracle.weighted_mean(got, prob.hx, prob.hy, prob.hz)) <= 1e-14 * np.abs(got).max()


def test_zero_rhs_gives_zero():
    prob = inputs.make_uniform(16, 16, 16, ("DD", "P", "NN"), seed=1)
    prob.rhs = np.zeros_like(prob.rhs)
    got, _ = gpu_solve(prob)
    assert np.all(got == 0.0)


def test_largest_lengths():
    prob = inputs.make_uniform(1024, 6, 512, ("ND", "P", "DD"), seed=2, stretch_z=1.8)
    got, _ = gpu_solve(prob)
    assert rel_l2(got, oracle_solve(prob)) <= TOL64


# --------------------------------------------------------------- full-size workloads

def test_channel_full_size():
    """The channel workload at its full size (512 x 256 x 192, tanh z)."""
    prob = inputs.channel(0)
    say("channel full size")
    got, _ = gpu_solve(prob)
    ref = oracle_solve(prob)
    err = rel_l2(got, ref)
    say("channel rel-L2", err)
    assert err <= TOL64


# --------------------------------------------------------------- precision

@pytest.mark.parametrize("shape,bcs,stretched", [
    ((64, 64, 64), ("DD", "ND", "P"), False),
    ((48, 40, 36), ("P", "P", "NN"), True),
    ((40, 36, 30), ("NN", "NN", "NN"), False),
    ((32, 30, 28), ("P", "P", "P"), False),
    ((128, 96, 192), ("P", "P", "NN"), True),
    ((256, 20, 64), ("DD", "P", "P"), False),
    ((64, 512, 24), ("P", "DN", "DD"), True),
])
def test_mixed_precision_refinement(shape, bcs, stretched):
    prob = inputs.make_uniform(*shape, bcs, seed=5, stretch_z=1.8 if stretched else None)
    got, (iters, rel, conv) = gpu_solve(prob, mixed=True, tol=1e-10, max_iters=6)
    err = rel_l2(got, oracle_solve(prob))
    say("mixed", shape, bcs, "iters", iters, "last update", rel, "rel-L2", err)
    assert conv
    assert err <= 1e-10
    assert iters <= 4


def test_mixed_precision_not_converged_flag():
    prob = inputs.make_uniform(32, 32, 32, ("DD", "ND", "P"), seed=6)
    got, (iters, rel, conv) = gpu_solve(prob, mixed=True, tol=1e-30, max_iters=2)
    assert iters == 2 and not conv


# --------------------------------------------------------------- batch

def test_batch_equals_single_solves():
    from paper_1802_10323_amd import Plan, batch_solve
    probs = inputs.batch(0, count=6, sizes=(16, 24, 30, 40))
    plans = [Plan.from_problem(p) for p in probs]
    fields = [to_dev(p.rhs) for p in probs]
    batch_solve(plans, fields)
    for p, f in zip(probs, fields):
        got = to_host(f)
        single, _ = gpu_solve(p)
        assert np.array_equal(got, single)
        assert rel_l2(got, oracle_solve(p)) <= TOL64
    for pl in plans:
        pl.close()


def _batch_case(seed, count):
    probs = inputs.batch(seed, count=count)
    return probs


def _synchronous_variants():
    """The batched kernels have the synchronous transform variants only:
    make single solves use variant 0 for the lengths whose default is the
    staging form, so that both run the same arithmetic."""
    from paper_1802_10323_amd import set_tuned_variant
    for fp64 in (True, False):
        for layout in (0, 1):
            for n in (256, 512):
                set_tuned_variant(0, n, layout, 0, fp64)


def test_persistent_batch_equals_single_solves(default_variants):
    """One persistent launch per stage over uneven instances (sizes from
    {64, ..., 256} per axis, random boundary pairs, stretched and uniform z):
    bitwise equal to single solves with the same kernel variants, within
    1e-14 of single solves with the default ones (staging transforms for
    length 256), and within 1e-12 of the oracle."""
    from paper_1802_10323_amd import Batch, Plan
    probs = _batch_case(1, 10)
    say("batch shapes", [p.shape for p in probs])
    plans = [Plan.from_problem(p) for p in probs]
    fields = [to_dev(p.rhs) for p in probs]
    batch = Batch(plans)
    batch.bind(fields)
    batch.launch()
    got = [to_host(f) for f in fields]
    defaults = [gpu_solve(p)[0] for p in probs]
    _synchronous_variants()
    for p, g, d in zip(probs, got, defaults):
        single, _ = gpu_solve(p)
        assert np.array_equal(g, single), p
        assert rel_l2(g, d) <= 1e-14, p
        assert rel_l2(g, oracle_solve(p)) <= TOL64, p
    batch.close()
    for pl in plans:
        pl.close()


def test_persistent_batch_graph_replays():
    """The HIP-graph form: several replays with eager work (refills, host
    synchronisations) between them, then a re-bind to other fields without
    re-capture; every replay equals the eager batched launch bit for bit."""
    import torch
    from paper_1802_10323_amd import Batch, Plan
    probs = _batch_case(2, 6)
    plans = [Plan.from_problem(p) for p in probs]
    src = [to_dev(p.rhs) for p in probs]
    eager = [s.clone() for s in src]
    batch = Batch(plans)
    batch.bind(eager)
    batch.launch(graph=False)
    ref = [to_host(f) for f in eager]
    work = [torch.empty_like(s) for s in src]
    batch.bind(work)
    for rep in range(3):
        for w, s in zip(work, src):
            w.copy_(s)
        torch.cuda.synchronize()
        batch.launch(graph=True)
        for w, r in zip(work, ref):
            assert np.array_equal(to_host(w), r), rep
        _ = torch.ones(1000, device="cuda").sum().item()     # eager work between replays
    other = [s.clone() for s in src]
    batch.bind(other)
    batch.launch(graph=True)
    for o, r in zip(other, ref):
        assert np.array_equal(to_host(o), r)
    batch.close()
    for pl in plans:
        pl.close()


def test_batch_rejects_unspecialised_lengths_and_batch_solve_falls_back():
    from paper_1802_10323_amd import Batch, Plan, PoissonError, batch_solve
    probs = inputs.batch(3, count=4, sizes=(16, 24, 30, 40))
    plans = [Plan.from_problem(p) for p in probs]
    with pytest.raises(PoissonError):
        Batch(plans)
    fields = [to_dev(p.rhs) for p in probs]
    batch_solve(plans, fields)
    for p, f in zip(probs, fields):
        assert rel_l2(to_host(f), oracle_solve(p)) <= TOL64
    for pl in plans:
        pl.close()


# --------------------------------------------------------------- served

def _solo(prob, field):
    """The request solved on its own, with a fresh plan, on the default stream."""
    from paper_1802_10323_amd import FP32_REFINED, Plan
    plan = Plan.from_problem(prob)
    if getattr(prob, "mixed", False):
        plan.set_precision(FP32_REFINED, 1e-10, 6)
    plan.solve(field)
    out = to_host(field)
    st = plan.status()
    plan.close()
    return out, st


def _solo_prec(prob, field, precision):
    from paper_1802_10323_amd import FP32_REFINED, Plan
    plan = Plan.from_problem(prob)
    if precision == FP32_REFINED:
        plan.set_precision(FP32_REFINED, 1e-10, 6)
    plan.solve(field)
    out = to_host(field)
    st = plan.status()
    plan.close()
    return out, st


def test_server_results_equal_solo_solves():
    """Requests of mixed sizes, boundary pairs and precisions submitted at
    once run concurrently on the server's streams; each result equals the
    same request solved alone, bit for bit (FP64 and FP32 + refinement), and
    the small ones match the oracle within their tolerance."""
    from paper_1802_10323_amd import FP32_REFINED, FP64, Server
    probs = [inputs.served_request(5, i, lo=32, hi=160) for i in range(14)]
    say("served", [(p.shape, p.bcs, p.mixed) for p in probs])
    inputs_dev = [to_dev(p.rhs) for p in probs]
    fields = [f.clone() for f in inputs_dev]
    srv = Server(slots=4)
    ids = [srv.submit(p, f, FP32_REFINED if p.mixed else FP64, 1e-10, 6)
           for p, f in zip(probs, fields)]
    infos = [srv.wait(i) for i in ids]
    for p, f, info, src in zip(probs, fields, infos, inputs_dev):
        assert info["status"] == 0, (p, info)
        got = to_host(f)
        solo, (iters, _, conv) = _solo(p, src.clone())
        assert np.array_equal(got, solo), p
        assert info["iters"] == (iters if p.mixed else 1)
        if p.points <= 200_000:
            assert rel_l2(got, oracle_solve(p)) <= (1e-10 if p.mixed else TOL64), p
    # the same problem again: its plan is reused from the cache
    again = inputs_dev[0].clone()
    rid = srv.submit(probs[0], again, FP32_REFINED if probs[0].mixed else FP64, 1e-10, 6)
    info = srv.wait(rid)
    assert info["plan_cached"] == 1
    assert np.array_equal(to_host(again), to_host(fields[0]))
    st = srv.stats()
    assert st["plan_hits"] >= 1
    srv.close()


def test_server_admission_by_hbm_budget():
    """With a budget that holds only the largest request (field plus
    refinement workspace), the fields admitted plus everything the server
    holds on the device never exceed the budget (admission waits), the
    device memory the server takes (hipMemGetInfo) stays within it, the
    results equal the solo ones, and a request larger than the budget is
    refused."""
    import torch
    from paper_1802_10323_amd import FP32_REFINED, FP64, PoissonError, Server
    probs = [inputs.served_request(6, i, lo=32, hi=96) for i in range(8)]
    for k in (1, 4):
        probs[k].mixed = True     # several refined requests: slot workspaces count
    work = [8 * p.points + ((12 * p.points + 8 * 2200) if p.mixed else 0) for p in probs]
    need = max(work) + 16 * 1024 * 1024      # + cached plans' tables
    src = [to_dev(p.rhs) for p in probs]
    fields = [f.clone() for f in src]
    srv = Server(slots=4, hbm_budget=need)
    # the runtime's own set-up of the server's streams is not the server's
    # memory: one tiny FP64 request on every slot first
    tiny = inputs.make_uniform(8, 8, 8, ("P", "P", "DD"), seed=2)
    warm = [to_dev(tiny.rhs) for _ in range(4)]
    for rid in [srv.submit(tiny, w) for w in warm]:
        srv.wait(rid)
    torch.cuda.synchronize()
    held0 = srv.usage()["held_bytes"]
    free0, _ = torch.cuda.mem_get_info()
    ids = [srv.submit(p, f, FP32_REFINED if p.mixed else FP64, 1e-10, 6)
           for p, f in zip(probs, fields)]
    infos = [srv.wait(i) for i in ids]
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    use = srv.usage()
    say("budget", need, "usage", use, "device memory taken", free0 - free1)
    assert use["peak_bytes"] <= need
    assert 0 < use["held_bytes"] <= need
    assert free0 - free1 <= need - held0
    for x in infos:
        assert x["status"] == 0, x
    for p, f, s in zip(probs, fields, src):
        solo, _ = _solo(p, s.clone())
        assert np.array_equal(to_host(f), solo)
    big = inputs.make_uniform(64, 64, 64, ("P", "P", "DD"), seed=1)
    if 8 * big.points > need:
        with pytest.raises(PoissonError):
            srv.submit(big, to_dev(big.rhs))
    srv.close()


def test_server_orders_solve_after_producer_stream():
    """A cache-hit request submitted right after an asynchronous fill of its
    field on the caller's stream (behind a long fill of another large
    buffer): the solve waits for the fill (the server's streams wait for an
    event recorded on the producer stream at submission), so the result is
    the solo one, bit for bit; also for a refined request."""
    import torch
    from paper_1802_10323_amd import FP32_REFINED, FP64, Server
    srv = Server(slots=4)
    big = torch.empty(1 << 28, dtype=torch.float64, device="cuda")     # 2 GiB
    cases = (((192, 160, 128), ("P", "P", "NN"), FP64),
             ((128, 96, 160), ("DD", "ND", "P"), FP32_REFINED))
    for k, (shape, bcs, prec) in enumerate(cases):
        prob = inputs.make_uniform(*shape, bcs, seed=40 + k)
        src = to_dev(prob.rhs)
        warm = src.clone()
        srv.wait(srv.submit(prob, warm, prec, 1e-10, 6))        # caches the plan
        solo, _ = _solo_prec(prob, src.clone(), prec)
        for _ in range(3):
            field = torch.zeros_like(src)
            torch.cuda.synchronize()
            big.uniform_(-1.0, 1.0)          # keeps the current stream busy
            field.copy_(src)                 # the request's input, written after it
            rid = srv.submit(prob, field, prec, 1e-10, 6)
            info = srv.wait(rid)
            assert info["plan_cached"] == 1 and info["status"] == 0, info
            assert np.array_equal(to_host(field), solo), (shape, bcs)
    del big
    srv.close()


# --------------------------------------------------------------- kernel variants


@pytest.mark.parametrize("V", [0, 1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("M", FAST_M)
def test_transform_variants(M, V, default_variants):
    """Every compiled transform variant (tile shape x radix order, and the
    asynchronous-staging form in both tile shapes; variant 6, FP32 only,
    falls back to variant 0 here) against the Table 2 sums, all five types,
    contiguous and strided (one partial and one multi-tile strided case, and
    an odd row length that the staging form must hand to variant 0); round
    trip is the identity."""
    from oracle import transforms as tr
    from paper_1802_10323_amd import Plan, set_tuned_variant
    n = 2 * M
    rng = np.random.default_rng(n + V)
    for layout in (0, 1):
        set_tuned_variant(0, n, layout, V)
    for kind in KINDS:
        for axis_name, shape in (("x", (3, 6, n)), ("y", (3, n, 8)), ("y", (2, n, 40)),
                                 ("y", (2, n, 7))):
            f = rng.uniform(-1, 1, shape)
            nz, ny, nx = shape
            if nx % 2:      # odd rows: x is the elimination axis, y is t1
                bcs, role = ("DD", kind, "P"), 0
            else:
                bcx, bcy = (kind, "P") if axis_name == "x" else ("P", kind)
                bcs, role = (bcx, bcy, "DD"), 0 if axis_name == "x" else 1
            plan = Plan(nx, ny, nz, 1.0, 1.0, np.ones(nz), bcs)
            assert plan.roles[role] == axis_name
            d = to_dev(f)
            plan.transform_stage(role, False, d)
            assert rel_l2(to_host(d), tr.forward(f, AXIS[axis_name], kind)) <= 1e-13, (kind, shape)
            plan.transform_stage(role, True, d)
            assert rel_l2(to_host(d), f) <= 1e-13, (kind, shape)
            plan.close()


@pytest.mark.parametrize("V", [1, 2, 3])
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", ELIM_LENGTHS)
def test_elimination_variants(n, kind, V, default_variants):
    """The second chunking (V = 1) and the staging form (V = 2) of every
    specialised elimination length, with the checks of
    test_elimination_lengths (their strided cases have an even x extent,
    so the staging form applies)."""
    from paper_1802_10323_amd import set_tuned_variant
    for layout in (0, 1):
        set_tuned_variant(1, n, layout, V)
    check_elimination(n, kind)


@pytest.mark.parametrize("vt,ve", [(1, 0), (2, 1), (3, 1)])
def test_fp32_variants_refine(vt, ve, default_variants):
    """FP32 kernels of the other variants inside the refined solve: it
    converges to the oracle within 1e-10 in at most 4 FP32 solves."""
    from paper_1802_10323_amd import set_tuned_variant
    prob = inputs.make_uniform(128, 96, 192, ("P", "P", "NN"), seed=9, stretch_z=1.8)
    for layout in (0, 1):
        set_tuned_variant(0, 128, layout, vt, fp64=False)
        set_tuned_variant(0, 96, layout, vt, fp64=False)
        set_tuned_variant(1, 192, layout, ve, fp64=False)
    got, (iters, rel, conv) = gpu_solve(prob, mixed=True, tol=1e-10, max_iters=6)
    assert conv and iters <= 4, (iters, rel)
    assert rel_l2(got, oracle_solve(prob)) <= 1e-10


@pytest.mark.parametrize("vt", [4, 5, 6])
def test_fp32_staging_variants_refine(vt, default_variants):
    """FP32 staging transforms of length 512 (all three tile shapes), on the
    contiguous axis (DCT-II) and on a strided one (DCT-IV), inside the
    refined solve: it converges to the oracle within 1e-10."""
    from paper_1802_10323_amd import set_tuned_variant
    for layout in (0, 1):
        set_tuned_variant(0, 512, layout, vt, fp64=False)
    for shape, bcs in (((512, 24, 20), ("DD", "P", "NN")), ((48, 512, 18), ("P", "ND", "DD"))):
        prob = inputs.make_uniform(*shape, bcs, seed=vt)
        got, (iters, rel, conv) = gpu_solve(prob, mixed=True, tol=1e-10, max_iters=6)
        say("fp32 staging", vt, shape, bcs, iters, rel)
        assert conv and iters <= 4, (iters, rel)
        assert rel_l2(got, oracle_solve(prob)) <= 1e-10


def test_autotune_records_fastest(default_variants):
    """plan_autotune times every variant and keeps the fastest; solves with
    the tuned table still match the oracle, and a batch built afterwards is
    still bitwise equal to single solves."""
    import torch
    from paper_1802_10323_amd import Batch, Plan, tuned_variant
    prob = inputs.make_uniform(128, 96, 192, ("P", "P", "NN"), seed=4, stretch_z=1.8)
    plan = Plan.from_problem(prob)
    scratch = torch.empty(prob.points, dtype=torch.float64, device="cuda")
    rep = plan.autotune(scratch, reps=3)
    say("autotune report", rep)
    for prec, fp64 in (("fp64", True), ("fp32", False)):
        r = rep[prec]
        assert all(v > 0 for v in r["t1"][:4] + r["t2"][:4] + r["elimination"][:3])
        assert r["elimination"][3] == -1.0      # the direct form takes contiguous lines only
        assert r["t2"][4] == r["t2"][5] == r["t2"][6] == r["t2"][7] == -1.0   # no staging form for 96
        t1 = [v if v > 0 else np.inf for v in r["t1"]]
        assert tuned_variant(0, 128, 1, fp64) == int(np.argmin(t1))
        assert tuned_variant(0, 96, 0, fp64) == int(np.argmin(r["t2"][:4]))
        elim = [v if v > 0 else np.inf for v in r["elimination"]]
        assert tuned_variant(1, 192, 0, fp64) == int(np.argmin(elim))
    got, _ = gpu_solve(prob)
    assert rel_l2(got, oracle_solve(prob)) <= TOL64
    probs = inputs.batch(7, count=4)
    plans = [Plan.from_problem(p) for p in probs]
    fields = [to_dev(p.rhs) for p in probs]
    b = Batch(plans)
    b.bind(fields)
    b.launch(graph=True)
    got = [to_host(f) for f in fields]
    _synchronous_variants()
    for p, g in zip(probs, got):
        single, _ = gpu_solve(p)
        assert np.array_equal(g, single)
    b.close()
    for pl in plans:
        pl.close()
    plan.close()


def test_refined_batch_equals_single_refined_solves(default_variants):
    """A batch of FP32 + refinement plans (uneven sizes, random boundary
    pairs, stretched and uniform z): each FP32 solve of the refinement is one
    batched launch per stage, the FP64 refinement kernels run per instance in
    between.  Bitwise equal to refined single solves with the same kernel
    variants, with the same refinement status; within 1e-10 of the oracle;
    also as graph replays with new fields bound between them; a plan with a
    lower iteration limit stops there (not converged) while the others go on."""
    import torch
    from paper_1802_10323_amd import FP32_REFINED, Batch, Plan
    probs = inputs.batch(13, count=5, sizes=(64, 96, 128))
    plans = [Plan.from_problem(p) for p in probs]
    for k, pl in enumerate(plans):
        if k == 2:
            pl.set_precision(FP32_REFINED, 1e-30, 2)    # stops after 2 FP32 solves
        else:
            pl.set_precision(FP32_REFINED, 1e-10, 6)
    _synchronous_variants()
    singles, stats = [], []
    for p, pl in zip(probs, plans):
        f = to_dev(p.rhs)
        pl.solve(f)
        torch.cuda.synchronize()
        singles.append(to_host(f))
        stats.append(pl.status())
    say("refined singles", [(p.shape, p.bcs, s) for p, s in zip(probs, stats)])
    assert stats[2][0] == 2 and not stats[2][2]
    b = Batch(plans)
    src = [to_dev(p.rhs) for p in probs]
    fields = [s.clone() for s in src]
    b.bind(fields)
    for graph in (False, True, True, True):   # eager, capture, two replays
        for f, s in zip(fields, src):
            f.copy_(s)
        torch.cuda.synchronize()
        b.launch(graph=graph)
        torch.cuda.synchronize()
        for k, (p, pl, f) in enumerate(zip(probs, plans, fields)):
            got = to_host(f)
            assert np.array_equal(got, singles[k]), (graph, k, p.shape, p.bcs)
            assert pl.status() == stats[k], (graph, k)
            if k != 2 and p.points <= 300_000:
                assert rel_l2(got, oracle_solve(p)) <= 1e-10, (k, p.shape)
    b.close()
    for pl in plans:
        pl.close()


def test_batch_rejects_mixed_precision_and_repeated_refined_plans():
    from paper_1802_10323_amd import FP32_REFINED, Batch, Plan, PoissonError
    probs = inputs.batch(14, count=2, sizes=(64,))
    a, c = Plan.from_problem(probs[0]), Plan.from_problem(probs[1])
    c.set_precision(FP32_REFINED, 1e-10, 4)
    with pytest.raises(PoissonError):
        Batch([a, c])
    with pytest.raises(PoissonError):
        Batch([c, c])
    a.close()
    c.close()


def test_batch_autotune_whole_batch():
    """batch_autotune times each step with the per-length choices and with
    every synchronous variant for all jobs, and keeps the fastest; a graph
    captured before tuning is captured again where the tuning changed its
    launches, and the tuned batch still matches the oracle and the single
    solves (to rounding: its steps may mix variants a single solve cannot)."""
    from paper_1802_10323_amd import Batch, Plan
    probs = inputs.batch(11, count=6)
    plans = [Plan.from_problem(p) for p in probs]
    fields = [to_dev(p.rhs) for p in probs]
    b = Batch(plans)
    b.bind(fields)
    b.launch(graph=True)                # captured with the default choices
    rep = b.autotune(reps=2)
    say("batch autotune", rep)
    for step, r in rep.items():
        count = 3 if step == "tridiag" else 5
        assert all(v > 0 for v in r[:count]), (step, r)
        assert all(v == -1.0 for v in r[count:]), (step, r)
    for _ in range(2):                  # replays of the (re)captured graph
        fresh = [to_dev(p.rhs) for p in probs]
        b.bind(fresh)
        b.launch(graph=True)
        for p, f in zip(probs, fresh):
            got = to_host(f)
            single, _ = gpu_solve(p)
            assert rel_l2(got, single) <= 1e-14, p.shape
            if p.points <= 300_000:
                assert rel_l2(got, oracle_solve(p)) <= TOL64, p.shape
    b.close()
    for pl in plans:
        pl.close()
