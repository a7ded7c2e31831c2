"""Multi-tile parity of the size-specialised kernels, above all the staging
forms (the next tile is read into LDS by DMA while the current one is
transformed or eliminated, and the previous tile's stores stay in flight).

Every kernel here is persistent: a block loops over tiles.  A block that
owns a single tile never runs the prefetch of a next tile, so every case
below makes each block loop over many tiles:

* with the persistent grid capped (POISSON_GRID_CAP) to a few blocks per
  XCD, on fields of about a million points, with ragged last tiles (line
  counts and x extents that are not multiples of the tile);
* at the real grid, on fields with more tiles than resident blocks (and the
  512^3 cube in test_gpu_fullsize.py).

Capped and uncapped launches must give the same bits: a tile's arithmetic
does not depend on which block runs it.

Transforms are compared with the oracle's Table 2 sums (FP64 stage,
<= 1e-13 relative L2, and the round trip); eliminations with the oracle's
Gauss elimination (backward error <= 1e-14 and the conditioned forward
bound); FP32 kernels through the refined solve (<= 1e-10 against the
oracle solve, Sec. 2.1 Eq. (poi))."""
import numpy as np
import pytest

from gpu_util import AXIS, check_elimination, oracle_solve, rel_l2, to_dev, to_host
from paper_1802_10323_amd import inputs

pytestmark = pytest.mark.gpu

KINDS = ("P", "NN", "DD", "ND", "DN")
CAP = 16            # blocks per launch: two per XCD


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_10323_amd import lib
    lib()


def say(*a):
    print(*a, flush=True)


def transform_case(axis, kind, n):
    """(nx, ny, nz), boundary pairs and transform role putting a length-n
    transform of type `kind` on `axis`; ragged tiles on every layout."""
    if axis == "x":     # contiguous: 60 * 33 = 1980 lines, no multiple of 8, 16 or 32
        return (n, 60, 33), (kind, "NN", "DD"), 0
    if axis == "y":     # strided: x extent 40 (ragged for 16- and 32-wide tiles)
        return (40, n, 53), ("NN", kind, "DD"), 1
    assert kind == "P"  # z is transformed only when periodic and uniform
    return (40, 48, n), ("DD", "NN", "P"), 1


TRANSFORM_CASES = ([("x", k, n) for k in KINDS for n in (256, 512)]
                   + [("y", k, n) for k in KINDS for n in (256, 512)]
                   + [("z", "P", n) for n in (256, 512)])


def _stage(shape, bcs, role, f, inverse, cap, monkeypatch):
    from paper_1802_10323_amd import Plan
    if cap:
        monkeypatch.setenv("POISSON_GRID_CAP", str(cap))
    else:
        monkeypatch.delenv("POISSON_GRID_CAP", raising=False)
    plan = Plan(shape[0], shape[1], shape[2], 1.0 / shape[0], 1.0 / shape[1],
                np.full(shape[2], 1.0 / shape[2]), bcs)
    d = to_dev(f)
    plan.transform_stage(role, inverse, d)
    out = to_host(d)
    plan.close()
    return out


@pytest.mark.parametrize("axis,kind,n", TRANSFORM_CASES)
def test_transform_multitile(axis, kind, n, monkeypatch, default_variants):
    """FP64 transform stage, default variant and each staging tile shape
    (variant 6 has no FP64 form and falls back to variant 0; variant 7, the
    register-staged 32-line form, runs on strided axes of length 512 with
    at least 32 x positions), grid capped and uncapped, against the Table 2
    sums; backward stage returns f."""
    from oracle import transforms as tr
    from paper_1802_10323_amd import set_tuned_variant, tuned_variant
    shape, bcs, role = transform_case(axis, kind, n)
    rng = np.random.default_rng(n + 7 * KINDS.index(kind))
    f = rng.uniform(-1.0, 1.0, (shape[2], shape[1], shape[0]))
    ref = tr.forward(f, AXIS[axis], kind)
    layout = 1 if axis == "x" else 0
    for V in (None, 4, 5, 6, 7):
        if V is not None:
            set_tuned_variant(0, n, layout, V)
        say("transform", axis, kind, n, "variant", tuned_variant(0, n, layout))
        capped = _stage(shape, bcs, role, f, False, CAP, monkeypatch)
        err = rel_l2(capped, ref)
        assert err <= 1e-13, (axis, kind, n, V, err)
        full = _stage(shape, bcs, role, f, False, 0, monkeypatch)
        assert np.array_equal(capped, full), (axis, kind, n, V)
        back = _stage(shape, bcs, role, capped, True, CAP, monkeypatch)
        assert rel_l2(back, f) <= 1e-13, (axis, kind, n, V)


def test_transform_more_tiles_than_blocks(monkeypatch):
    """Uncapped grid on fields with several times more tiles than resident
    blocks (at most 512 per launch; 1024 tiles of 16 lines here): the
    strided length-512 DFT along z, the strided length-512 DCT-IV along y
    and the contiguous length-512 DST-II along x."""
    from oracle import transforms as tr
    monkeypatch.delenv("POISSON_GRID_CAP", raising=False)
    rng = np.random.default_rng(11)
    for axis, shape, bcs, role, kind in (
            ("z", (64, 256, 512), ("DD", "NN", "P"), 1, "P"),
            ("y", (64, 512, 256), ("NN", "ND", "DD"), 1, "ND"),
            ("x", (512, 128, 128), ("DD", "NN", "NN"), 0, "DD")):
        f = rng.uniform(-1.0, 1.0, (shape[2], shape[1], shape[0]))
        got = _stage(shape, bcs, role, f, False, 0, monkeypatch)
        err = rel_l2(got, tr.forward(f, AXIS[axis], kind))
        say("uncapped", axis, shape, kind, err)
        assert err <= 1e-13, (axis, shape, err)
        back = _stage(shape, bcs, role, got, True, 0, monkeypatch)
        assert rel_l2(back, f) <= 1e-13


ELIM_CASES = [(n, k) for n in (64, 128, 192, 256, 384, 512) for k in ("NN", "DD", "ND", "DN")]


@pytest.mark.parametrize("V", [0, 1, 2, 3])
@pytest.mark.parametrize("n,kind", ELIM_CASES)
def test_elimination_multitile(n, kind, V, monkeypatch, default_variants):
    """FP64 elimination, every variant (two chunkings, the staging form and
    the direct form of contiguous lines),
    grid capped, contiguous (s = x; 1080 lines, ragged) and strided (s = z;
    x extent 40, ragged), regular, singular and stretched."""
    from paper_1802_10323_amd import set_tuned_variant
    monkeypatch.setenv("POISSON_GRID_CAP", str(CAP))
    for layout in (0, 1):
        set_tuned_variant(1, n, layout, V)
    cases = [((n, 30, 36), (kind, "P", "P"), "x"), ((n, 30, 36), (kind, "NN", "P"), "x"),
             ((40, 30, n), ("P", "P", kind), "z"), ((40, 30, n), ("P", "DD", kind), "z")]
    check_elimination(n, kind, cases)


def _refined(prob, cap, monkeypatch, tol=1e-10, max_iters=6):
    from paper_1802_10323_amd import FP32_REFINED, Plan
    if cap:
        monkeypatch.setenv("POISSON_GRID_CAP", str(cap))
    else:
        monkeypatch.delenv("POISSON_GRID_CAP", raising=False)
    plan = Plan.from_problem(prob)
    plan.set_precision(FP32_REFINED, tol, max_iters)
    d = to_dev(prob.rhs)
    plan.solve(d)
    got = to_host(d)
    status = plan.status()
    plan.close()
    return got, status


@pytest.mark.parametrize("axis,kind,n", TRANSFORM_CASES)
def test_fp32_transform_multitile_refined(axis, kind, n, monkeypatch, default_variants):
    """FP32 transforms of length n on `axis` inside the refined solve, the
    default variant and every staging tile shape (6: the 32-line FP32
    shape), grid capped: converges to the oracle solve within 1e-10; the
    uncapped default run gives the same bits."""
    from paper_1802_10323_amd import set_tuned_variant
    shape, bcs, _ = transform_case(axis, kind, n)
    prob = inputs.make_uniform(*shape, bcs, seed=3 + n)
    ref = oracle_solve(prob)
    layout = 1 if axis == "x" else 0
    for V in (None, 4, 5, 6):
        if V is not None:
            set_tuned_variant(0, n, layout, V, fp64=False)
        got, (iters, rel, conv) = _refined(prob, CAP, monkeypatch)
        err = rel_l2(got, ref)
        say("fp32 transform", axis, kind, n, V, "iters", iters, "rel-L2", err)
        assert conv and iters <= 4, (axis, kind, n, V, iters, rel)
        assert err <= 1e-10, (axis, kind, n, V, err)
        if V is None:
            full, _ = _refined(prob, 0, monkeypatch)
            assert np.array_equal(full, got), (axis, kind, n)


@pytest.mark.parametrize("V", [0, 1, 2, 3])
@pytest.mark.parametrize("n", [256, 384, 512])
@pytest.mark.parametrize("layout", ["x", "z"])
def test_fp32_elimination_multitile_refined(layout, n, V, monkeypatch, default_variants):
    """FP32 elimination (its recurrences run in FP64 on FP32 data) in every
    variant, contiguous (s = x) and strided (s = z), inside the refined
    solve with the grid capped: within 1e-10 of the oracle solve."""
    from paper_1802_10323_amd import set_tuned_variant
    for lay in (0, 1):
        set_tuned_variant(1, n, lay, V, fp64=False)
    if layout == "x":
        prob = inputs.make_uniform(n, 30, 36, ("DD", "P", "P"), seed=n + V)
    else:
        prob = inputs.make_uniform(40, 30, n, ("P", "DD", "ND"), seed=n + V, stretch_z=1.8)
    ref = oracle_solve(prob)
    got, (iters, rel, conv) = _refined(prob, CAP, monkeypatch)
    err = rel_l2(got, ref)
    say("fp32 elimination", layout, n, V, "iters", iters, "rel-L2", err)
    assert conv and iters <= 4, (layout, n, V, iters, rel)
    assert err <= 1e-10, (layout, n, V, err)


def test_fp32_contiguous_elimination_default(monkeypatch, default_variants):
    """The default FP32 elimination of contiguous lines of 512 points is the
    direct form (the 512^3 cube's refined solve runs it): uncapped, on a
    field with more line groups than resident waves ((512, 128, 64): 8192
    lines), within 1e-10 of the oracle solve."""
    from paper_1802_10323_amd import tuned_variant
    assert tuned_variant(1, 512, 1, fp64=False) == 3
    prob = inputs.make_uniform(512, 128, 64, ("DD", "ND", "P"), seed=21)
    ref = oracle_solve(prob)
    got, (iters, rel, conv) = _refined(prob, 0, monkeypatch)
    err = rel_l2(got, ref)
    say("fp32 direct elimination (512, 128, 64)", iters, err)
    assert conv and iters <= 4
    assert err <= 1e-10
