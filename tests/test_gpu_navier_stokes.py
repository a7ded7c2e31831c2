"""GPU parity of the Navier-Stokes time step (Sec. 2: Eq. (up), the
pressure correction of every substep; the tri-periodic Taylor-Green case of
Sec. 4.1) against the oracle (oracle/navier_stokes.py), through the C ABI.

Tolerance.  The prediction is one FP64 stencil per face (a few tens of
operations: relative error a few units of 2^-53 on |u| + dt |AD|); the
right-hand side divides the divergence of u* by gamma_k dt, so the two
sides' rounding differences of order 1e-16 |u| / dx grow to
1e-16 |u| / (dx gamma_k dt) there, against a right-hand side of order
|AD| / dx.  For the grids below that is below 1e-12 relative, the bound the
solve itself meets; the velocity, the pressure, Phi and AD are held to 1e-12
relative L2 per array (AD and the velocity in practice near 1e-15).  At
512^3 the Taylor-Green Phi is four orders below p and its conditioning
with respect to the rounding of u* (measured in the test) sets its bound.

Shapes: several blocks per plane with ragged rows, three different spacings,
a grid larger than one pass of the grid-stride launch, and the 512^3
Taylor-Green vortex, the workload the benchmark times, in the same launch
configuration: its first substep against the oracle's, the whole step (each
projection applied by the next prediction) by divergence and the energy
budget.  Rejections of plans the step does not
support come last."""
import math

import numpy as np
import pytest

from gpu_util import rel_l2, to_dev, to_host
from paper_1802_10323_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_10323_amd import lib
    lib()


def periodic_plan(nx, ny, nz, lengths):
    from paper_1802_10323_amd import Plan
    d = (lengths[0] / nx, lengths[1] / ny, lengths[2] / nz)
    return Plan(nx, ny, nz, d[0], d[1], inputs.uniform_widths(nz, lengths[2]), ("P", "P", "P")), d


def random_state(seed, shape):
    rng = np.random.default_rng(seed)
    vel = [rng.uniform(-1, 1, shape) for _ in range(3)]
    ad = [rng.uniform(-1, 1, shape) for _ in range(3)]
    p = rng.uniform(-1, 1, shape)
    return vel, ad, p


def device_state(vel, ad, p):
    """Device buffers; ad fills both AD buffers (substep 2 reads the first,
    substep 3 the second)."""
    import torch
    n = p.size
    dvel = to_dev(np.concatenate([a.reshape(-1) for a in vel]))
    dad = to_dev(np.concatenate([a.reshape(-1) for a in ad] * 2))
    work = torch.empty(3 * n, dtype=torch.float64, device="cuda")
    phi = torch.empty(n, dtype=torch.float64, device="cuda")
    return dvel, work, dad, to_dev(p), phi


def scratch_for(shape):
    import torch
    return torch.empty(2 * int(np.prod(shape)), dtype=torch.float64, device="cuda")


def split(t, shape):
    a = to_host(t)
    n = int(np.prod(shape))
    return [a[c * n:(c + 1) * n].reshape(shape) for c in range(len(a) // n)]


SUBSTEP_CASES = [
    # nx, ny, nz, lengths, dt, nu
    (32, 24, 20, (1.0, 0.8, 1.3), 0.003, 0.01),       # x narrower than a tile
    (200, 12, 150, (1.0, 0.3, 0.9), 0.001, 0.005),    # ragged x tiles, several z ranges
    (90, 30, 9, (2.0, 1.0, 0.5), 0.001, 0.002),      # ragged rows, odd short z
    (160, 128, 130, (1.0, 1.0, 1.0), 0.0005, 0.001),  # more cells than one grid-stride pass
    (128, 16, 192, (1.0, 0.6, 1.4), 0.001, 0.004),    # whole tiles, three z ranges: the branch-free loop
]


@pytest.mark.parametrize("kernel", ["fused", "tiled", "simple"])
@pytest.mark.parametrize("case", SUBSTEP_CASES, ids=lambda c: "x".join(map(str, c[:3])))
@pytest.mark.parametrize("k", [1, 2, 3])
def test_substep_vs_oracle(case, k, kernel, monkeypatch):
    """Every prediction kernel: the z-marching LDS tile kernel with the
    right-hand side fused (default), the same without it (the right-hand
    side in a sweep of its own; POISSON_RK3_KERNEL=tiled) and one cell per
    thread (POISSON_RK3_KERNEL=simple)."""
    from oracle import navier_stokes as ns
    if kernel != "fused":
        monkeypatch.setenv("POISSON_RK3_KERNEL", kernel)
    nx, ny, nz, lengths, dt, nu = case
    shape = (nz, ny, nx)
    say("rk3 substep", k, case, kernel)
    plan, (dx, dy, dz) = periodic_plan(nx, ny, nz, lengths)
    vel, ad_prev, p = random_state(100 * k + nx, shape)
    dvel, work, dad, dp, phi = device_state(vel, ad_prev, p)
    plan.rk3_substep(k, dt, nu, dvel, work, dad, dp, phi)
    ref = ns.rk3_substep(k, *vel, p, ad_prev, dt, nu, dx, dy, dz)
    got_vel = split(dvel, shape)
    got_ad = split(dad, shape)
    errs = {}
    for c, name in enumerate("uvw"):
        errs[name] = rel_l2(got_vel[c], ref[c])
    errs["p"] = rel_l2(to_host(dp).reshape(shape), ref[3])
    errs["phi"] = rel_l2(to_host(phi).reshape(shape), ref[5])
    for c, name in enumerate(("adu", "adv", "adw")):
        # substep 1 writes its AD into the first buffer, substep 2 into the
        # second; the other buffer (and both after substep 3) keep AD_prev
        first = ref[4][c] if k == 1 else ad_prev[c]
        second = ref[4][c] if k == 2 else ad_prev[c]
        errs[name] = max(rel_l2(got_ad[c], first), rel_l2(got_ad[3 + c], second))
    say("  rel-L2", {a: f"{b:.2e}" for a, b in errs.items()})
    assert max(errs.values()) <= TOL, errs
    plan.close()


@pytest.mark.parametrize("shape", [(128, 16, 192), (64, 8, 128)], ids=lambda s: "x".join(map(str, s)))
def test_whole_tile_loop_equals_general_loop(shape, monkeypatch):
    """On whole tiles (nx, ny, nz multiples of 64, 4, 64) the fused
    prediction runs its branch-free z loop; POISSON_RK3_GENERAL=1 forces
    the general loop.  Both run the same cell arithmetic in the same order:
    a whole step (three predictions, the correcting ones included) is
    equal bit for bit."""
    import torch
    nx, ny, nz = shape
    vel, _, p = random_state(11 + nx, (nz, ny, nx))
    out = {}
    for general in (False, True):
        if general:
            monkeypatch.setenv("POISSON_RK3_GENERAL", "1")
        else:
            monkeypatch.delenv("POISSON_RK3_GENERAL", raising=False)
        plan, _ = periodic_plan(nx, ny, nz, (1.0, 0.7, 1.2))
        dvel, work, dad, dp, phi = device_state(vel, np.zeros_like(vel), p)
        plan.rk3_step(0.001, 0.003, dvel, work, dad, dp, phi, scratch_for((nz, ny, nx)))
        torch.cuda.synchronize()
        out[general] = (dvel.clone(), dp.clone())
        plan.close()
    say("whole-tile loop", shape)
    assert torch.equal(out[False][0], out[True][0]) and torch.equal(out[False][1], out[True][1])


@pytest.mark.parametrize("case", SUBSTEP_CASES, ids=lambda c: "x".join(map(str, c[:3])))
@pytest.mark.parametrize("k", [1, 2, 3])
def test_fused_right_hand_side(case, k, monkeypatch):
    """rk3_predict: the fused kernel's u* and AD agree with the tiled
    kernel's to rounding (one cell function, compiled in two kernels that
    may contract differently), and its right-hand side with the separate
    divergence sweep over the tiled u*, on the scale of the divergence's
    terms, |u*| / (dx gamma dt); both against the oracle's prediction and
    right-hand side."""
    import torch
    from oracle import navier_stokes as ns
    from oracle import projection as pj
    nx, ny, nz, lengths, dt, nu = case
    shape = (nz, ny, nx)
    vel, ad_prev, p = random_state(7 * k + nx, shape)
    out = {}
    for kernel in ("fused", "tiled"):
        if kernel == "tiled":
            monkeypatch.setenv("POISSON_RK3_KERNEL", "tiled")
        plan, (dx, dy, dz) = periodic_plan(nx, ny, nz, lengths)
        dvel, work, dad, dp, rhs = device_state(vel, ad_prev, p)
        plan.rk3_predict(k, dt, nu, dvel, work, dad, dp, rhs)
        torch.cuda.synchronize()
        out[kernel] = (work.clone(), dad.clone(), rhs.clone())
        plan.close()
    star, ad = ns.prediction(k, *vel, p, ad_prev, dt, nu, dx, dy, dz)
    scale = max(np.abs(a).max() for a in star) / (min(dx, dy, dz) * ns.GAMMA[k - 1] * dt)
    for a, b, name, sc in zip(out["fused"], out["tiled"], ("u*", "AD", "rhs"),
                              (float(torch.abs(out["tiled"][0]).max()),
                               float(torch.abs(out["tiled"][1]).max()), scale)):
        d = float(torch.abs(a - b).max()) / sc
        say("  fused vs tiled", name, d)
        assert d <= 4 * 2.0 ** -52, name
    h = [ns.widths(n, d) for n, d in zip((nx, ny, nz), (dx, dy, dz))]
    rhs_ref = pj.projection_rhs(*star, ns.GAMMA[k - 1] * dt, *h, ("P", "P", "P"))
    got_star = split(out["fused"][0], shape)
    assert max(rel_l2(g, r) for g, r in zip(got_star, star)) <= TOL
    # the right-hand side is the small divergence of a nearly cancelling sum:
    # bound it on the scale of its terms
    err = np.abs(to_host(out["fused"][2]).reshape(shape) - rhs_ref).max() / scale
    say("rk3_predict", case, k, "rhs max error / (|u*| / (dx gamma dt))", err)
    assert err <= 1e-14


STEP_CASES = [(64, None, 0.0, 0.0)] + [((nx, ny, nz), L, dt, nu) for nx, ny, nz, L, dt, nu in SUBSTEP_CASES]


@pytest.mark.parametrize("kernel", ["fused", "tiled"])
@pytest.mark.parametrize("case", STEP_CASES, ids=lambda c: "tg64" if c[1] is None else "x".join(map(str, c[0])))
def test_step_vs_oracle(case, kernel, monkeypatch):
    """One whole step: the Taylor-Green start at 64^3 (2 pi box, Re 1600) and
    random fields on the substep shapes (ragged tiles, several z ranges).
    Default: each substep's projection applied by the next prediction;
    tiled: substep by substep."""
    from oracle import navier_stokes as ns
    if kernel != "fused":
        monkeypatch.setenv("POISSON_RK3_KERNEL", kernel)
    n, lengths, dt, nu = case
    if lengths is None:
        u, v, w, p, d = inputs.taylor_green(n)
        vel = [u, v, w]
        shape = u.shape
        plan, (dx, dy, dz) = periodic_plan(n, n, n, (2 * math.pi,) * 3)
        nu = 1.0 / 1600
        dt = 0.9 * ns.stable_dt(u, v, w, dx, dy, dz, nu)
    else:
        nx, ny, nz = n
        shape = (nz, ny, nx)
        vel, _, p = random_state(7, shape)
        plan, (dx, dy, dz) = periodic_plan(nx, ny, nz, lengths)
        dt = 0.5 * ns.stable_dt(*vel, dx, dy, dz, nu)
    say("rk3 step", shape, kernel, "dt", dt)
    zeros = [np.zeros(shape)] * 3
    dvel, work, dad, dp, phi = device_state(vel, zeros, p)
    plan.rk3_step(dt, nu, dvel, work, dad, dp, phi, scratch_for(shape))
    ref = ns.rk3_step(*vel, p, dt, nu, dx, dy, dz)
    got = split(dvel, shape) + [to_host(dp).reshape(shape)]
    errs = [rel_l2(g, r) for g, r in zip(got, ref) if np.linalg.norm(r) > 0]
    say("  rel-L2 u, v, (w), p", ["%.2e" % e for e in errs])
    assert max(errs) <= TOL
    plan.close()


def test_step_with_a_refined_plan():
    """The step's solves run in the plan's precision mode: on an FP32 +
    FP64-refinement plan (tolerance 1e-10 on Phi) one Taylor-Green step at
    48^3 stays within 1e-10 of the oracle's step (Phi enters u through
    gamma dt grad Phi, a small correction of u)."""
    from oracle import navier_stokes as ns
    from paper_1802_10323_amd import FP32_REFINED
    n = 48
    u, v, w, p, d = inputs.taylor_green(n)
    nu = 1.0 / 1600
    dt = 0.9 * ns.stable_dt(u, v, w, d, d, d, nu)
    plan, _ = periodic_plan(n, n, n, (2 * math.pi,) * 3)
    plan.set_precision(FP32_REFINED, 1e-10, 4)
    shape = u.shape
    dvel, work, dad, dp, phi = device_state([u, v, w], [np.zeros(shape)] * 3, p)
    plan.rk3_step(dt, nu, dvel, work, dad, dp, phi, scratch_for(shape))
    ref = ns.rk3_step(u, v, w, p, dt, nu, d, d, d)
    got = split(dvel, shape) + [to_host(dp).reshape(shape)]
    errs = [rel_l2(g, r) for g, r in zip(got, ref)]
    say("refined plan step: rel-L2 u, v, w, p", ["%.2e" % x for x in errs])
    assert max(errs) <= 1e-10
    plan.close()


def test_ten_steps_vs_oracle():
    """Ten steps of the 48^3 Taylor-Green vortex (Re 1600, dt at 0.9 of the
    stability bound) on the same buffers, against ten oracle steps: the
    velocity and the pressure within 1e-12 after each, and the kinetic
    energy decreasing every step."""
    import torch
    from oracle import navier_stokes as ns
    n = 48
    u, v, w, p, d = inputs.taylor_green(n)
    nu = 1.0 / 1600
    dt = 0.9 * ns.stable_dt(u, v, w, d, d, d, nu)
    plan, _ = periodic_plan(n, n, n, (2 * math.pi,) * 3)
    shape = u.shape
    dvel, work, dad, dp, phi = device_state([u, v, w], [np.zeros(shape)] * 3, p)
    scratch = scratch_for(shape)
    ref = (u, v, w, p)
    energy = 0.5 * sum(float(np.sum(a * a)) for a in (u, v, w))
    for step in range(10):
        plan.rk3_step(dt, nu, dvel, work, dad, dp, phi, scratch)
        ref = ns.rk3_step(*ref, dt, nu, d, d, d)
        got = split(dvel, shape) + [to_host(dp).reshape(shape)]
        errs = [rel_l2(g, r) for g, r in zip(got, ref)]
        e = 0.5 * sum(float(np.sum(a * a)) for a in got[:3])
        assert max(errs) <= TOL, (step, errs)
        assert e < energy, (step, e, energy)
        energy = e
    say("ten steps: rel-L2 u, v, w, p", ["%.2e" % x for x in errs])
    plan.close()


@pytest.mark.parametrize("kernel", ["fused", "tiled"])
def test_substeps_compose_to_the_step(kernel, monkeypatch):
    """rk3_step against substeps 1, 2, 3 on the same inputs: bitwise when the
    step runs substep by substep (tiled), to rounding when it applies each
    projection inside the next prediction (the same arithmetic compiled in
    another kernel: each value within 4 ulp of the field's largest)."""
    import torch
    if kernel != "fused":
        monkeypatch.setenv("POISSON_RK3_KERNEL", kernel)
    nx, ny, nz = 40, 36, 20
    shape = (nz, ny, nx)
    plan, _ = periodic_plan(nx, ny, nz, (1.0, 1.0, 1.0))
    vel, ad, p = random_state(3, shape)
    a = device_state(vel, ad, p)
    b = device_state(vel, ad, p)
    plan.rk3_step(0.002, 0.01, *a, scratch_for(shape))
    for k in (1, 2, 3):
        plan.rk3_substep(k, 0.002, 0.01, *b)
    torch.cuda.synchronize()
    for x, y, name in zip(a, b, ("vel", "work", "ad", "p", "phi")):
        if name in ("work", "ad"):
            continue                                    # scratch, and AD of the last substeps
        if kernel == "fused":
            d = float(torch.abs(x - y).max()) / float(torch.abs(y).max())
            say("  fused step vs substeps", name, d)
            assert d <= 4 * 2.0 ** -52, name
        else:
            assert torch.equal(x, y), name
    plan.close()


@pytest.mark.timeout(900)
def test_taylor_green_512_vs_oracle():
    """The benchmark's workload, the 512^3 Taylor-Green vortex (Re 1600, dt
    at 0.9 of the stability bound), in the launch configuration it times.
    The first substep against the oracle's (about a minute and 40 GiB of
    host memory); the whole step by properties that hold at any size: zero
    divergence, and the kinetic energy budget of the start, where advection
    exchanges no energy and diffusion removes it at the rate 6 nu E (the
    field is an eigenfunction of the Laplacian with eigenvalue -3, the
    discrete one within 2e-5 of it at this spacing)."""
    import torch
    import oracle
    from oracle import navier_stokes as ns
    from oracle import projection as pj
    n = 512
    u, v, w, p, d = inputs.taylor_green(n)
    shape = u.shape
    nu = 1.0 / 1600
    dt = 0.9 * ns.stable_dt(u, v, w, d, d, d, nu)
    plan, _ = periodic_plan(n, n, n, (2 * math.pi,) * 3)
    dvel = to_dev(np.concatenate([u.reshape(-1), v.reshape(-1), w.reshape(-1)]))
    dad = torch.zeros(2 * dvel.numel(), dtype=torch.float64, device="cuda")
    work = torch.empty_like(dvel)
    dp = to_dev(p)
    phi = torch.empty_like(dp)
    say("rk3 substep 1 of the 512^3 Taylor-Green start on the GPU, dt", dt)
    plan.rk3_substep(1, dt, nu, dvel, work, dad, dp, phi)
    got = split(dvel, shape) + [to_host(dp).reshape(shape), to_host(phi).reshape(shape)]
    got_ad = split(dad, shape)[:3]
    say("oracle substep 1")
    ref = ns.rk3_substep(1, u, v, w, p, None, dt, nu, d, d, d)
    errs = {name: rel_l2(g, r) for name, g, r in zip(("u", "v", "w", "p", "phi"), got, ref[:4] + ref[5:])}
    errs.update({name: rel_l2(g, r) for name, g, r in zip(("adu", "adv", "adw"), got_ad, ref[4])})
    # Phi is a small increment of p (1e-4 of it here) made from the
    # divergence of a nearly divergence-free u*, so the rounding of u* alone
    # moves it far more than the solve's own error: its bound is that
    # sensitivity, measured on the oracle (Phi's relative change when u* is
    # perturbed by half an ulp with random signs), times 4.
    h = ns.widths(n, d)
    star, _ = ns.prediction(1, u, v, w, p, None, dt, nu, d, d, d)
    rng = np.random.default_rng(5)
    star = [a * (1.0 + 2.0 ** -53 * rng.choice([-1.0, 1.0], a.shape)) for a in star]
    rhs = pj.projection_rhs(*star, ns.GAMMA[0] * dt, h, h, h, ("P", "P", "P"))
    del star
    sens = rel_l2(oracle.solve(rhs, h, h, h, "P", "P", "P"), ref[5])
    del rhs
    phi_tol = max(TOL, 4.0 * sens)
    say("  rel-L2", {a: f"{b:.2e}" for a, b in errs.items()}, "Phi sensitivity", f"{sens:.2e}")
    assert errs.pop("phi") <= phi_tol, (errs, sens)
    assert max(errs.values()) <= TOL, errs
    del ref, got, got_ad
    # the whole step on the GPU from the start (each projection applied by
    # the next prediction), then the properties
    dvel.copy_(to_dev(np.concatenate([u.reshape(-1), v.reshape(-1), w.reshape(-1)])))
    dp.copy_(to_dev(p))
    scratch = scratch_for(shape)
    say("rk3 step 512^3")
    plan.rk3_step(dt, nu, dvel, work, dad, dp, phi, scratch)
    u1, v1, w1 = split(dvel, shape)
    del work, dad, phi, dvel, dp, scratch
    torch.cuda.empty_cache()
    div = pj.divergence(u1, v1, w1, h, h, h, ("P", "P", "P"))
    div_scale = np.abs(u1).max() / d
    e0 = 0.5 * sum(float(np.sum(a * a)) for a in (u, v, w))
    e1 = 0.5 * sum(float(np.sum(a * a)) for a in (u1, v1, w1))
    rate = (e1 - e0) / (dt * e0)
    say("  max |div u| / (max |u| / dx)", np.abs(div).max() / div_scale,
        "energy rate / (6 nu)", rate / (6 * nu), "max |w|", np.abs(w1).max())
    assert np.abs(div).max() <= 1e-13 * div_scale
    # the oracle's step gives 1.2e-2, 1.6e-3, 1.2e-4 off at 32^3, 64^3, 128^3
    assert abs(rate / (-6 * nu) - 1.0) <= 1e-3
    plan.close()


def test_unsupported_plans_are_refused():
    import torch
    from paper_1802_10323_amd import Plan, PoissonError
    h = inputs.uniform_widths(16)
    shape = (16, 16, 16)
    state = device_state(*random_state(1, shape))
    for bcs, hz in ((("P", "P", "NN"), h), (("P", "P", "P"), inputs.tanh_widths(16, 1.0, 1.5))):
        plan = Plan(16, 16, 16, h[0], h[0], hz, bcs)
        with pytest.raises(PoissonError):
            plan.rk3_step(0.01, 0.01, *state, scratch_for(shape))
        plan.close()
    plan = Plan(16, 16, 16, h[0], h[0], h, ("P", "P", "P"))
    for k, dt, nu in ((0, 0.01, 0.1), (4, 0.01, 0.1), (1, 0.0, 0.1), (1, 0.01, -1.0)):
        with pytest.raises(PoissonError):
            plan.rk3_substep(k, dt, nu, *state)
    with pytest.raises(ValueError):
        plan.rk3_step(0.01, 0.01, state[0][:10], *state[1:], scratch_for(shape))
    with pytest.raises(ValueError):
        plan.rk3_step(0.01, 0.01, *state, state[4])      # scratch too small
    torch.cuda.synchronize()
    plan.close()
