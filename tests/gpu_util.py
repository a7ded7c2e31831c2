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
    return oracle.solve(prob.rhs, prob.hx, prob.hy, prob.hz, *prob.bcs, roles=roles,
                        shift=getattr(prob, "shift", 0.0))


UNIT = 2.0 ** -53


def _line_systems(x, f, a, b, c, periodic, shift):
    """Largest normwise backward error over the lines (columns) of
    (b + shift) x + a x_{k-1} + c x_{k+1} = f."""
    ax = (b[:, None] + shift[None, :]) * x
    ax[1:] += a[1:, None] * x[:-1]
    ax[:-1] += c[:-1, None] * x[1:]
    if periodic:
        ax[0] += a[0] * x[-1]
        ax[-1] += c[-1] * x[0]
    norm_a = (np.abs(a)[:, None] + np.abs(b[:, None] + shift[None, :]) + np.abs(c)[:, None]).max(axis=0)
    scale = norm_a * np.linalg.norm(x, axis=0) + np.linalg.norm(f, axis=0)
    return float((np.linalg.norm(ax - f, axis=0) / scale).max())


def check_elimination(n, kind, cases=None):
    """The elimination stage alone for lengths that have size-specialised
    kernels (and the size-generic kernel on the same input), on the strided
    (s = z) and contiguous (s = x) layouts, singular and regular, uniform and
    stretched, with ragged last tiles (`cases`: other (shape, bcs, expected
    elimination axis) triples).

    Checks: (1) every regular line's normwise backward error is at rounding
    level (<= 1e-14, condition-independent); (2) the result matches the
    oracle within max(1e-12, kappa u), kappa the 2-norm condition number of
    the zero-shift (or, when singular, pinned) line operator, which bounds
    the forward error of any backward-stable solver of the worst line."""
    from oracle import transforms as tr
    from oracle import tridiagonal as td
    from oracle.poisson import tridiagonal_stage
    from paper_1802_10323_amd import Plan, inputs
    import oracle
    if cases is None and kind == "P":
        # a periodic elimination axis: all axes periodic; contiguous (s = x
        # when y and z take the DFT) and strided (a stretched z is always s)
        cases = [((n, 10, 6), ("P", "P", "P"), "x"), ((20, 10, n), ("P", "P", "P"), "z", (True,))]
    elif cases is None:
        cases = [((20, 10, n), ("P", "P", kind), "z"), ((20, 10, n), ("P", "DD", kind), "z"),
                 ((n, 10, 6), (kind, "P", "P"), "x"), ((n, 10, 6), (kind, "DD", "P"), "x")]
    for case in cases:
        shape, bcs, s_expect = case[:3]
        stretch_options = case[3] if len(case) > 3 else (
            (False, True) if bcs[2] != "P" else (False,))
        for stretched in stretch_options:
            prob = inputs.make_uniform(*shape, bcs, seed=n + len(kind),
                                       stretch_z=1.8 if stretched else None)
            plan = Plan.from_problem(prob)
            t1, t2, s = plan.roles
            assert s == s_expect
            h = {"x": prob.hx, "y": prob.hy, "z": prob.hz}
            bc = dict(zip("xyz", bcs))
            dims = dict(zip("xyz", shape))
            singular = oracle.is_singular(*bcs)
            # lines along s as columns: (n_s, n_t1 * n_t2)
            order = (AXIS[s], AXIS[t1], AXIS[t2])
            fin = np.transpose(prob.rhs, order).copy()
            if singular:   # the zero-wavenumber line of a transformed compatible field
                w = h[s]
                fin[:, 0, 0] -= (w * fin[:, 0, 0]).sum() / w.sum()
            f = np.ascontiguousarray(np.transpose(fin, np.argsort(order)))
            lam1 = tr.eigenvalues(bc[t1], dims[t1]) / h[t1][0] ** 2
            lam2 = tr.eigenvalues(bc[t2], dims[t2]) / h[t2][0] ** 2
            ref = tridiagonal_stage(f, s, h[s], bc[s], lam1, lam2, t1, t2, singular)
            d = to_dev(f)
            plan.tridiag_stage(d)
            got = to_host(d)
            plan.close()
            a, b, c, periodic = td.coefficients(h[s], bc[s])
            shift = (lam1[:, None] + lam2[None, :]).reshape(-1)
            xg = np.transpose(got, order).reshape(dims[s], -1)
            fl = fin.reshape(dims[s], -1)
            first = 1 if singular else 0
            back = _line_systems(xg[:, first:], fl[:, first:], a, b, c, periodic, shift[first:])
            assert back <= 1e-14, (shape, bcs, stretched, "backward error", back)
            ops = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
            kappa = np.linalg.cond(ops[:-1, :-1] if singular else ops)
            err = rel_l2(got, ref)
            assert err <= max(1e-12, kappa * UNIT), (shape, bcs, stretched, err, kappa)
