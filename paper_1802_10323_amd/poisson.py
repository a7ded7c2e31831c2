"""Thin ctypes binding of the C ABI in ``include/poisson.h``.

Argument marshalling only: every step of a solve runs in the HIP library
(``libpoisson_hip.so``).  PyTorch supplies device memory and streams.  If the
library is missing the binding raises; there is no other code path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# POISSON_HIP_LIB selects another build of the same library (A/B timing)
LIB_PATH = os.environ.get("POISSON_HIP_LIB") or os.path.join(HERE, "libpoisson_hip.so")

BC = {"P": 0, "NN": 1, "DD": 2, "ND": 3, "DN": 4, "DDn": 5, "NNn": 6}
AXES = "xyz"
FP64 = 0
FP32_REFINED = 1

OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP, ENOTCONVERGED = 0, -1, -2, -3, -4, -5

# exported symbol -> (restype, argtypes); mirrors include/poisson.h
_VP = ctypes.c_void_p
SIGNATURES = {
    "plan_create": (_VP, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                          ctypes.c_double, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                          ctypes.c_int, ctypes.c_int]),
    "plan_create_helmholtz": (_VP, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_double]),
    "solve": (ctypes.c_int, [_VP, _VP, _VP]),
    "plan_destroy": (None, [_VP]),
    "last_error": (ctypes.c_int, []),
    "last_error_message": (ctypes.c_char_p, []),
    "plan_set_precision": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_double, ctypes.c_int]),
    "plan_workspace_bytes": (ctypes.c_size_t, [_VP]),
    "solve_status": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_double)]),
    "batch_solve": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.c_int, _VP]),
    "plan_roles": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int)]),
    "transform_stage": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _VP, _VP]),
    "tridiag_stage": (ctypes.c_int, [_VP, _VP, _VP]),
    "batch_create": (_VP, [ctypes.POINTER(_VP), ctypes.c_int]),
    "batch_bind": (ctypes.c_int, [_VP, ctypes.POINTER(_VP)]),
    "batch_launch": (ctypes.c_int, [_VP, _VP, ctypes.c_int]),
    "batch_destroy": (None, [_VP]),
    "batch_autotune": (ctypes.c_int, [_VP, ctypes.c_int, _VP, ctypes.POINTER(ctypes.c_double)]),
    "plan_autotune": (ctypes.c_int, [_VP, _VP, ctypes.c_int, _VP, ctypes.POINTER(ctypes.c_double)]),
    "tuned_variant": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "set_tuned_variant": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int]),
    "server_create": (_VP, [ctypes.c_int, ctypes.c_size_t, ctypes.c_int]),
    "server_submit": (ctypes.c_longlong, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_double,
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_int, _VP, _VP]),
    "server_wait": (ctypes.c_int, [_VP, ctypes.c_longlong, _VP]),
    "server_stats": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_longlong),
                                    ctypes.POINTER(ctypes.c_longlong),
                                    ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_size_t)]),
    "server_usage": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_size_t),
                                    ctypes.POINTER(ctypes.c_size_t)]),
    "server_destroy": (None, [_VP]),
    "projection_rhs": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_double, _VP, _VP]),
    "projection_update": (ctypes.c_int, [_VP, _VP, ctypes.c_double, _VP, _VP, _VP, _VP, _VP]),
    "pressure_correction": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, ctypes.c_double, _VP, _VP]),
    "rk3_predict": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   _VP, _VP, _VP, _VP, _VP, _VP]),
    "rk3_substep": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   _VP, _VP, _VP, _VP, _VP, _VP]),
    "rk3_step": (ctypes.c_int, [_VP, ctypes.c_double, ctypes.c_double, _VP, _VP, _VP, _VP, _VP, _VP,
                                _VP]),
    "refined_noalloc_max_points": (ctypes.c_size_t, []),
    "solve_refined_noalloc": (ctypes.c_int, [_VP, _VP, ctypes.c_double, ctypes.c_int, _VP, _VP]),
}

_lib = None


class PoissonError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"[{code}] {message}")
        self.code = code


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run `python -m paper_1802_10323_amd.build`)")
        # torch ships its own HIP runtime under the same soname as the system
        # one; loading torch first makes this library bind to that runtime,
        # so that both share one runtime (and one device context).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        L = lib()
        msg = L.last_error_message()
        raise PoissonError(rc, msg.decode() if msg else "")
    return rc


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _field_ptr(t, dtype_name="float64"):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("field must be a torch tensor")
    if not t.is_cuda:
        raise ValueError("field must be a device tensor")
    if t.dtype != getattr(torch, dtype_name):
        raise ValueError(f"field must be {dtype_name}")
    if not t.is_contiguous():
        raise ValueError("field must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A solver plan for an nx x ny x nz staggered grid (owns device tables).

    ``dz`` is an array of nz cell widths (z may be stretched); x and y are
    uniform with spacings dx, dy.  ``bcs`` = (bc_x, bc_y, bc_z), each one of
    "P", "NN", "DD", "ND", "DN" (first letter = low face)."""

    def __init__(self, nx, ny, nz, dx, dy, dz, bcs, shift=0.0):
        L = lib()
        dz = np.ascontiguousarray(np.broadcast_to(np.asarray(dz, dtype=np.float64), (nz,)))
        self.shape = (nz, ny, nx)
        self.bcs = tuple(bcs)
        self.shift = float(shift)
        codes = [BC[b] if isinstance(b, str) else int(b) for b in bcs]
        if self.shift == 0.0:
            h = L.plan_create(int(nx), int(ny), int(nz), float(dx), float(dy),
                              dz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), *codes)
        else:   # the Helmholtz operator (A + shift)
            h = L.plan_create_helmholtz(int(nx), int(ny), int(nz), float(dx), float(dy),
                                        dz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), *codes,
                                        self.shift)
        if not h:
            _check(L.last_error() or EINVAL)
        self._h = ctypes.c_void_p(h)

    @classmethod
    def from_problem(cls, p):
        return cls(p.nx, p.ny, p.nz, p.dx, p.dy, p.hz, p.bcs, getattr(p, "shift", 0.0))

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("plan destroyed")
        return self._h

    def solve(self, field, stream=None):
        """Solve in place: ``field`` (float64, device, contiguous, shape
        (nz, ny, nx)) holds f on entry and Phi on exit (asynchronous)."""
        if tuple(field.shape) != self.shape and field.numel() != int(np.prod(self.shape)):
            raise ValueError(f"field shape {tuple(field.shape)} != {self.shape}")
        _check(lib().solve(self.handle, _field_ptr(field), _stream_handle(stream)))
        return field

    def solve_refined_noalloc(self, field, tol=1e-10, max_iters=4, status=None, stream=None):
        """FP32 + FP64 refinement solve of ``field`` in place on the
        library's static workspace (allocates nothing; see
        ``solve_refined_noalloc`` in include/poisson.h).  ``status``: optional
        device float64 tensor of 3 values, filled at the end of the stream
        with (FP32 solves, converged 1/0, last relative update)."""
        if field.numel() != int(np.prod(self.shape)):
            raise ValueError(f"field shape {tuple(field.shape)} != {self.shape}")
        sp = None
        if status is not None:
            if status.numel() < 3:
                raise ValueError("status needs 3 values")
            sp = _field_ptr(status)
        _check(lib().solve_refined_noalloc(self.handle, _field_ptr(field), float(tol),
                                           int(max_iters), sp, _stream_handle(stream)))
        return field

    def velocity_shapes(self):
        """Shapes (z, y, x order) of the face arrays u, v, w: one more face
        along a walled axis than cells."""
        nz, ny, nx = self.shape
        walled = [0 if (b == "P" or b == 0) else 1 for b in self.bcs]
        return ((nz, ny, nx + walled[0]), (nz, ny + walled[1], nx), (nz + walled[2], ny, nx))

    def _check_velocity(self, u, v, w):
        for t, shp, name in zip((u, v, w), self.velocity_shapes(), "uvw"):
            if t.numel() != int(np.prod(shp)):
                raise ValueError(f"{name} has {t.numel()} values, expected shape {shp}")

    def projection_rhs(self, u, v, w, gamma_dt, rhs, stream=None):
        """rhs = div(u, v, w) / gamma_dt (Eq. (poi_ns)) at the cells."""
        self._check_velocity(u, v, w)
        if rhs.numel() != int(np.prod(self.shape)):
            raise ValueError("rhs size does not match the grid")
        _check(lib().projection_rhs(self.handle, _field_ptr(u), _field_ptr(v), _field_ptr(w),
                                    float(gamma_dt), _field_ptr(rhs), _stream_handle(stream)))
        return rhs

    def projection_update(self, phi, gamma_dt, u, v, w, p, stream=None):
        """In place: u, v, w -= gamma_dt grad(phi); p += phi."""
        self._check_velocity(u, v, w)
        for t in (phi, p):
            if t.numel() != int(np.prod(self.shape)):
                raise ValueError("cell field size does not match the grid")
        _check(lib().projection_update(self.handle, _field_ptr(phi), float(gamma_dt),
                                       _field_ptr(u), _field_ptr(v), _field_ptr(w),
                                       _field_ptr(p), _stream_handle(stream)))

    def pressure_correction(self, u, v, w, p, gamma_dt, phi, stream=None):
        """The whole pressure-correction step; phi (cell field) receives the
        correction pressure."""
        self._check_velocity(u, v, w)
        for t in (phi, p):
            if t.numel() != int(np.prod(self.shape)):
                raise ValueError("cell field size does not match the grid")
        _check(lib().pressure_correction(self.handle, _field_ptr(u), _field_ptr(v), _field_ptr(w),
                                         _field_ptr(p), float(gamma_dt), _field_ptr(phi),
                                         _stream_handle(stream)))
        return phi

    def _check_step_fields(self, vel, work, ad, p, phi):
        n = int(np.prod(self.shape))
        for t, m, name in ((vel, 3 * n, "vel"), (work, 3 * n, "work"), (ad, 6 * n, "ad"),
                           (p, n, "p"), (phi, n, "phi")):
            if t.numel() != m:
                raise ValueError(f"{name} has {t.numel()} values, expected {m}")

    def rk3_predict(self, k, dt, nu, vel, work, ad, p, rhs, stream=None):
        """The prediction u* of substep k into work (and AD into ad) and the
        right-hand side div(u*) / (gamma_k dt) into rhs (Eq. (up),
        Eq. (poi_ns))."""
        self._check_step_fields(vel, work, ad, p, rhs)
        _check(lib().rk3_predict(self.handle, int(k), float(dt), float(nu), _field_ptr(vel),
                                 _field_ptr(work), _field_ptr(ad), _field_ptr(p), _field_ptr(rhs),
                                 _stream_handle(stream)))

    def rk3_substep(self, k, dt, nu, vel, work, ad, p, phi, stream=None):
        """Substep k (1, 2, 3) of the Runge-Kutta step with its pressure
        correction (Sec. 2); vel = (u, v, w) stacked, 3 N doubles."""
        self._check_step_fields(vel, work, ad, p, phi)
        _check(lib().rk3_substep(self.handle, int(k), float(dt), float(nu), _field_ptr(vel),
                                 _field_ptr(work), _field_ptr(ad), _field_ptr(p), _field_ptr(phi),
                                 _stream_handle(stream)))

    def rk3_step(self, dt, nu, vel, work, ad, p, phi, scratch, stream=None):
        """One time step: the three substeps (scratch: 2 N doubles)."""
        self._check_step_fields(vel, work, ad, p, phi)
        if scratch.numel() != 2 * int(np.prod(self.shape)):
            raise ValueError(f"scratch has {scratch.numel()} values, expected {2 * int(np.prod(self.shape))}")
        _check(lib().rk3_step(self.handle, float(dt), float(nu), _field_ptr(vel), _field_ptr(work),
                              _field_ptr(ad), _field_ptr(p), _field_ptr(phi), _field_ptr(scratch),
                              _stream_handle(stream)))

    def set_precision(self, mode, tol=1e-10, max_iters=4):
        _check(lib().plan_set_precision(self.handle, int(mode), float(tol), int(max_iters)))

    def status(self):
        """(fp32 solves performed, last relative update, converged) of the
        last solve; valid once its stream has completed."""
        it = ctypes.c_int(0)
        rel = ctypes.c_double(0.0)
        rc = lib().solve_status(self.handle, ctypes.byref(it), ctypes.byref(rel))
        if rc not in (OK, ENOTCONVERGED):
            _check(rc)
        return it.value, rel.value, rc == OK

    @property
    def roles(self):
        r = (ctypes.c_int * 3)()
        _check(lib().plan_roles(self.handle, r))
        return tuple(AXES[i] for i in r)

    @property
    def workspace_bytes(self):
        return int(lib().plan_workspace_bytes(self.handle))

    def transform_stage(self, role, inverse, field, stream=None):
        _check(lib().transform_stage(self.handle, int(role), int(bool(inverse)),
                                     _field_ptr(field), _stream_handle(stream)))
        return field

    def tridiag_stage(self, field, stream=None):
        _check(lib().tridiag_stage(self.handle, _field_ptr(field), _stream_handle(stream)))
        return field

    def autotune(self, scratch, reps=5, stream=None):
        """Time every kernel variant of this plan on ``scratch`` (a device
        float64 tensor of the field's size, overwritten) and record the
        fastest per length; returns the timing report (ms) as
        {"fp64"|"fp32": {"t1": [8], "t2": [8], "elimination": [4]}}
        (-1 where a variant does not apply)."""
        if scratch.numel() < int(np.prod(self.shape)):
            raise ValueError("scratch is smaller than the field")
        rep = (ctypes.c_double * 40)()
        _check(lib().plan_autotune(self.handle, _field_ptr(scratch), int(reps),
                                   _stream_handle(stream), rep))
        out = {}
        for k, name in enumerate(("fp64", "fp32")):
            r = list(rep)[20 * k:20 * (k + 1)]
            out[name] = {"t1": r[0:8], "t2": r[8:16], "elimination": r[16:20]}
        return out

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_solve(plans, fields, stream=None):
    """Solve many independent problems (FP64 plans) in one batched launch
    sequence; fields[i] is solved in place with plans[i]."""
    n = len(plans)
    if len(fields) != n:
        raise ValueError("plans and fields differ in length")
    hp = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    fp = (ctypes.c_void_p * n)(*[_field_ptr(f).value for f in fields])
    _check(lib().batch_solve(hp, fp, n, _stream_handle(stream)))
    return fields


class Batch:
    """Many independent problems solved by one persistent launch per stage
    (``batch_create`` / ``batch_bind`` / ``batch_launch``): all FP64 plans,
    or all FP32 + refinement plans (each FP32 solve batched, the refinement
    kernels batched between them; ``Plan.status`` reports each plan's
    refinement afterwards).  The plans must outlive the batch; ``bind`` sets
    the fields (device, float64, contiguous; solved in place) and must not be
    called while a launch of this batch is in flight."""

    def __init__(self, plans):
        L = lib()
        self.plans = list(plans)
        hp = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        h = L.batch_create(hp, len(self.plans))
        if not h:
            _check(L.last_error() or EINVAL)
        self._h = ctypes.c_void_p(h)

    def bind(self, fields):
        if len(fields) != len(self.plans):
            raise ValueError("one field per plan")
        for p, f in zip(self.plans, fields):
            if f.numel() != int(np.prod(p.shape)):
                raise ValueError(f"field of {f.numel()} values for a {p.shape} plan")
        fp = (ctypes.c_void_p * len(fields))(*[_field_ptr(f).value for f in fields])
        _check(lib().batch_bind(self._h, fp))

    def launch(self, stream=None, graph=False):
        """Enqueue the five stage launches (or replay them as a HIP graph)."""
        _check(lib().batch_launch(self._h, _stream_handle(stream), int(bool(graph))))

    def autotune(self, reps=5, stream=None):
        """Pick the variant of each step for this batch as a whole
        (``batch_autotune``); overwrites the bound fields.  Returns the
        timings (ms) per step: [table, variant 0, 1, 2, 3], -1 where a
        variant does not apply."""
        rep = (ctypes.c_double * 25)()
        _check(lib().batch_autotune(self._h, int(reps), _stream_handle(stream), rep))
        r = list(rep)
        steps = ("fwd_t1", "fwd_t2", "tridiag", "inv_t2", "inv_t1")
        return {s: r[5 * k:5 * (k + 1)] for k, s in enumerate(steps)}

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RequestInfo(ctypes.Structure):
    """poisson_request_info of include/poisson.h."""
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("plan_cached", ctypes.c_int),
                ("last_update_rel", ctypes.c_double), ("submit_s", ctypes.c_double),
                ("start_s", ctypes.c_double), ("done_s", ctypes.c_double),
                ("points", ctypes.c_longlong)]


class Server:
    """Continuous-batching solve server (``server_create`` ...): requests are
    admitted in arrival order as stream slots and HBM budget free up, and run
    concurrently on the device.  Fields are solved in place and must stay
    alive until ``wait`` returns for them (this object keeps a reference)."""

    def __init__(self, slots=8, hbm_budget=0, max_plans=4096):
        L = lib()
        h = L.server_create(int(slots), int(hbm_budget), int(max_plans))
        if not h:
            _check(L.last_error() or EINVAL)
        self._h = ctypes.c_void_p(h)
        self._fields = {}

    def submit(self, problem, field, precision=FP64, tol=1e-10, max_iters=4, stream=None):
        """Queue the solve of ``problem`` (an inputs.Problem or anything with
        nx, ny, nz, dx, dy, hz, bcs) on ``field`` (device float64, contiguous),
        after the work already enqueued on ``stream`` (default: torch's
        current stream, where the field was written); returns the request
        id."""
        dz = np.ascontiguousarray(np.asarray(problem.hz, dtype=np.float64))
        if field.numel() != problem.nx * problem.ny * problem.nz:
            raise ValueError("field size does not match the problem")
        codes = [BC[b] if isinstance(b, str) else int(b) for b in problem.bcs]
        rid = lib().server_submit(self._h, int(problem.nx), int(problem.ny), int(problem.nz),
                                  float(problem.dx), float(problem.dy),
                                  dz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), *codes,
                                  int(precision), float(tol), int(max_iters),
                                  _field_ptr(field), _stream_handle(stream))
        if rid < 0:
            _check(int(rid))
        self._fields[rid] = field
        return rid

    def wait(self, rid):
        """Block until request ``rid`` is done; returns its RequestInfo as a
        dict (times in host steady-clock seconds)."""
        info = RequestInfo()
        rc = lib().server_wait(self._h, int(rid), ctypes.byref(info))
        self._fields.pop(rid, None)
        if rc not in (OK, ENOTCONVERGED):
            _check(rc)
        return {k: getattr(info, k) for k, _ in RequestInfo._fields_}

    def stats(self):
        hits, misses = ctypes.c_longlong(0), ctypes.c_longlong(0)
        resident, budget = ctypes.c_int(0), ctypes.c_size_t(0)
        _check(lib().server_stats(self._h, ctypes.byref(hits), ctypes.byref(misses),
                                  ctypes.byref(resident), ctypes.byref(budget)))
        return {"plan_hits": hits.value, "plan_misses": misses.value,
                "plans_resident": resident.value, "hbm_budget": budget.value}

    def usage(self):
        """Device bytes the server holds now and the peak of held bytes plus
        admitted fields."""
        held, peak = ctypes.c_size_t(0), ctypes.c_size_t(0)
        _check(lib().server_usage(self._h, ctypes.byref(held), ctypes.byref(peak)))
        return {"held_bytes": held.value, "peak_bytes": peak.value}

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().server_destroy(self._h)
            self._h = None
            self._fields.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def refined_noalloc_max_points():
    """Largest grid (points) that ``Plan.solve_refined_noalloc`` accepts."""
    return int(lib().refined_noalloc_max_points())


def tuned_variant(family, n, layout, fp64=True):
    """Variant in the autotuner's table (family 0 transform, 1 elimination;
    layout 0 strided, 1 contiguous)."""
    v = lib().tuned_variant(int(family), int(n), int(layout), int(bool(fp64)))
    if v < 0:
        _check(v)
    return v


def set_tuned_variant(family, n, layout, variant, fp64=True):
    _check(lib().set_tuned_variant(int(family), int(n), int(layout), int(bool(fp64)), int(variant)))
