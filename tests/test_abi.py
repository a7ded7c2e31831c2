"""The C ABI library without a GPU: it loads, exports every function that
include/poisson.h declares (with C linkage), the binding's signature table
covers exactly those, and argument validation fails loudly before any
device call."""
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1802_10323_amd import poisson as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "poisson.h")

needs_lib = pytest.mark.skipif(not os.path.exists(P.LIB_PATH), reason="library not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*[A-Za-z_][\w\s\*]*?[\s\*](\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("plan_create", "solve", "plan_destroy", "last_error", "last_error_message",
                     "plan_set_precision", "plan_workspace_bytes", "solve_status", "batch_solve",
                     "plan_roles", "transform_stage", "tridiag_stage"):
        assert required in names
    assert set(names) == set(P.SIGNATURES)


@needs_lib
def test_library_exports_every_declared_symbol():
    L = P.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for name in declared_functions():
        assert name in exported, f"{name} not exported with C linkage"


@needs_lib
@pytest.mark.parametrize("args,code", [
    ((0, 4, 4, 1.0, 1.0, "P", "P", "NN"), P.EINVAL),
    ((4, 4, 4, -1.0, 1.0, "P", "P", "NN"), P.EINVAL),
    ((4, 4, 4, 1.0, float("nan"), "P", "P", "NN"), P.EINVAL),
    ((4, 4, 4, 1.0, 1.0, "P", "P", 7), P.EINVAL),
    ((7, 4, 4, 1.0, 1.0, "P", "P", "NN"), P.EUNSUPPORTED),        # odd transformed length
    ((14, 4, 4, 1.0, 1.0, "P", "P", "NN"), P.EUNSUPPORTED),       # n/2 = 7
    ((2048, 4, 4, 1.0, 1.0, "P", "P", "NN"), P.EUNSUPPORTED),     # too long
    ((4, 4, 600, 1.0, 1.0, "P", "P", "NN"), P.EUNSUPPORTED),      # elimination axis > 512
    ((2, 4, 4, 1.0, 1.0, "P", "P", "P"), P.EUNSUPPORTED),         # periodic s = x with n < 3
])
def test_plan_create_rejects(args, code):
    nx, ny, nz, dx, dy, bx, by, bz = args
    with pytest.raises(P.PoissonError) as ei:
        P.Plan(nx, ny, nz, dx, dy, np.ones(max(nz, 1)), (bx, by, bz))
    assert ei.value.code == code
    assert P.lib().last_error() == code
    assert P.lib().last_error_message()


@needs_lib
def test_bad_dz_rejected():
    dz = np.ones(6)
    dz[3] = 0.0
    with pytest.raises(P.PoissonError) as ei:
        P.Plan(4, 4, 6, 1.0, 1.0, dz, ("P", "P", "NN"))
    assert ei.value.code == P.EINVAL


@needs_lib
def test_null_plan_calls_fail():
    L = P.lib()
    assert L.solve(None, None, None) == P.EINVAL
    assert L.tridiag_stage(None, None, None) == P.EINVAL
    assert L.plan_set_precision(None, 0, 1e-10, 4) == P.EINVAL
    assert L.plan_workspace_bytes(None) == 0
    L.plan_destroy(None)
    assert L.batch_solve(None, None, -1, None) == P.EINVAL
