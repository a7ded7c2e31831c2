"""The 512 x 256 x 192 channel (P, P, NN; tanh-stretched z) with a
manufactured right-hand side of 64 discrete eigenmodes (Fourier x and y,
eigenvectors of the stretched z operator, the benchmark generator's
seeded draws; tests/channel_modes.py) against its exact discrete solution,
in the launch configuration the benchmark times: FP64 within 1e-12
relative L2 and FP32 + FP64 refinement within 1e-10 (Sec. 2.1, Table 1;
the finite-volume rows of the non-uniform axis)."""
import numpy as np
import pytest

from channel_modes import manufactured_channel
from gpu_util import gpu_solve, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def channel():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_10323_amd import lib
    lib()
    return manufactured_channel(seed=0)


@pytest.mark.parametrize("mixed,tol", [(False, 1e-12), (True, 1e-10)])
def test_channel_manufactured_solution(channel, mixed, tol):
    prob, exact = channel
    got, status = gpu_solve(prob, mixed=mixed)
    err = rel_l2(got, exact)
    print("channel eigenmodes", "FP32+refinement" if mixed else "FP64", "rel-L2 vs exact", err,
          "status", status, flush=True)
    assert err <= tol
