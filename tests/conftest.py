import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


FAST_M = [16, 32, 48, 64, 72, 80, 96, 128, 144, 160, 192, 256]
ELIM_LENGTHS = [64, 96, 128, 192, 256, 384, 512]


@pytest.fixture
def default_variants():
    """Put every entry of the kernel-variant table back to what it was
    before the test."""
    from paper_1802_10323_amd import set_tuned_variant, tuned_variant
    keys = [(0, 2 * M, layout, fp64) for M in FAST_M for layout in (0, 1) for fp64 in (True, False)]
    keys += [(1, n, layout, fp64) for n in ELIM_LENGTHS for layout in (0, 1) for fp64 in (True, False)]
    saved = [(k, tuned_variant(*k)) for k in keys]
    yield
    for (family, n, layout, fp64), v in saved:
        set_tuned_variant(family, n, layout, v, fp64)
