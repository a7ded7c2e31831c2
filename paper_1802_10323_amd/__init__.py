"""MI355X (gfx950) direct solver for the staggered second-order Poisson
equation by eigenfunction expansion: hand-written HIP kernels behind a C ABI
(``include/poisson.h``), with a thin Python binding (``poisson``)."""
from .poisson import (BC, FP32_REFINED, FP64, Batch, Plan, PoissonError, Server,  # noqa: F401
                      batch_solve, lib, refined_noalloc_max_points, set_tuned_variant,
                      tuned_variant)
