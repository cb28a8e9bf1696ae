"""CPU FP64 dynamic-relaxation oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  It shares no code with the HIP path.
"""
from .oracle import (  # noqa: F401
    CONVERGED, MAX_ITER, NONFINITE, START_AFFINE, START_ZERO, START_WARM,
    OracleResult, build, derived, energy, evaluate, internal_force, solve, solve_batch,
)
