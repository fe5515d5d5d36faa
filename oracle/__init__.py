"""FP64 CPU oracle of the bump-function D3Q19 lattice Boltzmann step.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU-baseline leg use
this package. The GPU library neither imports nor links it, and it shares no code with it.
"""
from .oracle import (OracleLattice, feq, feq_std, beq, table_m, forcing, velocity_set, gradient, project,  # noqa: F401
                     projection_classes,
                     lib_path)
