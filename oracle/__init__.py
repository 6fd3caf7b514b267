"""Plain FP64 CPU oracle of the free-surface LBM time step (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package. It is built from ``fslbm_oracle.c`` with gcc and shares
no code with the GPU library.
"""
from .oracle import Oracle, OracleReport, build_oracle, equilibrium, lattice, opposite  # noqa: F401
from .oracle import collide_cell, reconstruct_set, bc_value  # noqa: F401
