"""CPU FP64 oracle of the pseudopotential thermal LB step (Li & Luo,
arXiv:1405.2232).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.
"""
from .lbmref import Oracle, PLAIN, CORRECTED, FD_RK2, feq, guo, corr, pressure, sc_force_field, velocities  # noqa: F401
