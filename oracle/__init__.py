"""FP64 CPU oracle of the hybrid LBM / finite-difference Ericksen-Leslie step.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark; the product package never imports it.
"""
from .oracle import Oracle, OracleParams, build, lattice, equilibrium, guo_source  # noqa: F401
