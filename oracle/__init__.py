"""FP64 CPU oracle of the two-component Shan-Chen evaporation step.

Test infrastructure only: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it. The product path (the HIP library and its binding)
never imports it.
"""
from .oracle import Oracle, OracleParams, lattice_tables, feq, build  # noqa: F401
