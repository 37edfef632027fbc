"""MI355X-native two-component Shan-Chen lattice Boltzmann step with the
mass-conserving evaporation sink (arXiv:1701.03637), behind the lbsc C ABI.

The kernels are hand-written HIP for gfx950 in ``csrc/``; ``lbsc.py`` is the
ctypes binding used by the tests and the benchmark.
"""
from .lbsc import (FP16S, FP32S, FP64, LbscError, Sim, load_library, make_params)  # noqa: F401
