"""MI355X-native two-component Shan-Chen lattice Boltzmann step with the
mass-conserving evaporation sink (arXiv:1701.03637), behind the lbsc C ABI.

The kernels are hand-written HIP for gfx950 in ``csrc/``; ``lbsc.py`` is the
ctypes binding used by the tests and the benchmark.
"""
from .lbsc import (FLAG_FP16S_SINK, FP16N, FP16S, FP32S, FP64, LbscError, Sim, load_library,  # noqa: F401
                   make_params)
