"""MI355X-native growing-tissue D2Q9 lattice Boltzmann method (arXiv 2303.02210).

The simulation runs in the gfx950 HIP library ``liblbmgrow.so`` behind the C
ABI of ``include/lbmgrow.h``; this package marshals arguments to it and uses
PyTorch for device memory and streams only.
"""
from ._ffi import LbmError, lib, make_params  # noqa: F401
from .sim import Sim  # noqa: F401
from .ensemble import Ensemble  # noqa: F401

__all__ = ["Sim", "Ensemble", "LbmError", "lib", "make_params"]
