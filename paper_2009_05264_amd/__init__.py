"""MI355X (gfx950) implementation of the coupled pseudopotential / thermal
D2Q9 lattice-Boltzmann step for flow boiling (arXiv:2009.05264).

The compute path is the HIP library ``liblbmflow.so`` (C ABI in
``include/lbmflow.h``); :mod:`.lbmflow` is its ctypes binding.
"""
from . import lbmflow  # noqa: F401
from .lbmflow import Batch, Domain, LbmError, default_params, maxwell  # noqa: F401
