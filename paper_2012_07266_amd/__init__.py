"""MI355X (gfx950) hot path of the MADLens lensing simulator (arXiv 2012.07266).

The work runs in libmadlens_amd.so (hand-written HIP kernels behind a C ABI,
include/madlens.h); this package marshals torch tensors into it.
"""
from ._lib import lib, MadlensError  # noqa: F401
from .sim import Simulation, footprint  # noqa: F401
