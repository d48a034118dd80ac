"""MI355X (gfx950) smoothed-aggregation AMG + CG for 3D elasticity in 3x3 block form.

The solve phase runs in hand-written HIP kernels behind the C ABI declared in
include/saamg.h; the hierarchy is built on the host in FP64 by the same
library.  This package only marshals arguments (ctypes) and uses PyTorch for
device memory and streams.
"""
from . import _capi
from ._capi import AmgError, load, library_path
from .hierarchy import HostHierarchy, make_params
from .solver import Solver, BatchSolver

__all__ = ["AmgError", "load", "library_path", "HostHierarchy", "make_params", "Solver",
           "BatchSolver"]
