"""MI355X (gfx950) vertex-patch smoother with nested matrix-free p-multigrid
local solvers (arXiv 2510.17785), behind the C ABI of include/pmg.h.

    from paper_2510_17785_amd import PatchSmoother, GMGSolver

The compute path is libpmg.so (HIP kernels, built in-tree by
`python -m paper_2510_17785_amd.build`); torch provides device memory and
streams.  Importing this package does not load the library; constructing a
solver does, and fails loudly when it is missing.
"""
from .api import (BoundNet, GMGSolver, PatchBatch, PatchSmoother, SimplexBatch,  # noqa: F401
                  SmootherBatch, n_features, simplex_numbering)
from . import _lib  # noqa: F401

__all__ = ["PatchSmoother", "PatchBatch", "SmootherBatch", "SimplexBatch", "BoundNet", "GMGSolver",
           "n_features", "simplex_numbering"]
