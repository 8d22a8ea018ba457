"""MI355X-native block stochastic gradient descent (BSGD) for tomographic reconstruction.

The hot path (Siddon forward projection of sampled rays, matched back projection
into sampled blocks, the importance-sampled block step and the TV proximal step)
runs in hand-written HIP kernels for gfx950 behind the C ABI in include/bsgd.h;
``paper_1903_11874_amd.bsgd`` is the ctypes binding.
"""
from .bsgd import Geometry, Solver, solve, step_batch, normal_residual, BsgdError, load_library, LIB_PATH

__all__ = ["Geometry", "Solver", "solve", "step_batch", "normal_residual", "BsgdError", "load_library", "LIB_PATH"]
