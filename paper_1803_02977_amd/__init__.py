"""MI355X (gfx950) implementation of the per-timestep hot path of R. Barnes,
"Accelerating a Landscape Evolution Model with Parallelism" (arXiv:1803.02977).

The computation lives in hand-written HIP kernels behind the C ABI declared in
``include/lem.h`` (``liblem.so``); ``lem`` is its ctypes binding.
"""
from .lem import *  # noqa: F401,F403
from .lem import Batch, MfdSolver, Solver, LemError, load, EXPORTS  # noqa: F401
