"""Subcycled RK4 with dense-output refinement-boundary ghosts on one MI355X.

The compute path is libsubcyc.so (HIP kernels for gfx950 behind a C ABI,
declared in include/subcyc.h); this package is its ctypes binding.
"""
from .binding import *  # noqa: F401,F403
from .binding import Context, ScError, lib  # noqa: F401
