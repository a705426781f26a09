"""MI355X solver for the rigidly constrained immersed-boundary Stokes system.

The numerical work happens in ``libibr.so`` (HIP kernels for gfx950 behind the
C ABI of include/ibr.h); ``ibr`` is the thin ctypes binding.
"""
from . import ibr  # noqa: F401
from .ibr import FP64, MIXED, PC_FULL, PC_LOWER, IbrError, Solver, from_problem  # noqa: F401
