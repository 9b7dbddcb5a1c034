"""Two-stage preconditioned FGMRES for multiphase poromechanics on AMD MI355X.

The solver lives in libps.so (HIP kernels for gfx950 + host C++ setup) behind the
C ABI of include/ps.h; `ps` is its ctypes binding.
"""
from . import ps  # noqa: F401

__all__ = ["ps"]
