"""MI355X-native interpolation-based H^2 matrices for Galerkin BEM.

The compute path is libh2mi355x.so (HIP kernels for gfx950 behind the C ABI
of include/h2.h); `h2` is its ctypes binding.  Importing this package does not
load the library; the first call into `h2` does, and fails loudly if the
library has not been built.
"""
from . import h2  # noqa: F401

__all__ = ["h2"]
