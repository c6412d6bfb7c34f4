"""MI355X (gfx950) Aggregate Risk Analysis: HIP kernels behind a C ABI.

The library (libara.so, built from csrc/) exports the calls declared in
include/ara.h; ``ara`` is its ctypes binding.  Importing the package loads
nothing; the first binding call loads the library or raises.
"""

__all__ = ["ara"]
