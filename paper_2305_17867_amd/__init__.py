"""MI355X-native PDE-compressed Cartesian-Taylor FMM translation operators.

The compute path is libfmm.so (hand-written HIP for gfx950) behind the C ABI in
include/fmm.h; ``fmm`` is its thin torch binding.  Importing the package does not
load the library; the first call does, and raises if it is not built.
"""
__all__ = ["fmm", "build"]
