"""MI355X-native TS2-GauSum split step for the rotating fractional NLS/GPE.

The compute path is libfse.so (hand-written HIP for gfx950 behind a C ABI,
include/fse.h); `fse` is its ctypes binding.  Importing the package does not
load the library; the first call into `fse` does, and raises if it is missing.
"""
__all__ = ["fse"]
