"""MI355X (gfx950) HBS-preconditioned Lippmann-Schwinger solver.

The compute path is the HIP library ``liblsh.so`` (C ABI in include/lsh.h);
``paper_2007_12718_amd.lsh`` is its ctypes binding.
"""
from . import lsh  # noqa: F401
