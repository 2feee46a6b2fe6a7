"""Trajectory-parallel Krotov optimisation on AMD MI355X (gfx950).

The compute path lives in ``libtrajkrotov.so`` (HIP kernels behind a C ABI,
``include/trajkrotov.h``); ``paper_1801_04382_amd.trajkrotov`` is its ctypes
binding.  Importing the binding fails loudly when the library is not built.
"""

__all__ = ["build", "trajkrotov"]
