"""MI355X-native steady gray GSIS / source-iteration solver.

The compute path lives in ``libgsis.so`` (HIP kernels for gfx950 behind the
C-ABI declared in ``include/gsis.h``); :mod:`paper_2507_03975_amd.gsis` is the
thin ctypes binding with the same names. Importing the package loads nothing;
the library is opened on first use and a missing build raises.
"""
__all__ = ["inputs"]
