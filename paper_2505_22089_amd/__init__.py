"""MI355X-native cascade-hashing feature matcher.

The package holds the seeded workload generator (``synth``) and the thin
ctypes binding (``chm``) over the C-ABI library ``libchm.so`` whose kernels
are hand-written HIP for gfx950.  Importing the package loads nothing; the
binding loads the library on first use and raises if it is missing.
"""
__all__ = ["synth", "chm"]
