"""MI355X-native planar photoacoustic operator A, its adjoint A^T and FISTA.

The compute path is the HIP library ``libpat.so`` (built for gfx950) behind
the C ABI declared in ``include/pat.h``; this package is a thin ctypes
binding over it plus the method-level helpers (autograd wrapper, server).
Importing the package loads nothing; the library is opened on first use and
a missing or unloadable library is an error, never a fallback.
"""
