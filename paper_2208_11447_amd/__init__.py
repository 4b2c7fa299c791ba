"""skfab: sketched Krylov approximation of f(A) b on AMD Instinct MI355X (gfx950).

The numerical work runs in ``libskfab.so`` (hand-written HIP kernels behind the C
ABI of include/skfab.h); this package holds the build script and a thin ctypes
binding with the same function names.
"""
from . import _native  # noqa: F401

__all__ = ["_native"]
