"""MI355X (gfx950) adaptive Chebyshev-filtered subspace iteration.

The compute path is the HIP library ``libafsi.so`` (C ABI in include/afsi.h);
``afsi`` is its thin ctypes binding and ``serve`` the continuous-batching
request loop built on it.  Build with ``paper_2604_00914_amd.build.build()``.
"""
from . import afsi  # noqa: F401
from .afsi import AfsiError, Matrix, block  # noqa: F401

__all__ = ["afsi", "AfsiError", "Matrix", "block"]
