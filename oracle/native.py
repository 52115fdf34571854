"""Build and load the oracle's C CSR product (``csr_spmm.c``) with gcc + OpenMP.

Test infrastructure only.  The shared object is written next to the source
under ``oracle/_build/`` and is never linked into the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csr_spmm.c")
_OUT = os.path.join(_HERE, "_build", "liboracle_spmm.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile csr_spmm.c into oracle/_build/liboracle_spmm.so."""
    if not force and os.path.exists(_OUT):
        return _OUT
    os.makedirs(os.path.dirname(_OUT), exist_ok=True)
    tmp = _OUT + f".tmp{os.getpid()}"
    subprocess.check_call(
        ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", _SRC, "-o", tmp]
    )
    os.replace(tmp, _OUT)
    return _OUT


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_OUT):
            build()
        L = ctypes.CDLL(_OUT)
        for name in ("oracle_spmm_f64", "oracle_spmm_c128"):
            f = getattr(L, name)
            f.restype = None
            f.argtypes = [
                ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
            ]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.restype = None
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Thread count of later products (for single-thread timing)."""
    lib().oracle_set_num_threads(int(n))


def spmm(A, B: np.ndarray) -> np.ndarray:
    """C = A @ B for a workloads.CSR A and a 2-D block B (float64 or complex128)."""
    L = lib()
    B = np.asarray(B)
    one_d = B.ndim == 1
    if one_d:
        B = B[:, None]
    if B.shape[0] != A.n:
        raise ValueError("shape mismatch")
    row_ptr = np.ascontiguousarray(A.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(A.col, dtype=np.int32)
    cplx = np.iscomplexobj(A.val) or np.iscomplexobj(B)
    dt = np.complex128 if cplx else np.float64
    val = np.ascontiguousarray(A.val, dtype=dt)
    Bc = np.ascontiguousarray(B, dtype=dt)
    C = np.empty((A.n, B.shape[1]), dtype=dt)
    f = L.oracle_spmm_c128 if cplx else L.oracle_spmm_f64
    f(A.n, row_ptr.ctypes.data, col.ctypes.data, val.ctypes.data, Bc.ctypes.data, B.shape[1], C.ctypes.data)
    return C[:, 0] if one_d else C
