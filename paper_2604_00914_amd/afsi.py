"""Thin Python binding of ``libafsi.so`` (include/afsi.h).

Argument marshalling only: every entry point forwards to the C function of the
same name.  Dense blocks are torch tensors on the GPU (2-D, unit column stride);
host arrays are numpy arrays.  A missing or unloadable library raises
:class:`AfsiError`; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libafsi.so")

R64, R32, C128, C64 = 0, 1, 2, 3
DAMP_NONE, DAMP_JACKSON, DAMP_LANCZOS = 0, 1, 2
_DAMPING = {"none": DAMP_NONE, "jackson": DAMP_JACKSON, "lanczos": DAMP_LANCZOS}

STATUS = {
    0: "OK", -1: "E_INVALID", -2: "E_NOMEM", -3: "E_HIP", -4: "E_NOT_HPD",
    -5: "E_BOUNDS", -6: "E_NOCONV", -7: "E_BUSY", -8: "E_NODEVICE",
}


class AfsiError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class afsi_block(C.Structure):
    _fields_ = [("ptr", C.c_void_p), ("rows", C.c_int64), ("cols", C.c_int64),
                ("ld", C.c_int64), ("dtype", C.c_int32)]


class afsi_step_group(C.Structure):
    _fields_ = [("col0", C.c_int64), ("ncols", C.c_int64), ("src", C.c_int32),
                ("dst", C.c_int32), ("has_v", C.c_int32), ("active", C.c_int32),
                ("sigma", C.c_double), ("tau", C.c_double), ("alpha", C.c_double)]


class afsi_slice_blocks(C.Structure):
    _fields_ = [("step", afsi_step_group), ("X", C.c_void_p), ("P0", C.c_void_p), ("P1", C.c_void_p),
                ("ld", C.c_int64)]


class afsi_options(C.Structure):
    _fields_ = [("kmax", C.c_int32), ("k_init", C.c_int32), ("adaptive", C.c_int32),
                ("damping", C.c_int32), ("m_exp", C.c_double), ("tau_a", C.c_double),
                ("tau_c", C.c_double), ("C", C.c_double), ("max_iter", C.c_int32),
                ("filter_dtype", C.c_int32)]


class afsi_result(C.Structure):
    _fields_ = [("count", C.c_int64), ("iterations", C.c_int32), ("converged", C.c_int32),
                ("spmv", C.c_int64), ("avg_degree", C.c_double),
                ("time_filter_ms", C.c_double), ("time_orth_ms", C.c_double),
                ("time_rr_ms", C.c_double), ("time_resid_ms", C.c_double),
                ("time_host_ms", C.c_double)]


class afsi_lanczos_options(C.Structure):
    _fields_ = [("degree", C.c_int32), ("damping", C.c_int32), ("m_exp", C.c_double),
                ("block", C.c_int32), ("basis", C.c_int32), ("tau_c", C.c_double),
                ("max_cycles", C.c_int32), ("mixed", C.c_int32)]


class afsi_lanczos_result(C.Structure):
    _fields_ = [("count", C.c_int64), ("cycles", C.c_int32), ("converged", C.c_int32),
                ("filter_columns", C.c_int64), ("locked_outside", C.c_int64), ("time_ms", C.c_double)]


class afsi_request_info(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("count", C.c_int64),
                ("iterations", C.c_int32), ("converged", C.c_int32), ("spmv", C.c_int64),
                ("avg_degree", C.c_double), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double)]


class afsi_server_stats(C.Structure):
    _fields_ = [("bytes_in_use", C.c_int64), ("budget", C.c_int64), ("queued", C.c_int64),
                ("running", C.c_int64), ("done", C.c_int64), ("pools", C.c_int64),
                ("batched_launches", C.c_int64), ("batched_groups", C.c_int64),
                ("kernel_launches", C.c_int64), ("kernel_slices", C.c_int64), ("now", C.c_double)]


class afsi_slice_filter(C.Structure):
    _fields_ = [("coeffs", C.c_void_p), ("degree", C.c_int32), ("X", C.c_void_p), ("Y", C.c_void_p),
                ("work", C.c_void_p), ("ncols", C.c_int64), ("ld", C.c_int64)]


_P = C.c_void_p
_I64P = C.POINTER(C.c_int64)
_DP = C.POINTER(C.c_double)
_BP = C.POINTER(afsi_block)
_SIGS = {
    "afsi_last_error": (C.c_char_p, []),
    "afsi_version": (C.c_char_p, []),
    "afsi_device_count": (C.c_int, []),
    "afsi_matrix_create_csr": (C.c_int, [C.c_int, C.c_int64, C.c_int64, _P, _P, _P, C.c_int32, C.POINTER(_P)]),
    "afsi_matrix_destroy": (C.c_int, [_P]),
    "afsi_matrix_set_column_block": (C.c_int, [_P, C.c_int64]),
    "afsi_matrix_get_column_block": (C.c_int, [_P, _I64P]),
    "afsi_matrix_info": (C.c_int, [_P, _I64P, _I64P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "afsi_set_spectral_bounds": (C.c_int, [_P, C.c_double, C.c_double]),
    "afsi_get_spectral_bounds": (C.c_int, [_P, _DP, _DP]),
    "afsi_estimate_spectral_bounds": (C.c_int, [_P, C.c_int, C.c_uint64, _P, _DP, _DP]),
    "afsi_filter_coefficients": (C.c_int, [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int32, C.c_double, _P]),
    "afsi_filter_block": (C.c_int, [_P, _P, C.c_int, _BP, _BP, _BP, _P]),
    "afsi_filter_block_profiled": (C.c_int, [_P, _P, C.c_int, _BP, _BP, _BP, _P, _P, _P]),
    "afsi_estimate_eigencount": (C.c_int, [_P, C.c_double, C.c_double, C.c_int, C.c_int32, C.c_double, _BP, _BP, _BP, _P, _DP, _P]),
    "afsi_spmm": (C.c_int, [_P, _BP, _BP, _P]),
    "afsi_clenshaw_step_params": (C.c_int, [_P, C.c_int, C.c_int, C.c_double, C.c_double, C.POINTER(afsi_step_group)]),
    "afsi_clenshaw_step_batched": (C.c_int, [_P, C.c_int, C.POINTER(afsi_step_group), _BP, _BP, _BP, _P]),
    "afsi_clenshaw_step_grouped": (C.c_int, [_P, C.c_int, C.POINTER(afsi_slice_blocks), C.c_int32, _P]),
    "afsi_filter_batched": (C.c_int, [_P, C.c_int, C.POINTER(afsi_slice_filter), C.c_int32, _P]),
    "afsi_block_size": (C.c_int, [C.c_double, C.c_double, C.c_int64, _I64P]),
    "afsi_block_inner": (C.c_int, [_BP, _BP, _BP, _P]),
    "afsi_block_gemm": (C.c_int, [_BP, _BP, C.c_double, _BP, _P]),
    "afsi_orthonormalize": (C.c_int, [_BP, _BP, _BP, _P]),
    "afsi_rayleigh_ritz": (C.c_int, [_P, _BP, _BP, _BP, _P, _P]),
    "afsi_orthonormalize_rayleigh_ritz": (C.c_int, [_P, _BP, _BP, _BP, _BP, _P, _P]),
    "afsi_residual_norms": (C.c_int, [_BP, _BP, _P, _P, _P]),
    "afsi_residual_norms_noalloc": (C.c_int, [_BP, _BP, _P, _P, _P]),
    "afsi_convert_block": (C.c_int, [_BP, _BP, _P]),
    "afsi_gather_columns": (C.c_int, [_BP, _P, C.c_int64, _BP, _P]),
    "afsi_permute_rows": (C.c_int, [_BP, _P, C.c_int32, _BP, _P]),
    "afsi_grid_order": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, C.c_int64, C.c_int64, C.c_int32, _P]),
    "afsi_csr_permute": (C.c_int, [C.c_int64, C.c_int64, _P, _P, _P, C.c_int32, _P, _P, _P, _P]),
    "afsi_select_degree": (C.c_int, [_P, C.c_int64, C.c_int64, _P, C.c_int, C.c_double, C.c_double, C.c_double, C.POINTER(C.c_int)]),
    "afsi_lock_select": (C.c_int, [_P, C.c_int64, _P, _P, C.c_double, C.c_double, C.c_double, C.c_int64, _I64P, _P, C.POINTER(C.c_int)]),
    "afsi_host_eigh": (C.c_int, [C.c_int64, C.c_int32, _P, C.c_int64, _P, _P, C.c_int64]),
    "afsi_host_cholesky_inverse": (C.c_int, [C.c_int64, C.c_int32, _P, C.c_int64, C.c_double]),
    "afsi_options_default": (None, [C.POINTER(afsi_options), C.c_int]),
    "afsi_solve": (C.c_int, [_P, C.c_double, C.c_double, C.POINTER(afsi_options), _BP, _BP, C.c_int64, _P, _P, C.POINTER(afsi_result), _P]),
    "afsi_lanczos_options_default": (None, [C.POINTER(afsi_lanczos_options), C.c_int]),
    "afsi_filtered_lanczos": (C.c_int, [_P, C.c_double, C.c_double, C.POINTER(afsi_lanczos_options), _BP, _BP, C.c_int64, _P, _P, C.POINTER(afsi_lanczos_result), _P]),
    "afsi_server_create": (C.c_int, [C.c_int, C.c_int64, C.POINTER(_P)]),
    "afsi_server_destroy": (C.c_int, [_P]),
    "afsi_server_set_pool_columns": (C.c_int, [_P, _P, C.c_int64]),
    "afsi_server_submit": (C.c_int, [_P, _P, C.c_double, C.c_double, C.c_int64, C.POINTER(afsi_options), C.c_uint64, _I64P]),
    "afsi_server_info": (C.c_int, [_P, C.c_int64, C.POINTER(afsi_request_info)]),
    "afsi_server_wait": (C.c_int, [_P, C.c_int64, C.c_double, C.POINTER(afsi_request_info)]),
    "afsi_server_wait_any": (C.c_int, [_P, C.c_double, _I64P]),
    "afsi_server_fetch": (C.c_int, [_P, C.c_int64, _P, _P, C.c_int64, _BP, _P]),
    "afsi_server_get_stats": (C.c_int, [_P, C.POINTER(afsi_server_stats)]),
}

_lib = None


def lib():
    """Load libafsi.so (raises AfsiError if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise AfsiError(-8, f"{LIB_PATH} is not built; run paper_2604_00914_amd.build.build()")
        # torch ships its own HIP runtime (same soname as ROCm's).  Loading torch first
        # makes libafsi.so bind to that already-loaded runtime, so one process never
        # holds two HIP runtimes (which leaves the second without devices).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(status: int):
    if status != 0:
        raise AfsiError(status, lib().afsi_last_error().decode())


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ------------------------------------------------------------------ blocks and streams

def block(t, rows: int | None = None, cols: int | None = None) -> afsi_block:
    """afsi_block describing a 2-D CUDA tensor (row-major, unit column stride)."""
    import torch

    dt = {torch.float64: R64, torch.float32: R32, torch.complex128: C128, torch.complex64: C64}.get(t.dtype)
    if dt is None:
        raise AfsiError(-1, f"unsupported tensor dtype {t.dtype}")
    if t.dim() != 2 or (t.numel() > 0 and t.stride(1) != 1):
        raise AfsiError(-1, "block tensors must be 2-D with unit column stride")
    if not t.is_cuda:
        raise AfsiError(-1, "block tensors must live on the GPU")
    r, c = t.shape
    return afsi_block(t.data_ptr(), r if rows is None else rows, c if cols is None else cols,
                      max(t.stride(0), 1), dt)


def _bref(b):
    return C.byref(b) if b is not None else None


def current_stream():
    import torch

    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _stream(s):
    if s is None:
        return current_stream()
    if isinstance(s, C.c_void_p):
        return s
    return C.c_void_p(getattr(s, "cuda_stream", s))


# ------------------------------------------------------------------ entry points

def afsi_version() -> str:
    return lib().afsi_version().decode()


def afsi_device_count() -> int:
    return lib().afsi_device_count()


def afsi_matrix_create_csr(device: int, n: int, nnz: int, row_ptr, col_idx, vals, val_dtype: int):
    rp = _np(row_ptr, np.int64)
    ci = _np(col_idx, np.int32)
    va = _np(vals, np.complex128 if val_dtype == C128 else np.float64)
    h = C.c_void_p()
    _check(lib().afsi_matrix_create_csr(device, n, nnz, _ptr(rp), _ptr(ci), _ptr(va), val_dtype, C.byref(h)))
    return h


def afsi_matrix_destroy(h):
    _check(lib().afsi_matrix_destroy(h))


def afsi_matrix_info(h):
    n, nnz, dt, dev = C.c_int64(), C.c_int64(), C.c_int32(), C.c_int32()
    _check(lib().afsi_matrix_info(h, C.byref(n), C.byref(nnz), C.byref(dt), C.byref(dev)))
    return n.value, nnz.value, dt.value, dev.value


def afsi_set_spectral_bounds(h, lmin: float, lmax: float):
    _check(lib().afsi_set_spectral_bounds(h, lmin, lmax))


def afsi_get_spectral_bounds(h):
    lo, hi = C.c_double(), C.c_double()
    _check(lib().afsi_get_spectral_bounds(h, C.byref(lo), C.byref(hi)))
    return lo.value, hi.value


def afsi_estimate_spectral_bounds(h, steps: int = 40, seed: int = 0, stream=None):
    lo, hi = C.c_double(), C.c_double()
    _check(lib().afsi_estimate_spectral_bounds(h, steps, seed, _stream(stream), C.byref(lo), C.byref(hi)))
    return lo.value, hi.value


def afsi_matrix_set_column_block(h, nbytes: int):
    _check(lib().afsi_matrix_set_column_block(h, int(nbytes)))


def afsi_matrix_get_column_block(h) -> int:
    v = C.c_int64(0)
    _check(lib().afsi_matrix_get_column_block(h, C.byref(v)))
    return v.value


def afsi_filter_coefficients(lmin, lmax, a, b, kmax, damping="jackson", m_exp=0.5) -> np.ndarray:
    out = np.empty(kmax + 1, dtype=np.float64)
    _check(lib().afsi_filter_coefficients(lmin, lmax, a, b, kmax, _DAMPING.get(damping, damping), m_exp, _ptr(out)))
    return out


def afsi_filter_block(h, coeffs, degree: int, X, Y, work, stream=None):
    c = _np(coeffs, np.float64)
    _check(lib().afsi_filter_block(h, _ptr(c), degree, _bref(_blk(X)), _bref(_blk(Y)), _bref(_blk(work)), _stream(stream)))


def afsi_filter_block_profiled(h, coeffs, degree: int, X, Y, work, stream=None):
    """Returns (step_ms[degree], step_kind[degree]); kind bit 0 = in-place V, bit 1 = X term."""
    c = _np(coeffs, np.float64)
    ms = np.zeros(degree, dtype=np.float32)
    kind = np.zeros(degree, dtype=np.int32)
    _check(lib().afsi_filter_block_profiled(h, _ptr(c), degree, _bref(_blk(X)), _bref(_blk(Y)), _bref(_blk(work)),
                                            _stream(stream), _ptr(ms), _ptr(kind)))
    return ms, kind


def afsi_estimate_eigencount(h, a, b, degree: int, Z, Y, work, damping="lanczos", m_exp=0.5, stream=None):
    """Returns (estimate, per_probe[m]): mean and values of Re z_i^H rho(A) z_i."""
    z = _blk(Z)
    per = np.empty(z.cols, dtype=np.float64)
    est = C.c_double(0.0)
    _check(lib().afsi_estimate_eigencount(h, a, b, degree, _DAMPING.get(damping, damping), m_exp, _bref(z),
                                          _bref(_blk(Y)), _bref(_blk(work)), _ptr(per), C.byref(est), _stream(stream)))
    return est.value, per


def afsi_spmm(h, X, Y, stream=None):
    _check(lib().afsi_spmm(h, _bref(_blk(X)), _bref(_blk(Y)), _stream(stream)))


def afsi_clenshaw_step_params(coeffs, degree: int, step: int, l1: float, l2: float,
                              col0: int = 0, ncols: int = 0) -> afsi_step_group:
    c = _np(coeffs, np.float64)
    g = afsi_step_group(col0=col0, ncols=ncols)
    _check(lib().afsi_clenshaw_step_params(_ptr(c), degree, step, l1, l2, C.byref(g)))
    return g


def afsi_clenshaw_step_batched(h, groups, X, P0, P1, stream=None):
    arr = (afsi_step_group * max(len(groups), 1))(*groups)
    _check(lib().afsi_clenshaw_step_batched(h, len(groups), arr, _bref(_blk(X)), _bref(_blk(P0)), _bref(_blk(P1)), _stream(stream)))


def afsi_clenshaw_step_grouped(h, slices, stream=None):
    """slices: list of (afsi_step_group, X, P0, P1) with torch blocks of one dtype, each
    n x step.ncols (its own leading dimension)."""
    arr = (afsi_slice_blocks * max(len(slices), 1))()
    dt = R64
    for i, (g, X, P0, P1) in enumerate(slices):
        bx, b0, b1 = _blk(X), _blk(P0), _blk(P1)
        if not (bx.ld == b0.ld == b1.ld and bx.dtype == b0.dtype == b1.dtype):
            raise AfsiError(-1, "a slice's X, P0, P1 must share ld and dtype")
        arr[i] = afsi_slice_blocks(g, bx.ptr, b0.ptr, b1.ptr, bx.ld)
        dt = bx.dtype
    _check(lib().afsi_clenshaw_step_grouped(h, len(slices), arr, dt, _stream(stream)))


def afsi_filter_batched(h, slices, stream=None):
    """slices: list of (coeffs, degree, X, Y, work) with torch blocks of one dtype, each
    n x ncols (X, Y and work of a slice share their leading dimension)."""
    arr = (afsi_slice_filter * max(len(slices), 1))()
    keep = []
    dt = R64
    for i, (coeffs, degree, X, Y, W) in enumerate(slices):
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        if c.size < degree + 1:
            raise AfsiError(-1, f"slice {i}: {c.size} coefficients for degree {degree}")
        keep.append(c)
        bx, by, bw = _blk(X), _blk(Y), _blk(W)
        if not (bx.ld == by.ld == bw.ld and bx.cols == by.cols == bw.cols
                and bx.dtype == by.dtype == bw.dtype):
            raise AfsiError(-1, "a slice's X, Y, work must share shape, ld and dtype")
        arr[i] = afsi_slice_filter(c.ctypes.data, int(degree), bx.ptr, by.ptr, bw.ptr, bx.cols, bx.ld)
        dt = bx.dtype
    _check(lib().afsi_filter_batched(h, len(slices), arr, dt, _stream(stream)))


def afsi_block_size(estimate: float, mu: float, n: int) -> int:
    """p = ceil(mu * estimate) clipped to [1, n] (Section 3.4)."""
    p = C.c_int64(0)
    _check(lib().afsi_block_size(float(estimate), float(mu), int(n), C.byref(p)))
    return p.value


def afsi_block_inner(X, Y, G, stream=None):
    _check(lib().afsi_block_inner(_bref(_blk(X)), _bref(_blk(Y)), _bref(_blk(G)), _stream(stream)))


def afsi_block_gemm(X, M, beta: float, Y, stream=None):
    _check(lib().afsi_block_gemm(_bref(_blk(X)), _bref(_blk(M)), beta, _bref(_blk(Y)), _stream(stream)))


def afsi_orthonormalize(locked, X, work, stream=None):
    _check(lib().afsi_orthonormalize(_bref(_blk(locked)) if locked is not None else None,
                                     _bref(_blk(X)), _bref(_blk(work)), _stream(stream)))


def afsi_rayleigh_ritz(h, Q, V, AV, stream=None) -> np.ndarray:
    q = _blk(Q)
    ritz = np.empty(q.cols, dtype=np.float64)
    _check(lib().afsi_rayleigh_ritz(h, _bref(q), _bref(_blk(V)), _bref(_blk(AV)), _ptr(ritz), _stream(stream)))
    return ritz


def afsi_orthonormalize_rayleigh_ritz(h, X, work, V, AV, stream=None) -> np.ndarray:
    x = _blk(X)
    ritz = np.empty(x.cols, dtype=np.float64)
    _check(lib().afsi_orthonormalize_rayleigh_ritz(h, _bref(x), _bref(_blk(work)), _bref(_blk(V)),
                                                   _bref(_blk(AV)), _ptr(ritz), _stream(stream)))
    return ritz


def afsi_residual_norms(V, AV, lam, stream=None) -> np.ndarray:
    v = _blk(V)
    lam = _np(lam, np.float64)
    out = np.empty(v.cols, dtype=np.float64)
    _check(lib().afsi_residual_norms(_bref(v), _bref(_blk(AV)), _ptr(lam), _ptr(out), _stream(stream)))
    return out


def afsi_residual_norms_noalloc(V, AV, lam, stream=None) -> np.ndarray:
    v = _blk(V)
    lam = _np(lam, np.float64)
    out = np.empty(v.cols, dtype=np.float64)
    _check(lib().afsi_residual_norms_noalloc(_bref(v), _bref(_blk(AV)), _ptr(lam), _ptr(out),
                                             _stream(stream)))
    return out


def afsi_convert_block(src, dst, stream=None):
    _check(lib().afsi_convert_block(_bref(_blk(src)), _bref(_blk(dst)), _stream(stream)))


def afsi_gather_columns(src, cols, dst, stream=None):
    c = _np(cols, np.int32)
    _check(lib().afsi_gather_columns(_bref(_blk(src)), _ptr(c), c.size, _bref(_blk(dst)), _stream(stream)))


def afsi_permute_rows(src, perm, dst, inverse: bool = False, stream=None):
    """dst row i = src row perm[i]; with inverse, dst row perm[i] = src row i."""
    pm = _np(perm, np.int64)
    _check(lib().afsi_permute_rows(_bref(_blk(src)), _ptr(pm), int(bool(inverse)), _bref(_blk(dst)), _stream(stream)))


def afsi_grid_order(nx: int, ny: int, nz: int, ty: int, tz: int, fold_x: bool = False) -> np.ndarray:
    """Pencil ordering of an nx x ny x nz grid (perm[new] = old); fold_x for a periodic x."""
    perm = np.empty(max(0, nx * ny * nz), dtype=np.int64)
    _check(lib().afsi_grid_order(nx, ny, nz, ty, tz, int(bool(fold_x)), _ptr(perm)))
    return perm


def afsi_csr_permute(csr, perm):
    """P A P^T of a CSR (workloads.CSR fields n, row_ptr, col, val) as a new CSR."""
    from workloads.matrices import CSR

    cplx = np.iscomplexobj(csr.val)
    rp = _np(csr.row_ptr, np.int64)
    ci = _np(csr.col, np.int32)
    v = _np(csr.val, np.complex128 if cplx else np.float64)
    pm = _np(perm, np.int64)
    n, nnz = int(csr.n), int(rp[-1])
    orp = np.empty(n + 1, dtype=np.int64)
    oci = np.empty(nnz, dtype=np.int32)
    ov = np.empty(nnz, dtype=v.dtype)
    _check(lib().afsi_csr_permute(n, nnz, _ptr(rp), _ptr(ci), _ptr(v), C128 if cplx else R64, _ptr(pm),
                                  _ptr(orp), _ptr(oci), _ptr(ov)))
    return CSR(n, orp, oci, ov)


def afsi_select_degree(ritz, e: int, coeffs, l1: float, l2: float, tau_a: float) -> int:
    r = _np(ritz, np.float64)
    c = _np(coeffs, np.float64)
    out = C.c_int()
    _check(lib().afsi_select_degree(_ptr(r), r.size, e, _ptr(c), c.size - 1, l1, l2, tau_a, C.byref(out)))
    return out.value


def afsi_lock_select(ritz, res, in_interval, a, b, tau_abs, n_lock, n_check_prev):
    """Returns (in_interval_after, lock, done, n_check)."""
    r = _np(ritz, np.float64)
    rs = _np(res, np.float64)
    I = _np(in_interval, np.uint8).copy()
    lock = np.zeros(r.size, dtype=np.uint8)
    ncp = C.c_int64(n_check_prev)
    done = C.c_int()
    _check(lib().afsi_lock_select(_ptr(r), r.size, _ptr(rs), _ptr(I), a, b, tau_abs, n_lock, C.byref(ncp), _ptr(lock), C.byref(done)))
    return I.astype(bool), lock.astype(bool), bool(done.value), ncp.value


def afsi_host_eigh(B: np.ndarray):
    cplx = np.iscomplexobj(B)
    Bc = _np(B, np.complex128 if cplx else np.float64)
    p = Bc.shape[0]
    w = np.empty(p)
    U = np.empty_like(Bc)
    _check(lib().afsi_host_eigh(p, C128 if cplx else R64, _ptr(Bc), p, _ptr(w), _ptr(U), p))
    return w, U


def afsi_host_cholesky_inverse(G: np.ndarray, shift: float = 0.0) -> np.ndarray:
    cplx = np.iscomplexobj(G)
    Gc = _np(G, np.complex128 if cplx else np.float64).copy()
    _check(lib().afsi_host_cholesky_inverse(Gc.shape[0], C128 if cplx else R64, _ptr(Gc), Gc.shape[0], shift))
    return Gc


def afsi_options_default(kmax: int) -> afsi_options:
    o = afsi_options()
    lib().afsi_options_default(C.byref(o), kmax)
    return o


def afsi_solve(h, a: float, b: float, opts: afsi_options, X0, evecs, capacity: int | None = None, stream=None):
    """Returns (status, eigenvalues, residuals, afsi_result); E_NOCONV is returned, not raised."""
    e = _blk(evecs)
    cap = e.cols if capacity is None else capacity
    lam = np.zeros(max(cap, 1))
    res = np.zeros(max(cap, 1))
    r = afsi_result()
    st = lib().afsi_solve(h, a, b, C.byref(opts), _bref(_blk(X0)), _bref(e), cap, _ptr(lam), _ptr(res), C.byref(r), _stream(stream))
    if st not in (0, -6):
        _check(st)
    return st, lam[: r.count].copy(), res[: r.count].copy(), r


def afsi_lanczos_options_default(degree: int) -> afsi_lanczos_options:
    o = afsi_lanczos_options()
    lib().afsi_lanczos_options_default(C.byref(o), degree)
    return o


def afsi_filtered_lanczos(h, a: float, b: float, opts: afsi_lanczos_options, X0, evecs,
                          capacity: int | None = None, stream=None):
    """Returns (status, eigenvalues, residuals, afsi_lanczos_result); E_NOCONV is returned,
    not raised."""
    e = _blk(evecs)
    cap = e.cols if capacity is None else capacity
    lam = np.zeros(max(cap, 1))
    res = np.zeros(max(cap, 1))
    r = afsi_lanczos_result()
    st = lib().afsi_filtered_lanczos(h, a, b, C.byref(opts), _bref(_blk(X0)), _bref(e), cap, _ptr(lam),
                                     _ptr(res), C.byref(r), _stream(stream))
    if st not in (0, -6):
        _check(st)
    return st, lam[: r.count].copy(), res[: r.count].copy(), r


def afsi_server_create(device: int, hbm_budget_bytes: int):
    h = C.c_void_p()
    _check(lib().afsi_server_create(device, int(hbm_budget_bytes), C.byref(h)))
    return h


def afsi_server_destroy(S):
    _check(lib().afsi_server_destroy(S))


def afsi_server_set_pool_columns(S, A, cols: int):
    _check(lib().afsi_server_set_pool_columns(S, A, cols))


def afsi_server_submit(S, A, a: float, b: float, p: int, opts: afsi_options, seed: int) -> int:
    rid = C.c_int64()
    _check(lib().afsi_server_submit(S, A, a, b, p, C.byref(opts), seed, C.byref(rid)))
    return rid.value


def afsi_server_info(S, rid: int) -> afsi_request_info:
    info = afsi_request_info()
    _check(lib().afsi_server_info(S, rid, C.byref(info)))
    return info


def afsi_server_wait(S, rid: int, timeout_s: float) -> afsi_request_info:
    info = afsi_request_info()
    _check(lib().afsi_server_wait(S, rid, timeout_s, C.byref(info)))
    return info


def afsi_server_wait_any(S, timeout_s: float) -> int:
    rid = C.c_int64()
    _check(lib().afsi_server_wait_any(S, timeout_s, C.byref(rid)))
    return rid.value


def afsi_server_fetch(S, rid: int, capacity: int, evecs=None, stream=None):
    """Returns (eigenvalues, residuals) and copies eigenvectors into `evecs` if given."""
    lam = np.zeros(max(capacity, 1))
    res = np.zeros(max(capacity, 1))
    info = afsi_server_info(S, rid)
    _check(lib().afsi_server_fetch(S, rid, _ptr(lam), _ptr(res), capacity,
                                   _bref(_blk(evecs)) if evecs is not None else None,
                                   _stream(stream) if evecs is not None else None))
    return lam[: info.count].copy(), res[: info.count].copy()


def afsi_server_get_stats(S) -> afsi_server_stats:
    st = afsi_server_stats()
    _check(lib().afsi_server_get_stats(S, C.byref(st)))
    return st


def _blk(x):
    if x is None or isinstance(x, afsi_block):
        return x
    return block(x)


# ------------------------------------------------------------------ convenience

class Matrix:
    """Owns an afsi_matrix_t built from a CSR (e.g. workloads.CSR)."""

    def __init__(self, csr, device: int = 0, bounds=None):
        cplx = np.iscomplexobj(csr.val)
        self.n = int(csr.n)
        self.nnz = int(csr.row_ptr[-1])
        self.complex = cplx
        self.handle = afsi_matrix_create_csr(device, self.n, self.nnz, csr.row_ptr, csr.col, csr.val, C128 if cplx else R64)
        if bounds is not None:
            afsi_set_spectral_bounds(self.handle, *bounds)

    def close(self):
        if self.handle:
            afsi_matrix_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
