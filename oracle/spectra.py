"""Reference eigenvalues of a real symmetric sparse matrix inside an interval.

Test infrastructure only.  The method's result is, by definition, every eigenvalue
of the Hermitian matrix A inside [a, b], counted with multiplicity (the problem
statement of Section 1).  For a real symmetric matrix whose nonzeros lie within a
band |i - j| <= w (the 3-D grid Laplacians in natural order: w = N^2), LAPACK's
banded symmetric eigensolver computes exactly that set: reduction of the band to
tridiagonal form by orthogonal transformations, then bisection restricted to
[a, b] (scipy.linalg.eigvals_banded with select='v').  The only steps here are
copying A's nonzeros into band storage and that library call.  LAPACK's value range
is half-open, (a, b]; the windows this is used for keep both ends inside spectral
gaps, where the two definitions agree.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def bandwidth(A) -> int:
    """Largest |i - j| over the stored nonzeros of the CSR matrix A."""
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    if rows.size == 0:
        return 0
    return int(np.max(np.abs(A.col.astype(np.int64) - rows)))


def lower_band(A) -> np.ndarray:
    """Lower band storage of real symmetric A: ab[d, j] = A[j + d, j], d = 0..w."""
    if np.iscomplexobj(A.val):
        raise ValueError("lower_band: real symmetric matrices only")
    w = bandwidth(A)
    ab = np.zeros((w + 1, A.n))
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    cols = A.col.astype(np.int64)
    low = rows >= cols
    ab[rows[low] - cols[low], cols[low]] = A.val[low]
    return ab


def eigenvalues_in_interval(A, a: float, b: float) -> np.ndarray:
    """All eigenvalues of real symmetric banded A in [a, b], ascending, with multiplicity."""
    if not a < b:
        raise ValueError("eigenvalues_in_interval: need a < b")
    ab = lower_band(A)
    w = scipy.linalg.eigvals_banded(ab, lower=True, select="v", select_range=(a, b))
    return np.sort(w)
