"""Sparse Hermitian test matrices in CSR form, built from a seed.

Every generator returns a :class:`CSR` whose rows have strictly increasing
column indices and no duplicate entries.  Values are float64 or complex128;
the HIP path converts to lower precision itself when asked.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    """Compressed sparse row matrix (square, n x n)."""

    n: int
    row_ptr: np.ndarray  # int64, n + 1
    col: np.ndarray      # int32, nnz
    val: np.ndarray      # float64 or complex128, nnz

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def is_complex(self) -> bool:
        return np.iscomplexobj(self.val)

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        out = np.zeros((self.n, self.n), dtype=self.val.dtype)
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        out[rows, self.col] = self.val
        return out


def _from_padded(cols: np.ndarray, vals: np.ndarray, valid: np.ndarray) -> CSR:
    """Compress an (n, w) table of candidate entries; columns must already be sorted per row."""
    n = cols.shape[0]
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(n, row_ptr, cols[valid].astype(np.int32), vals[valid])


def laplacian_2d_dirichlet(nx: int, ny: int | None = None) -> CSR:
    """5-point Laplacian on an nx x ny grid with Dirichlet boundary.

    Row index is ``ix * ny + iy``; diagonal 4, each in-grid neighbour -1.
    """
    ny = nx if ny is None else ny
    n = nx * ny
    idx = np.arange(n, dtype=np.int64)
    ix, iy = idx // ny, idx % ny
    offs = np.array([-ny, -1, 0, 1, ny], dtype=np.int64)
    cols = idx[:, None] + offs[None, :]
    valid = np.stack([ix > 0, iy > 0, np.ones(n, bool), iy < ny - 1, ix < nx - 1], axis=1)
    vals = np.where(offs[None, :] == 0, 4.0, -1.0) * np.ones((n, 1))
    return _from_padded(cols, vals, valid)


def laplacian_3d_dirichlet(N: int, potential_scale: float = 0.0, seed: int = 0) -> CSR:
    """7-point Laplacian on an N^3 Dirichlet grid plus a random diagonal potential.

    Row index is ``(ix * N + iy) * N + iz``.  Diagonal ``6 + potential_scale * U(0,1)``
    (the U(0,1) draws come from ``numpy.random.default_rng(seed)``), off-diagonal -1.
    ``potential_scale = 0`` gives the plain Laplacian with closed-form spectrum.
    """
    n = N ** 3
    idx = np.arange(n, dtype=np.int64)
    ix, iy, iz = idx // (N * N), (idx // N) % N, idx % N
    offs = np.array([-N * N, -N, -1, 0, 1, N, N * N], dtype=np.int64)
    cols = idx[:, None] + offs[None, :]
    valid = np.stack(
        [ix > 0, iy > 0, iz > 0, np.ones(n, bool), iz < N - 1, iy < N - 1, ix < N - 1], axis=1
    )
    diag = np.full(n, 6.0)
    if potential_scale != 0.0:
        rng = np.random.default_rng(seed)
        diag = diag + potential_scale * rng.uniform(0.0, 1.0, size=n)
    vals = np.empty((n, 7), dtype=np.float64)
    vals[:] = -1.0
    vals[:, 3] = diag
    return _from_padded(cols, vals, valid)


def tight_binding_3d_periodic(L: int, seed: int = 0) -> CSR:
    """Complex Hermitian nearest-neighbour hopping on a periodic L^3 lattice.

    Each bond from a site to its +x, +y, +z neighbour carries ``-exp(i theta)`` with
    ``theta ~ U(0, 2 pi)``; the reverse entry is the conjugate.  On-site energies are
    U(-1, 1).  Draw order from ``default_rng(seed)``: theta (n x 3), then on-site (n).
    Requires ``L >= 3`` so that the six neighbours of a site are distinct.
    """
    if L < 3:
        raise ValueError("periodic lattice needs L >= 3")
    n = L ** 3
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, 2.0 * np.pi, size=(n, 3))
    onsite = rng.uniform(-1.0, 1.0, size=n)
    idx = np.arange(n, dtype=np.int64)
    ix, iy, iz = idx // (L * L), (idx // L) % L, idx % L

    def site(x, y, z):
        return ((x % L) * L + (y % L)) * L + (z % L)

    plus = [site(ix + 1, iy, iz), site(ix, iy + 1, iz), site(ix, iy, iz + 1)]
    minus = [site(ix - 1, iy, iz), site(ix, iy - 1, iz), site(ix, iy, iz - 1)]
    cols = np.empty((n, 7), dtype=np.int64)
    vals = np.empty((n, 7), dtype=np.complex128)
    cols[:, 0] = idx
    vals[:, 0] = onsite
    for d in range(3):
        cols[:, 1 + d] = plus[d]
        vals[:, 1 + d] = -np.exp(1j * theta[:, d])
        cols[:, 4 + d] = minus[d]
        vals[:, 4 + d] = -np.exp(-1j * theta[minus[d], d])
    order = np.argsort(cols, axis=1, kind="stable")
    cols = np.take_along_axis(cols, order, axis=1)
    vals = np.take_along_axis(vals, order, axis=1)
    return _from_padded(cols, vals, np.ones((n, 7), dtype=bool))


def random_banded_symmetric(
    n: int,
    seed: int = 0,
    band: int = 64,
    per_row_band: int = 6,
    per_row_random: int = 6,
    diag_sigma: float = 2.0,
) -> CSR:
    """Irregular real symmetric matrix: half banded, half uniformly random columns.

    B has, per row i, ``per_row_band`` columns uniform in ``[i-band, i+band]`` (clipped to
    the matrix) and ``per_row_random`` columns uniform in ``[0, n)``, values N(0,1).
    A = B + B^T (coinciding entries summed) + diag(N(0, diag_sigma^2)).
    Draw order: band offsets, random columns, B values, diagonal.
    """
    import scipy.sparse as sp

    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n, dtype=np.int64), per_row_band + per_row_random)
    boff = rng.integers(-band, band + 1, size=(n, per_row_band))
    bcol = np.clip(np.arange(n)[:, None] + boff, 0, n - 1)
    rcol = rng.integers(0, n, size=(n, per_row_random))
    cols = np.concatenate([bcol, rcol], axis=1).reshape(-1)
    vals = rng.standard_normal(rows.size)
    diag = diag_sigma * rng.standard_normal(n)
    B = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A = (B + B.T + sp.diags(diag)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return CSR(n, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64))


def random_dense_symmetric_csr(n: int, density: float, seed: int = 0, complex_: bool = False) -> CSR:
    """Small random Hermitian matrix with roughly ``density`` fill, stored as CSR."""
    rng = np.random.default_rng(seed)
    mask = rng.uniform(size=(n, n)) < density
    mask = np.triu(mask, 1)
    M = rng.standard_normal((n, n))
    if complex_:
        M = M + 1j * rng.standard_normal((n, n))
    M = np.where(mask, M, 0)
    H = M + M.conj().T + np.diag(rng.standard_normal(n))
    rows, cols = np.nonzero(H)
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    val = H[rows, cols]
    return CSR(n, row_ptr, cols.astype(np.int32), val.astype(np.complex128 if complex_ else np.float64))


def gershgorin_bounds(A: CSR) -> tuple[float, float]:
    """Gershgorin enclosure [lo, hi] of the (real) spectrum of a Hermitian CSR matrix."""
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    is_diag = rows == A.col
    diag = np.bincount(rows[is_diag], weights=np.real(A.val[is_diag]), minlength=A.n)
    radius = np.bincount(rows[~is_diag], weights=np.abs(A.val[~is_diag]), minlength=A.n)
    return float(np.min(diag - radius)), float(np.max(diag + radius))
