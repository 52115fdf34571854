"""Closed-form spectra of Dirichlet grid Laplacians (definition-level results).

Test infrastructure only.  The 1D Dirichlet second-difference matrix of order N
(diagonal 2, off-diagonals -1) has eigenvalues 2 - 2 cos(j pi / (N+1)) and
eigenvectors sin(j pi x / (N+1)), x = 1..N; the 2D and 3D Laplacians are Kronecker
sums, so their eigenpairs are sums and tensor products of these.  Row ordering
matches workloads.matrices (ix slowest).
"""
from __future__ import annotations

import numpy as np


def lap1d_eigs(N: int) -> np.ndarray:
    j = np.arange(1, N + 1)
    return 2.0 - 2.0 * np.cos(j * np.pi / (N + 1))


def lap2d_eigs(nx: int, ny: int | None = None) -> np.ndarray:
    ny = nx if ny is None else ny
    return np.sort(np.add.outer(lap1d_eigs(nx), lap1d_eigs(ny)).ravel())


def lap3d_eigs(N: int) -> np.ndarray:
    e = lap1d_eigs(N)
    return np.sort((e[:, None, None] + e[None, :, None] + e[None, None, :]).ravel())


def _mode(N: int, j: int) -> np.ndarray:
    x = np.arange(1, N + 1)
    v = np.sin(j * np.pi * x / (N + 1))
    return v / np.linalg.norm(v)


def lap2d_mode(nx: int, ny: int, i: int, j: int):
    """(eigenvalue, unit eigenvector) for mode (i, j), 1-based."""
    lam = lap1d_eigs(nx)[i - 1] + lap1d_eigs(ny)[j - 1]
    return lam, np.kron(_mode(nx, i), _mode(ny, j))


def lap3d_mode(N: int, i: int, j: int, k: int):
    lam = lap1d_eigs(N)[i - 1] + lap1d_eigs(N)[j - 1] + lap1d_eigs(N)[k - 1]
    return lam, np.kron(np.kron(_mode(N, i), _mode(N, j)), _mode(N, k))
