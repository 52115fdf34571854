"""Dense steps of the filtered subspace iteration (Algorithm 1 and Algorithm 4).

Test infrastructure only.

* orthonormalize: Q = orth([V_locked, X]) restricted to the columns that belong
  to X (Algorithm 4, orthogonalisation step), i.e. X made orthogonal to the
  locked vectors and then orthonormalised.  The oracle projects the locked
  vectors out twice and uses Householder QR (numpy.linalg.qr) -- deliberately a
  different algorithm from the Cholesky-QR the GPU path uses.
* rayleigh_ritz: B = Q^* A Q, B = U Lambda U^*, V = Q U (Algorithm 1, the
  Rayleigh-Ritz function).  A Q is also returned multiplied by U so that
  residuals A v - lambda v can be formed without another product with A.
* residual_norms: ||A v_j - lambda_j v_j||_2 per column (Algorithm 4, residual
  step; the norm of Section 4).
"""
from __future__ import annotations

import numpy as np

from . import native


def project_out(X: np.ndarray, V: np.ndarray | None) -> np.ndarray:
    if V is None or V.shape[1] == 0:
        return X
    for _ in range(2):
        X = X - V @ (V.conj().T @ X)
    return X


def orthonormalize(X: np.ndarray, V_locked: np.ndarray | None = None) -> np.ndarray:
    X = project_out(np.asarray(X), V_locked)
    Q, _ = np.linalg.qr(X, mode="reduced")
    return Q


def rayleigh_ritz(A, Q: np.ndarray):
    """Return (ritz values ascending, V = Q U, AV = (A Q) U)."""
    AQ = native.spmm(A, Q)
    B = Q.conj().T @ AQ
    B = 0.5 * (B + B.conj().T)
    w, U = np.linalg.eigh(B)
    return w, Q @ U, AQ @ U


def residual_norms(V: np.ndarray, AV: np.ndarray, w: np.ndarray) -> np.ndarray:
    return np.linalg.norm(AV - V * w[None, :], axis=0)
