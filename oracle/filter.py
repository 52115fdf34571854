"""Applying the polynomial filter rho(l(A)) X (Section 2.2, Algorithm 2).

Test infrastructure only.

Algorithm 2 evaluates sum_j a_j T_j(l(A)) X by Clenshaw's backward recurrence.
As printed it seeds the recurrence with a_k X and divides by a_k; a_k can be
exactly zero (every odd c_j vanishes when l(a) = -l(b)), so this oracle uses the
division-free standard form, which is algebraically the same polynomial and
still costs k products with A:

    b_{k+1} = b_{k+2} = 0
    b_j     = a_j X + 2 l(A) b_{j+1} - b_{j+2},      j = k, ..., 1
    Y       = a_0 X + l(A) b_1 - b_2

with l(A) B = l1 (A B) + l2 B.  The forward three-term recurrence
T_{j+1} = 2 l(A) T_j - T_{j-1} is provided as an independent check.
"""
from __future__ import annotations

import numpy as np

from . import native


def _lmap(A, B, l1, l2):
    return l1 * native.spmm(A, B) + l2 * B


def clenshaw_filter(A, X: np.ndarray, coeffs: np.ndarray, l1: float, l2: float, degree: int | None = None) -> np.ndarray:
    """Y = sum_{j=0}^{degree} coeffs[j] T_j(l(A)) X by the backward recurrence."""
    k = len(coeffs) - 1 if degree is None else degree
    if k < 0:
        raise ValueError("degree must be >= 0")
    X = np.asarray(X)
    b1 = np.zeros_like(X)  # b_{j+1}
    b2 = np.zeros_like(X)  # b_{j+2}
    for j in range(k, 0, -1):
        bj = coeffs[j] * X + 2.0 * _lmap(A, b1, l1, l2) - b2
        b2, b1 = b1, bj
    return coeffs[0] * X + _lmap(A, b1, l1, l2) - b2


def forward_filter(A, X: np.ndarray, coeffs: np.ndarray, l1: float, l2: float, degree: int | None = None) -> np.ndarray:
    """Same polynomial by T_0 = X, T_1 = l(A) X, T_{j+1} = 2 l(A) T_j - T_{j-1}."""
    k = len(coeffs) - 1 if degree is None else degree
    X = np.asarray(X)
    T_prev = X
    Y = coeffs[0] * X
    if k == 0:
        return Y
    T_cur = _lmap(A, X, l1, l2)
    Y = Y + coeffs[1] * T_cur
    for j in range(2, k + 1):
        T_next = 2.0 * _lmap(A, T_cur, l1, l2) - T_prev
        Y = Y + coeffs[j] * T_next
        T_prev, T_cur = T_cur, T_next
    return Y


def clenshaw_steps(A, X, coeffs, l1, l2, degree=None):
    """Yield the Clenshaw state after each product with A (for step-level parity).

    Step s = 1..k yields the block produced by the s-th product: b_{k-s} for
    s < k and finally Y.  The first product acts on b_k = a_k X.
    """
    k = len(coeffs) - 1 if degree is None else degree
    X = np.asarray(X)
    b2 = np.zeros_like(X)
    b1 = coeffs[k] * X  # b_k (b_{k+1} = b_{k+2} = 0)
    for j in range(k - 1, 0, -1):
        bj = coeffs[j] * X + 2.0 * _lmap(A, b1, l1, l2) - b2
        b2, b1 = b1, bj
        yield bj
    yield coeffs[0] * X + _lmap(A, b1, l1, l2) - b2
