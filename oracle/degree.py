"""Degree selection for the adaptive filter (Section 3.1, Algorithm 3, eq. (compute_k_1)).

Test infrastructure only.

select_degree restates Algorithm 3: with t = l(lambda_hat) for the current Ritz
values, grow the truncated series gamma = sum_{i<=j} a_i T_i(t) one term at a
time (T_j by the three-term recurrence on the scalars t), order |gamma| from
large to small, and return the first j for which |gamma_p| / |gamma_e| < tau_a,
where p is the number of Ritz values and e the number inside [a, b].

Readings where the algorithm is silent: p and e are the counts of the current
iteration (after locking); if no j up to k meets the test the maximum degree k
is returned; e = 0 never reaches this function (Algorithm 4 skips the
iteration); a zero |gamma_e| counts as "not met".
"""
from __future__ import annotations

import numpy as np


def select_degree(ritz: np.ndarray, e: int, coeffs: np.ndarray, l1: float, l2: float, tau_a: float) -> int:
    ritz = np.asarray(ritz, dtype=np.float64)
    p = ritz.size
    k = len(coeffs) - 1
    if e <= 0 or e > p:
        raise ValueError("need 1 <= e <= p")
    t = l1 * ritz + l2
    h0 = np.ones_like(t)
    h1 = t.copy()
    gamma = coeffs[0] * h0
    for j in range(1, k + 1):
        gamma = gamma + coeffs[j] * h1
        mags = np.sort(np.abs(gamma))[::-1]
        g_p, g_e = mags[p - 1], mags[e - 1]
        if g_e != 0.0 and g_p / g_e < tau_a:
            return j
        h0, h1 = h1, 2.0 * t * h1 - h0
    return k
