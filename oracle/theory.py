"""Pointwise error bounds of the filter (Section 3.2).

Test infrastructure only.  Used as pins: the oracle's coefficients and damping
must satisfy these inequalities on every theta grid, so a dropped term, a sign
error or an index shift in eq. (c_j) or in the damping fails them.

* Lemma 3.1: |R_k(x)| <= 1 / ((k+1) sin(x/2)) for the tail of sum sin(jx)/j.
* Theorem 3.2 / eq. (J_theta): |g - g_k| <= J(theta) / (pi (k+1)).
* Remark after Theorem 3.2: J(theta) <= 4 pi / d(theta).
* Theorem 3.3 / eq. (C_m): the damped bound with three terms.
"""
from __future__ import annotations

import math

import numpy as np


def J_theta(theta, alpha: float, beta: float):
    """J(theta) of eq. (J_theta), including the special values at theta = alpha, beta."""
    theta = np.asarray(theta, dtype=np.float64)
    s = np.abs
    with np.errstate(divide="ignore"):
        gen = (
            1.0 / s(np.sin((theta + alpha) / 2))
            + 1.0 / s(np.sin((theta - alpha) / 2))
            + 1.0 / s(np.sin((theta + beta) / 2))
            + 1.0 / s(np.sin((theta - beta) / 2))
        )
    common = 1.0 / abs(math.sin((alpha + beta) / 2)) + 1.0 / abs(math.sin((alpha - beta) / 2))
    at_alpha = 1.0 / abs(math.sin(alpha)) + common if math.sin(alpha) != 0 else np.inf
    at_beta = 1.0 / abs(math.sin(beta)) + common if math.sin(beta) != 0 else np.inf
    out = np.where(theta == alpha, at_alpha, np.where(theta == beta, at_beta, gen))
    return out


def C_m(m: float, panels: int = 200, order: int = 20) -> float:
    """C_m of eq. (C_m) by composite Gauss-Legendre quadrature.

    Near u = 0 the integrand tends to 1/3 for every m (sin u - u cos u ~ u^3/3);
    near u = pi the factor (sin u)^(m-1) is singular when m < 1, so the
    substitution u = pi (1 - w^2), du = -2 pi w dw, is used to remove it.
    """
    xg, wg = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(0.0, 1.0, panels + 1)
    total = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        w = 0.5 * (hi - lo) * xg + 0.5 * (hi + lo)
        u = math.pi * (1.0 - w * w)
        f = np.sin(u) ** (m - 1.0) * (np.sin(u) - u * np.cos(u)) / u ** (m + 2.0)
        total += 0.5 * (hi - lo) * np.dot(wg, f * 2.0 * math.pi * w)
    return float(total)


def partial_tail(x, k: int, terms: int = 200000):
    """R_k(x) = (pi - x)/2 - sum_{j<=k} sin(jx)/j on (0, 2 pi) (Lemma 3.1)."""
    x = np.asarray(x, dtype=np.float64)
    j = np.arange(1, k + 1)
    S = np.sin(np.multiply.outer(x, j)) @ (1.0 / j)
    return (math.pi - x) / 2.0 - S


def undamped_bound(theta, alpha, beta, k):
    """Right-hand side of eq. (gk_bound)."""
    return J_theta(theta, alpha, beta) / (math.pi * (k + 1))


def damped_bound(theta, alpha, beta, ki, k, m, Cm=None):
    """Right-hand side of eq. (eq:damped_fourier_error_bound) for 1 <= ki <= k, m > 0."""
    theta = np.asarray(theta, dtype=np.float64)
    if Cm is None:
        Cm = C_m(m)
    t = ki * math.pi / (k + 1)
    d_ki = (math.sin(t) / t) ** m
    J = J_theta(theta, alpha, beta)
    return d_ki * J / (math.pi * (ki + 1)) + m * Cm * J / (k + 1) + m * math.pi * (math.pi - theta) / (3 * (k + 1) ** 2)


def step_in_theta(theta, alpha, beta):
    """g(theta): 1 on (beta, alpha), 1/2 at the ends, 0 elsewhere on [0, pi] (Section 3.2)."""
    theta = np.asarray(theta, dtype=np.float64)
    return np.where((theta > beta) & (theta < alpha), 1.0, np.where((theta == alpha) | (theta == beta), 0.5, 0.0))
