"""Polynomial filter construction (Section 2.2 and Section 3.1).

Test infrastructure only (see the package docstring).

* the affine map l(x) = l1 x + l2 taking [lambda_min, lambda_max] onto [-1, 1]
  (Section 2.2, the linear transformation after eq. (c_j));
* the Chebyshev coefficients c_j of the step function s(x) of eq. (step_func),
  given in closed form by eq. (c_j);
* damping factors: Jackson d^J_{j,k}, Lanczos sigma factors d^L_{j,k}, and the
  exponent-m Lanczos factors d^m_{j,k} of eq. (m_Lanczos_damping);
* the filter coefficients a_j = c_j d_{j,k} used by eq. (AdaPolySI), where the
  damping is always evaluated at the maximum degree k even when the series is
  truncated at k^(i) <= k.
"""
from __future__ import annotations

import math

import numpy as np


def affine_map(lmin: float, lmax: float) -> tuple[float, float]:
    """Return (l1, l2) with l(x) = (2x - lmax - lmin) / (lmax - lmin) = l1 x + l2."""
    if not lmax > lmin:
        raise ValueError("need lmax > lmin")
    width = lmax - lmin
    return 2.0 / width, -(lmax + lmin) / width


def interval_angles(a: float, b: float, lmin: float, lmax: float) -> tuple[float, float]:
    """alpha = arccos l(a), beta = arccos l(b) with l(.) clipped into [-1, 1].

    eq. (c_j) is written for the normalised frame [lambda_min, lambda_max] = [-1, 1];
    the general case maps a and b by l first.  An interval reaching past the
    spectral bounds (the extreme case of Section 1) is clipped to them.
    """
    if not b > a:
        raise ValueError("need b > a")
    affine_map(lmin, lmax)  # validates the bounds
    width = lmax - lmin
    # the quotient form of l(x) maps lmin and lmax to exactly -1 and 1
    xa = min(1.0, max(-1.0, (2.0 * a - lmax - lmin) / width))
    xb = min(1.0, max(-1.0, (2.0 * b - lmax - lmin) / width))
    return math.acos(xa), math.acos(xb)


def step_coefficients(alpha: float, beta: float, k: int) -> np.ndarray:
    """c_0..c_k of eq. (c_j): Chebyshev series of the interval indicator."""
    c = np.empty(k + 1)
    c[0] = (alpha - beta) / math.pi
    for j in range(1, k + 1):
        c[j] = 2.0 / math.pi * (math.sin(j * alpha) - math.sin(j * beta)) / j
    return c


def jackson_damping(k: int) -> np.ndarray:
    """Jackson factors d^J_{j,k}, j = 0..k (Section 2.2).

    The printed formula is stated for j > 0; at j = 0 it evaluates to exactly 1,
    which is the value used for the constant term.
    """
    q = math.pi / (k + 2)
    d = np.empty(k + 1)
    for j in range(k + 1):
        num = (k + 2 - j) * math.sin(q) * math.cos(j * q) + math.cos(q) * math.sin(j * q)
        d[j] = num / ((k + 2) * math.sin(q))
    return d


def lanczos_damping(k: int, m: float = 1.0) -> np.ndarray:
    """Exponent-m Lanczos factors of eq. (m_Lanczos_damping), j = 0..k.

    m = 1 gives the Lanczos sigma factors d^L; m = 0 gives no damping.  At j = 0
    the sinc quotient is 0/0 and its limit 1 is used.
    """
    if m < 0:
        raise ValueError("exponent m must be >= 0")
    d = np.empty(k + 1)
    d[0] = 1.0
    for j in range(1, k + 1):
        t = j * math.pi / (k + 1)
        d[j] = (math.sin(t) / t) ** m
    return d


def damping_factors(kind: str, k: int, m_exp: float = 0.5) -> np.ndarray:
    if kind == "none":
        return np.ones(k + 1)
    if kind == "jackson":
        return jackson_damping(k)
    if kind == "lanczos":
        return lanczos_damping(k, m_exp)
    raise ValueError(f"unknown damping {kind!r}")


def filter_coefficients(
    lmin: float, lmax: float, a: float, b: float, kmax: int, damping: str = "jackson", m_exp: float = 0.5
) -> np.ndarray:
    """a_j = c_j d_{j,kmax}, j = 0..kmax (eq. (AdaPolySI) with the damping at the max degree)."""
    alpha, beta = interval_angles(a, b, lmin, lmax)
    return step_coefficients(alpha, beta, kmax) * damping_factors(damping, kmax, m_exp)


def filter_value(x, coeffs: np.ndarray, lmin: float, lmax: float, degree: int | None = None):
    """rho(x) = sum_{j<=degree} a_j T_j(l(x)), evaluated in trigonometric form.

    Uses T_j(t) = cos(j arccos t) on |t| <= 1 (Section 3.2) and cosh(j arccosh |t|)
    with the sign (+-1)^j outside; independent of any recurrence.
    """
    degree = len(coeffs) - 1 if degree is None else degree
    l1, l2 = affine_map(lmin, lmax)
    t = l1 * np.asarray(x, dtype=np.float64) + l2
    out = np.zeros_like(t)
    inside = np.abs(t) <= 1.0
    th = np.arccos(np.clip(t, -1.0, 1.0))
    ch = np.arccosh(np.maximum(np.abs(t), 1.0))
    sgn = np.sign(t)
    for j in range(degree + 1):
        tj = np.where(inside, np.cos(j * th), (sgn ** j) * np.cosh(j * ch))
        out = out + coeffs[j] * tj
    return out


def initial_degree(alpha: float, beta: float, C: float = 1.4) -> int:
    """k^(1) = ceil(C / (alpha - beta)) - 1, eq. (compute_k_1)."""
    return int(math.ceil(C / (alpha - beta))) - 1
