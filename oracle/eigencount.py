"""Eigenvalue count in [a, b] by stochastic trace estimation (Section 3.4).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The damped step-function filter of eq. (AdaPolySI), taken at its full degree, is an
approximate spectral projector onto [a, b]; the number of eigenvalues in [a, b] is
estimated by its trace, and the trace by Hutchinson's estimator over probe vectors
z_i with E[z z^H] = I: tr rho(A) ~ (1/m) sum_i z_i^H rho(A) z_i.  The block size is
then p = ceil(mu * estimate) (mu = 1.8 in the paper's experiments, Section 4).
"""
from __future__ import annotations

import math

import numpy as np

from .coefficients import affine_map, filter_coefficients, filter_value
from .filter import clenshaw_filter


def probe_quadratic_forms(A, Z: np.ndarray, lmin: float, lmax: float, a: float, b: float,
                          degree: int, damping: str = "lanczos", m_exp: float = 0.5) -> np.ndarray:
    """Re z_i^H rho(A) z_i for every column z_i of Z."""
    c = filter_coefficients(lmin, lmax, a, b, degree, damping, m_exp)
    l1, l2 = affine_map(lmin, lmax)
    Y = clenshaw_filter(A, Z, c, l1, l2)
    return np.real(np.sum(np.conj(Z) * Y, axis=0))


def estimate_eigencount(A, Z: np.ndarray, lmin: float, lmax: float, a: float, b: float,
                        degree: int, damping: str = "lanczos", m_exp: float = 0.5) -> float:
    """Hutchinson estimate of tr rho(A): the mean of the probe quadratic forms."""
    return float(np.mean(probe_quadratic_forms(A, Z, lmin, lmax, a, b, degree, damping, m_exp)))


def filter_trace(eigenvalues: np.ndarray, lmin: float, lmax: float, a: float, b: float,
                 degree: int, damping: str = "lanczos", m_exp: float = 0.5) -> float:
    """tr rho(A) = sum_j rho(lambda_j) from the eigenvalues (definition level; rho in
    trigonometric form, no recurrence)."""
    c = filter_coefficients(lmin, lmax, a, b, degree, damping, m_exp)
    return float(np.sum(filter_value(np.asarray(eigenvalues, dtype=np.float64), c, lmin, lmax)))


def block_size(estimate: float, mu: float = 1.8) -> int:
    """p = ceil(mu * estimate) (Section 3.4)."""
    return int(math.ceil(mu * estimate))
