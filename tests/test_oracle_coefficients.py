"""Pins for the oracle's filter construction (Section 2.2, Section 3.2).

Each check compares the oracle against something it does not compute itself:
quadrature of the step function, closed-form special cases, numpy's Chebyshev
evaluation, and the paper's error bounds (Lemma 3.1, Theorems 3.2 and 3.3).
"""
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

from oracle import coefficients as co
from oracle import theory as th


INTERVALS = [  # (a, b) inside the normalised frame [-1, 1]
    (0.1, 0.6),        # the example of Section 3.2 (Fig. 1)
    (-0.3, 0.3),       # symmetric about the centre
    (-0.999, -0.8),    # near the lower end
    (0.01, 0.011),     # narrow
    (-1.0, 0.2),       # touching the end (extreme problem)
]


def _quadrature_coeffs(alpha, beta, k, nodes=400000):
    """(2/pi) int_0^pi g(theta) cos(j theta) dtheta by the midpoint rule (1/pi for j = 0)."""
    h = math.pi / nodes
    t = (np.arange(nodes) + 0.5) * h
    g = ((t > beta) & (t < alpha)).astype(np.float64)
    out = np.empty(k + 1)
    for j in range(k + 1):
        out[j] = (1.0 if j == 0 else 2.0) / math.pi * h * np.dot(g, np.cos(j * t))
    return out


@pytest.mark.parametrize("a,b", INTERVALS)
def test_cj_matches_quadrature_of_step(a, b):
    alpha, beta = co.interval_angles(a, b, -1.0, 1.0)
    c = co.step_coefficients(alpha, beta, 40)
    q = _quadrature_coeffs(alpha, beta, 40)
    assert np.max(np.abs(c - q)) < 2e-5


def test_symmetric_interval_has_zero_odd_coefficients():
    # l(a) = -l(b)  =>  alpha = pi - beta  =>  every odd c_j is zero
    lmin, lmax = -7.0, 7.0
    c = co.filter_coefficients(lmin, lmax, -0.25, 0.25, 151, "jackson")
    assert np.max(np.abs(c[1::2])) < 1e-15
    assert np.min(np.abs(c[0::2][:10])) > 0


def test_full_interval_gives_constant_one():
    c = co.filter_coefficients(2.0, 5.0, 2.0, 5.0, 30, "none")
    assert abs(c[0] - 1.0) < 1e-15 and np.max(np.abs(c[1:])) < 1e-15


def test_affine_map_endpoints():
    l1, l2 = co.affine_map(-3.0, 5.0)
    assert l1 * -3.0 + l2 == -1.0 and l1 * 5.0 + l2 == 1.0
    # interval reaching past the bounds is clipped (extreme eigenproblem)
    alpha, beta = co.interval_angles(-10.0, 1.0, -3.0, 5.0)
    assert alpha == math.pi


def test_jackson_closed_form_values():
    for k in (1, 5, 60, 200):
        d = co.jackson_damping(k)
        assert abs(d[0] - 1.0) < 1e-15
        # first Jackson factor is cos(pi / (k + 2))
        assert abs(d[1] - math.cos(math.pi / (k + 2))) < 1e-14
        assert np.all(np.diff(d) < 0) and np.all(d > 0) and np.all(d <= 1)
        # the formula vanishes at j = k + 1
        q = math.pi / (k + 2)
        j = k + 1
        num = (k + 2 - j) * math.sin(q) * math.cos(j * q) + math.cos(q) * math.sin(j * q)
        assert abs(num) < 1e-14


@pytest.mark.parametrize("a,b", INTERVALS[:4])
@pytest.mark.parametrize("k", [10, 60, 150])
def test_jackson_filter_stays_in_unit_interval(a, b, k):
    # the Jackson kernel is non-negative, so its smoothing of a 0/1 step lies in [0, 1]
    c = co.filter_coefficients(-1.0, 1.0, a, b, k, "jackson")
    x = np.cos(np.linspace(0.0, math.pi, 20001))
    r = co.filter_value(x, c, -1.0, 1.0)
    assert r.min() > -1e-13 and r.max() < 1 + 1e-13


def test_lanczos_damping_special_cases():
    k = 40
    assert np.all(co.lanczos_damping(k, 0.0) == 1.0)
    j = np.arange(1, k + 1)
    sinc = np.sin(j * np.pi / (k + 1)) / (j * np.pi / (k + 1))
    assert np.allclose(co.lanczos_damping(k, 1.0)[1:], sinc, rtol=0, atol=1e-15)
    assert np.allclose(co.lanczos_damping(k, 2.0), co.lanczos_damping(k, 1.0) ** 2, rtol=1e-14)
    d = co.lanczos_damping(k, 0.5)
    assert d[0] == 1.0 and np.all(np.diff(d) < 0) and np.all(d > 0)


def test_filter_value_matches_numpy_chebval():
    lmin, lmax = -2.0, 6.0
    c = co.filter_coefficients(lmin, lmax, 1.0, 1.7, 50, "lanczos", 0.5)
    x = np.linspace(lmin, lmax, 777)
    l1, l2 = co.affine_map(lmin, lmax)
    ref = npcheb.chebval(l1 * x + l2, c)
    assert np.max(np.abs(co.filter_value(x, c, lmin, lmax) - ref)) < 1e-12
    # outside the bounds T_j grows like cosh
    xo = np.array([lmin - 0.3, lmax + 0.2])
    ref_o = npcheb.chebval(l1 * xo + l2, c)
    assert np.allclose(co.filter_value(xo, c, lmin, lmax), ref_o, rtol=1e-10)


def test_initial_degree_rule():
    # eq. (compute_k_1) with C = 1.4
    assert co.initial_degree(0.5, 0.4, 1.4) == math.ceil(14.0) - 1 or co.initial_degree(0.5, 0.4, 1.4) == 14
    assert co.initial_degree(1.0, 0.0, 1.4) == 1
    alpha, beta = co.interval_angles(0.128538339316, 0.255551112680, 0.0, 8.0)
    assert co.initial_degree(alpha, beta, 1.4) == math.ceil(1.4 / (alpha - beta)) - 1


# ---------------------------------------------------------------- bounds (Section 3.2)

def test_lemma_3_1_tail_bound():
    x = np.linspace(1e-3, math.pi, 3000)
    for k in (1, 3, 10, 50, 200):
        R = th.partial_tail(x, k)
        assert np.all(np.abs(R) <= 1.0 / ((k + 1) * np.sin(x / 2)) + 1e-12)


def test_remark_J_le_4pi_over_distance():
    alpha, beta = co.interval_angles(0.1, 0.6, -1, 1)
    t = np.linspace(0, math.pi, 5001)
    t = t[(t != alpha) & (t != beta)]
    d = np.min(np.abs(np.stack([t - alpha, t + alpha, t - beta, t + beta])), axis=0)
    assert np.all(th.J_theta(t, alpha, beta) <= 4 * math.pi / d * (1 + 1e-12))


def _grid(alpha, beta):
    t = np.linspace(0.0, math.pi, 4001)
    return np.concatenate([t, [alpha, beta]])


@pytest.mark.parametrize("a,b", INTERVALS[:4])
@pytest.mark.parametrize("k", [1, 4, 20, 100, 400])
def test_theorem_3_2_undamped_bound(a, b, k):
    alpha, beta = co.interval_angles(a, b, -1.0, 1.0)
    c = co.step_coefficients(alpha, beta, k)
    t = _grid(alpha, beta)
    gk = np.cos(np.multiply.outer(t, np.arange(k + 1))) @ c
    err = np.abs(th.step_in_theta(t, alpha, beta) - gk)
    bound = th.undamped_bound(t, alpha, beta, k)
    assert np.all(err <= bound * (1 + 1e-10) + 1e-13)
    # the bound is not vacuous: it tracks the error within two orders of magnitude somewhere
    fin = np.isfinite(bound)
    if k >= 20:
        assert np.max(err[fin] / bound[fin]) > 1e-2


@pytest.mark.parametrize("m", [0.5, 1.0, 2.0, 3.0])
@pytest.mark.parametrize("a,b", INTERVALS[:4])
def test_theorem_3_3_damped_bound(m, a, b):
    alpha, beta = co.interval_angles(a, b, -1.0, 1.0)
    Cm = th.C_m(m)
    t = _grid(alpha, beta)
    for ki, k in [(1, 3), (5, 13), (20, 50), (40, 100), (100, 100), (200, 500)]:
        c = co.step_coefficients(alpha, beta, k)[: ki + 1]
        d = co.lanczos_damping(k, m)[: ki + 1]
        g = np.cos(np.multiply.outer(t, np.arange(ki + 1))) @ (c * d)
        err = np.abs(th.step_in_theta(t, alpha, beta) - g)
        bound = th.damped_bound(t, alpha, beta, ki, k, m, Cm)
        assert np.all(err <= bound * (1 + 1e-10) + 1e-13), (ki, k)


def test_fig1_example_bound_holds():
    # Section 3.2 example: a = 0.1, b = 0.6, m = 0.5, k = 2.5 k^(i); x = 0.3 and k = 100 sweeps
    alpha, beta = co.interval_angles(0.1, 0.6, -1.0, 1.0)
    Cm = th.C_m(0.5)
    theta = math.acos(0.3)
    for ki in range(1, 201):
        k = math.ceil(2.5 * ki)
        c = co.step_coefficients(alpha, beta, k)[: ki + 1] * co.lanczos_damping(k, 0.5)[: ki + 1]
        g = float(np.dot(c, np.cos(theta * np.arange(ki + 1))))
        assert abs(1.0 - g) <= th.damped_bound(theta, alpha, beta, ki, k, 0.5, Cm) + 1e-13
    x = np.linspace(-0.1, 0.3, 401)
    t = np.arccos(x)
    k, ki = 100, 40
    c = co.step_coefficients(alpha, beta, k)[: ki + 1] * co.lanczos_damping(k, 0.5)[: ki + 1]
    g = np.cos(np.multiply.outer(t, np.arange(ki + 1))) @ c
    err = np.abs(th.step_in_theta(t, alpha, beta) - g)
    assert np.all(err <= th.damped_bound(t, alpha, beta, ki, k, 0.5, Cm) + 1e-13)


@pytest.mark.parametrize("m", [0.5, 1.0, 2.0])
def test_C_m_against_scipy_quad(m):
    from scipy.integrate import quad

    f = lambda u: np.sin(u) ** (m - 1) * (np.sin(u) - u * np.cos(u)) / u ** (m + 2)
    ref, _ = quad(f, 1e-12, math.pi, limit=500, epsabs=1e-13)
    assert abs(th.C_m(m) - ref) < 1e-9
