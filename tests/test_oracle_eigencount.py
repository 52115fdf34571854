"""Pins of the eigenvalue-count oracle (trace estimation of the filter, Section 3.4).

* Over the complete set of sign vectors E[z z^H] = I holds exactly, so the averaged
  quadratic forms equal tr rho(A) = sum_j rho(lambda_j), computed from eigvalsh and the
  trigonometric form of the filter (no recurrence); real and complex probes.
* Unit-vector probes give the diagonal of V diag(rho(lambda)) V^H from eigh.
* Config 1 (64 x 64 Laplacian): the trace from the closed-form eigenvalues is within one
  of the true count 40, and 256 random probes estimate it within 5 standard errors.
* With damping and a degree far above the gap resolution the trace approaches the
  number of eigenvalues in [a, b] (the filter approaches the interval indicator).
"""
import itertools

import numpy as np
import pytest

from oracle import eigencount as ec
from workloads import build_config, probe_block
from workloads.matrices import CSR

from tests.golden_util import lap2d_window


def _small(n, cplx, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n)) + (1j * rng.standard_normal((n, n)) if cplx else 0)
    H = (M + M.conj().T) / 2
    rows, cols = np.nonzero(np.ones((n, n)))
    rp = np.arange(0, n * n + 1, n, dtype=np.int64)
    return CSR(n, rp, cols.astype(np.int32), H[rows, cols]), H


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("damping", ["jackson", "lanczos", "none"])
def test_complete_sign_set_average_is_the_trace(cplx, damping):
    n = 5
    A, H = _small(n, cplx, seed=11)
    w = np.linalg.eigvalsh(H)
    lmin, lmax = w[0] - 0.3, w[-1] + 0.2
    a, b = w[1] - 0.05, w[3] + 0.05
    signs = np.array(list(itertools.product([-1.0, 1.0], repeat=n))).T  # n x 2^n
    if cplx:
        Z = np.array([(s + 1j * t) / np.sqrt(2.0) for s in signs.T for t in signs.T]).T  # n x 4^n
    else:
        Z = signs
    est = ec.estimate_eigencount(A, Z, lmin, lmax, a, b, 40, damping)
    tr = ec.filter_trace(w, lmin, lmax, a, b, 40, damping)
    assert abs(est - tr) < 1e-12 * max(1.0, abs(tr))


@pytest.mark.parametrize("cplx", [False, True])
def test_unit_probes_give_the_projector_diagonal(cplx):
    n = 40
    A, H = _small(n, cplx, seed=4)
    w, V = np.linalg.eigh(H)
    lmin, lmax = w[0] - 0.1, w[-1] + 0.1
    a, b = 0.5 * (w[10] + w[11]), 0.5 * (w[25] + w[26])
    q = ec.probe_quadratic_forms(A, np.eye(n, dtype=H.dtype), lmin, lmax, a, b, 80, "lanczos")
    from oracle.coefficients import filter_coefficients, filter_value

    rho = filter_value(w, filter_coefficients(lmin, lmax, a, b, 80, "lanczos"), lmin, lmax)
    diag = np.real(np.sum((np.abs(V) ** 2) * rho[None, :], axis=1))
    assert np.max(np.abs(q - diag)) < 1e-12


def test_config1_closed_form_trace_and_estimate():
    A, (lmin, lmax), (a, b), cfg = build_config("lap2d_64")
    N = 64
    ii, jj = np.meshgrid(np.arange(1, N + 1), np.arange(1, N + 1))
    lam = (4 - 2 * np.cos(ii * np.pi / (N + 1)) - 2 * np.cos(jj * np.pi / (N + 1))).ravel()
    inside = np.sort(lam[(lam >= a) & (lam <= b)])
    assert np.allclose(inside, lap2d_window(), atol=1e-14, rtol=0)
    tr = ec.filter_trace(lam, lmin, lmax, a, b, cfg.degree, "jackson")
    assert abs(tr - 40) < 1.0
    q = ec.probe_quadratic_forms(A, probe_block(A.n, 256, seed=3), lmin, lmax, a, b, cfg.degree, "jackson")
    se = q.std(ddof=1) / np.sqrt(q.size)
    assert abs(q.mean() - tr) < 5 * se
    assert ec.block_size(q.mean()) == int(np.ceil(1.8 * q.mean()))


def test_high_degree_trace_approaches_the_count():
    rng = np.random.default_rng(2)
    lam = np.sort(rng.uniform(-1.0, 1.0, 300))
    lam = lam[(np.abs(lam - (-0.2)) > 0.02) & (np.abs(lam - 0.3) > 0.02)]  # gaps at the ends
    count = int(np.sum((lam >= -0.2) & (lam <= 0.3)))
    tr = ec.filter_trace(lam, -1.0, 1.0, -0.2, 0.3, 3000, "jackson")
    assert abs(tr - count) < 1e-3
