"""Pins for the oracle's filter application (Algorithm 2) and its CSR product."""
import numpy as np
import pytest

from oracle import closed_form, native
from oracle import coefficients as co
from oracle.filter import clenshaw_filter, clenshaw_steps, forward_filter
from workloads import (
    build_config,
    laplacian_2d_dirichlet,
    random_dense_symmetric_csr,
    start_block,
    tight_binding_3d_periodic,
)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("cplx", [False, True])
def test_spmm_matches_scipy(cplx):
    A = random_dense_symmetric_csr(300, 0.05, seed=3, complex_=cplx)
    # make a few empty rows
    A.val[A.row_ptr[5]:A.row_ptr[6]] = 0
    B = start_block(300, 7, seed=1, complex_=cplx)
    ref = A.to_scipy() @ B
    assert np.max(np.abs(native.spmm(A, B) - ref)) < 1e-12


def test_spmm_tight_binding_is_hermitian():
    A = tight_binding_3d_periodic(5, seed=2)
    D = A.to_dense()
    assert np.max(np.abs(D - D.conj().T)) == 0.0
    assert A.nnz == 7 * 125


@pytest.mark.parametrize("cplx", [False, True])
def test_clenshaw_equals_forward_recurrence(cplx):
    A = random_dense_symmetric_csr(400, 0.03, seed=5, complex_=cplx)
    D = A.to_dense()
    w = np.linalg.eigvalsh(D)
    lmin, lmax = w[0] - 0.01, w[-1] + 0.01
    c = co.filter_coefficients(lmin, lmax, 0.2 * lmin + 0.8 * 0.0, 0.3 * lmax, 80, "lanczos", 0.5)
    l1, l2 = co.affine_map(lmin, lmax)
    X = start_block(400, 9, seed=4, complex_=cplx)
    Y1 = clenshaw_filter(A, X, c, l1, l2)
    Y2 = forward_filter(A, X, c, l1, l2)
    assert _rel(Y1, Y2) < 1e-12


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("damping", ["jackson", "lanczos", "none"])
def test_clenshaw_equals_spectral_definition(cplx, damping):
    # rho(A) X = V diag(rho(lambda)) V^* X, with rho evaluated in trigonometric form
    n = 250
    A = random_dense_symmetric_csr(n, 0.05, seed=11, complex_=cplx)
    w, V = np.linalg.eigh(A.to_dense())
    lmin, lmax = w[0] - 0.05, w[-1] + 0.05
    a, b = w[100] - 1e-3, w[130] + 1e-3
    c = co.filter_coefficients(lmin, lmax, a, b, 120, damping, 0.5)
    l1, l2 = co.affine_map(lmin, lmax)
    X = start_block(n, 6, seed=12, complex_=cplx)
    ref = V @ (co.filter_value(w, c, lmin, lmax)[:, None] * (V.conj().T @ X))
    assert _rel(clenshaw_filter(A, X, c, l1, l2), ref) < 1e-11


def test_clenshaw_on_laplacian_eigenvectors():
    # Config-1 matrix: the closed-form eigenvectors are mapped to rho(lambda) v
    A, (lmin, lmax), (a, b), cfg = build_config("lap2d_64")
    c = co.filter_coefficients(lmin, lmax, a, b, cfg.degree, "jackson")
    l1, l2 = co.affine_map(lmin, lmax)
    modes = [(1, 1), (3, 5), (5, 6), (2, 7), (30, 30), (64, 64), (10, 1)]
    lams, vecs = zip(*(closed_form.lap2d_mode(64, 64, i, j) for i, j in modes))
    X = np.stack(vecs, axis=1)
    Y = clenshaw_filter(A, X, c, l1, l2)
    expect = X * co.filter_value(np.array(lams), c, lmin, lmax)[None, :]
    assert np.max(np.abs(Y - expect)) < 1e-13
    # filtered values: in-window modes near 1/2..1, far modes ~0
    assert np.all(co.filter_value(np.array(lams), c, lmin, lmax) <= 1.0 + 1e-14)


def test_degree_zero_one_and_step_generator():
    A = laplacian_2d_dirichlet(9, 7)
    X = start_block(A.n, 3, seed=0)
    c = co.filter_coefficients(0.0, 8.0, 1.0, 2.0, 10, "jackson")
    l1, l2 = co.affine_map(0.0, 8.0)
    assert np.array_equal(clenshaw_filter(A, X, c, l1, l2, 0), c[0] * X)
    Y1 = clenshaw_filter(A, X, c, l1, l2, 1)
    assert _rel(Y1, c[0] * X + c[1] * (l1 * (A.to_dense() @ X) + l2 * X)) < 1e-14
    steps = list(clenshaw_steps(A, X, c, l1, l2))
    assert len(steps) == 10
    assert _rel(steps[-1], clenshaw_filter(A, X, c, l1, l2)) < 1e-14


def test_symmetric_interval_no_division_breakdown():
    A = tight_binding_3d_periodic(4, seed=0)
    lmin, lmax = -7.0, 7.0
    c = co.filter_coefficients(lmin, lmax, -0.5, 0.5, 31, "jackson")  # odd degree, a_k = 0
    assert c[-1] == 0.0 or abs(c[-1]) < 1e-16
    l1, l2 = co.affine_map(lmin, lmax)
    X = start_block(A.n, 4, seed=0, complex_=True)
    Y = clenshaw_filter(A, X, c, l1, l2)
    assert np.all(np.isfinite(Y))
    assert _rel(Y, forward_filter(A, X, c, l1, l2)) < 1e-12
