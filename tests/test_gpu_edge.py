"""GPU edge cases through the C ABI: zero-column blocks, zero-row blocks and an empty
matrix are accepted and change nothing (or give the empty result), inactive or absent
batched groups touch nothing, and an n = 1 matrix filters like its scalar polynomial."""
import numpy as np
import pytest

from oracle import coefficients as co
from paper_2604_00914_amd import afsi
from tests.gpu_util import DEV, to_dev, torch
from workloads import CSR, laplacian_3d_dirichlet, start_block

pytestmark = pytest.mark.gpu


def test_zero_column_blocks_are_no_ops():
    t = torch()
    A = laplacian_3d_dirichlet(6, 1.0, seed=2)
    M = afsi.Matrix(A, bounds=(0.0, 14.0))
    E = lambda: t.empty((A.n, 0), dtype=t.float64, device=DEV)  # noqa: E731
    c = afsi.afsi_filter_coefficients(0.0, 14.0, 3.0, 4.0, 7)
    afsi.afsi_filter_block(M.handle, c, 7, E(), E(), E())
    afsi.afsi_spmm(M.handle, E(), E())
    afsi.afsi_orthonormalize(None, E(), E())
    assert afsi.afsi_rayleigh_ritz(M.handle, E(), E(), E()).size == 0
    assert afsi.afsi_residual_norms(E(), E(), np.zeros(0)).size == 0
    # X^H Y with no columns on one side, and a product with an empty inner dimension
    X = to_dev(start_block(A.n, 5, seed=1))
    G = t.full((0, 5), 7.0, dtype=t.float64, device=DEV)
    afsi.afsi_block_inner(E(), X, G)
    Y = to_dev(start_block(A.n, 3, seed=2))
    Y0 = Y.clone()
    afsi.afsi_block_gemm(E(), t.empty((0, 3), dtype=t.float64, device=DEV), 0.5, Y)
    assert t.equal(Y, 0.5 * Y0)
    dst = t.empty((A.n, 0), dtype=t.float64, device=DEV)
    afsi.afsi_gather_columns(X, np.zeros(0, np.int32), dst)
    t.cuda.synchronize()
    M.close()


def test_zero_row_inner_product_is_zero():
    t = torch()
    X = t.empty((0, 4), dtype=t.float64, device=DEV)
    Y = t.empty((0, 3), dtype=t.float64, device=DEV)
    G = t.full((4, 3), 7.0, dtype=t.float64, device=DEV)
    afsi.afsi_block_inner(X, Y, G)
    t.cuda.synchronize()
    assert not G.cpu().numpy().any()


def test_batched_without_active_groups_touches_nothing():
    t = torch()
    A = laplacian_3d_dirichlet(6, 1.0, seed=3)
    M = afsi.Matrix(A, bounds=(0.0, 14.0))
    X = to_dev(start_block(A.n, 32, seed=4))
    P0 = t.full_like(X, 3.0)
    P1 = t.full_like(X, 5.0)
    afsi.afsi_clenshaw_step_batched(M.handle, [], X, P0, P1)
    c = afsi.afsi_filter_coefficients(0.0, 14.0, 3.0, 4.0, 9)
    l1, l2 = co.affine_map(0.0, 14.0)
    g = afsi.afsi_clenshaw_step_params(c, 9, 3, l1, l2, col0=0, ncols=32)
    g.active = 0
    afsi.afsi_clenshaw_step_batched(M.handle, [g], X, P0, P1)
    t.cuda.synchronize()
    assert bool((P0 == 3.0).all()) and bool((P1 == 5.0).all())
    M.close()


def test_empty_matrix():
    t = torch()
    A = CSR(0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    M = afsi.Matrix(A, bounds=(-1.0, 1.0))
    X = t.empty((0, 8), dtype=t.float64, device=DEV)
    Y, W = t.empty_like(X), t.empty_like(X)
    c = afsi.afsi_filter_coefficients(-1.0, 1.0, -0.2, 0.3, 5)
    afsi.afsi_filter_block(M.handle, c, 5, X, Y, W)
    afsi.afsi_spmm(M.handle, X, Y)
    X32 = t.empty((0, 8), dtype=t.float32, device=DEV)
    afsi.afsi_filter_block(M.handle, c, 5, X32, t.empty_like(X32), t.empty_like(X32))
    t.cuda.synchronize()
    M.close()


@pytest.mark.parametrize("single", [False, True])
def test_one_by_one_matrix_is_the_scalar_polynomial(single):
    t = torch()
    lam = 0.37
    A = CSR(1, np.array([0, 1], np.int64), np.array([0], np.int32), np.array([lam]))
    lmin, lmax, k = -1.0, 1.0, 40
    c = afsi.afsi_filter_coefficients(lmin, lmax, -0.2, 0.5, k)
    M = afsi.Matrix(A, bounds=(lmin, lmax))
    x = np.array([[1.5, -2.0, 0.25, 4.0]])
    dt = t.float32 if single else t.float64
    X = to_dev(x).to(dt)
    Y, W = t.empty_like(X), t.empty_like(X)
    afsi.afsi_filter_block(M.handle, c, k, X, Y, W)
    t.cuda.synchronize()
    rho = float(co.filter_value(np.array([lam]), co.filter_coefficients(lmin, lmax, -0.2, 0.5, k), lmin, lmax)[0])
    tol = (k + 1) * 2.0 ** -21 if single else 1e-13
    assert np.allclose(Y.cpu().numpy().astype(np.float64), rho * x, rtol=tol, atol=tol)
    M.close()
