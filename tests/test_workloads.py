"""Generator sanity: sizes of the published workloads, symmetry, sorted CSR rows."""
import numpy as np
import pytest

from workloads import (
    build_config,
    laplacian_2d_dirichlet,
    laplacian_3d_dirichlet,
    random_banded_symmetric,
    start_block,
    tight_binding_3d_periodic,
)


def _check_csr(A):
    assert A.row_ptr[0] == 0 and A.row_ptr[-1] == A.col.size == A.val.size
    for i in range(min(A.n, 2000)):
        c = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)
    assert A.col.min() >= 0 and A.col.max() < A.n


def test_sizes_of_the_workloads():
    assert laplacian_2d_dirichlet(64).nnz == 20224
    assert laplacian_3d_dirichlet(100, 2.0).nnz == 6_940_000
    assert tight_binding_3d_periodic(64).nnz == 1_835_008


@pytest.mark.parametrize("make", [
    lambda: laplacian_2d_dirichlet(13, 7),
    lambda: laplacian_3d_dirichlet(6, 2.0, seed=3),
    lambda: tight_binding_3d_periodic(5, seed=3),
    lambda: random_banded_symmetric(500, seed=3, band=8),
])
def test_hermitian_and_sorted(make):
    A = make()
    _check_csr(A)
    D = A.to_dense()
    assert np.max(np.abs(D - D.conj().T)) < 1e-15


def test_random_banded_density():
    A = random_banded_symmetric(20000, seed=0)
    assert 22 < A.nnz / A.n < 26


def test_seeds_reproduce():
    assert np.array_equal(start_block(10, 3, 7), start_block(10, 3, 7))
    X = start_block(1000, 4, 1, complex_=True)
    assert abs(np.mean(np.abs(X) ** 2) - 1.0) < 0.1
    A1, _, _, _ = build_config("lap3d_pot_100", size=6, seed=2)
    A2, _, _, _ = build_config("lap3d_pot_100", size=6, seed=2)
    assert np.array_equal(A1.val, A2.val)
