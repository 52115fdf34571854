"""Host-side pins of the locality ordering entry points (no GPU).

* afsi_grid_order against the ordering written out as nested loops over tiles, x and
  the tile's points;
* afsi_csr_permute against the definition B[i, j] = A[perm[i], perm[j]] evaluated by
  scipy's fancy indexing, for real and complex matrices, with ragged rows;
* the spectrum is unchanged (dense eigvalsh of A and of P A P^T);
* invalid permutations and sizes are rejected.
"""
import numpy as np
import pytest

from paper_2604_00914_amd import afsi
from workloads import laplacian_3d_dirichlet, random_banded_symmetric, tight_binding_3d_periodic


def _loops(nx, ny, nz, ty, tz, fold=False):
    xs = list(range(nx))
    if fold:  # 0, nx-1, 1, nx-2, ...
        xs = [xs[i // 2] if i % 2 == 0 else xs[nx - 1 - i // 2] for i in range(nx)]
    out = []
    for y0 in range(0, ny, ty):
        for z0 in range(0, nz, tz):
            for x in xs:
                for y in range(y0, min(ny, y0 + ty)):
                    for z in range(z0, min(nz, z0 + tz)):
                        out.append((x * ny + y) * nz + z)
    return np.array(out, dtype=np.int64)


@pytest.mark.parametrize("dims", [(5, 7, 6, 3, 4), (4, 4, 4, 4, 4), (6, 5, 5, 1, 1), (3, 10, 9, 25, 25),
                                  (1, 1, 1, 1, 1), (0, 3, 3, 2, 2), (7, 3, 11, 2, 5)])
def test_grid_order_is_the_tiled_loop_order(dims):
    perm = afsi.afsi_grid_order(*dims)
    assert np.array_equal(perm, _loops(*dims))
    n = dims[0] * dims[1] * dims[2]
    assert np.array_equal(np.sort(perm), np.arange(n))


@pytest.mark.parametrize("dims", [(5, 7, 6, 3, 4), (6, 4, 4, 4, 4), (1, 2, 2, 1, 1), (9, 3, 11, 2, 5)])
def test_grid_order_folded_is_the_tiled_loop_order(dims):
    perm = afsi.afsi_grid_order(*dims, fold_x=True)
    assert np.array_equal(perm, _loops(*dims, fold=True))


def test_folded_order_keeps_periodic_neighbours_close():
    # the periodic 16^3 lattice in folded 4 x 8 pencils: every +-x neighbour (the
    # wrap-around pair included) is at most two cross-sections (2 * 32 rows) away
    L, ty, tz = 16, 4, 8
    A = tight_binding_3d_periodic(L, seed=0)
    perm = afsi.afsi_grid_order(L, L, L, ty, tz, fold_x=True)
    pos = np.empty_like(perm)
    pos[perm] = np.arange(perm.size)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    cols = A.col.astype(np.int64)
    xr, xc = rows // (L * L), cols // (L * L)
    xnb = xr != xc
    assert np.all(np.abs(pos[rows[xnb]] - pos[cols[xnb]]) <= 2 * ty * tz)


def test_grid_order_neighbour_distance():
    # a 7-point stencil in the 25 x 25 pencil ordering of the 100^3 grid: the +-x
    # neighbours sit 625 rows away, and only points on a tile face have a farther one
    N, t = 100, 25
    perm = afsi.afsi_grid_order(N, N, N, t, t)
    pos = np.empty_like(perm)
    pos[perm] = np.arange(perm.size)
    x, y, z = np.unravel_index(perm, (N, N, N))
    inner = (x > 0) & (y % t > 0) & (y % t < t - 1) & (z % t > 0) & (z % t < t - 1)
    i = np.nonzero(inner)[0]
    old = perm[i]
    assert np.all(pos[old - N * N] == i - t * t)
    assert np.all(pos[old - N] == i - t) and np.all(pos[old - 1] == i - 1)


@pytest.mark.parametrize("which", ["lap3d", "banded", "complex"])
def test_csr_permute_is_p_a_pt(which):
    A = {"lap3d": lambda: laplacian_3d_dirichlet(7, 2.0, seed=3),
         "banded": lambda: random_banded_symmetric(300, seed=2, band=9),
         "complex": lambda: tight_binding_3d_periodic(5, seed=4)}[which]()
    perm = np.random.default_rng(1).permutation(A.n) if which != "lap3d" else afsi.afsi_grid_order(7, 7, 7, 3, 2)
    B = afsi.afsi_csr_permute(A, perm)
    R = A.to_scipy()[perm][:, perm].tocsr()
    R.sort_indices()
    assert np.array_equal(B.row_ptr, R.indptr)
    assert np.array_equal(B.col, R.indices)
    assert np.array_equal(B.val, R.data)
    assert B.val.dtype == A.val.dtype
    wa = np.linalg.eigvalsh(A.to_dense())
    wb = np.linalg.eigvalsh(B.to_dense())
    assert np.max(np.abs(wa - wb)) <= 1e-12 * np.max(np.abs(wa))


def test_csr_permute_rejects_bad_input():
    A = laplacian_3d_dirichlet(3, 0.0)
    for bad in (np.zeros(A.n, dtype=np.int64), np.arange(1, A.n + 1), np.r_[np.arange(A.n - 1), -1]):
        with pytest.raises(afsi.AfsiError) as e:
            afsi.afsi_csr_permute(A, bad)
        assert e.value.status == -1
    with pytest.raises(afsi.AfsiError):
        afsi.afsi_grid_order(3, 3, 3, 0, 2)
    with pytest.raises(afsi.AfsiError):
        afsi.afsi_grid_order(-1, 3, 3, 1, 1)
