"""Pins of the oracle's filtered thick-restart block Lanczos (oracle/lanczos.py).

What fixes it, independently of the oracle's own formulas:
* the closed-form spectrum of the 64 x 64 Dirichlet Laplacian (config 1's window: 40
  eigenvalues, several of them double, exact count);
* dense eigh on n <= 2000 matrices of the workload families (3D Laplacian with
  potential, complex tight-binding lattice, random banded) for central windows;
* invariants: the returned vectors are orthonormal eigenvectors (residuals below the
  locking tolerance), every returned value lies in [a, b];
* a window made only of double eigenvalues (24 x 24 Laplacian): both copies of each,
  exact count.
"""
import numpy as np
import pytest

from oracle import closed_form
from oracle import lanczos as ol
from workloads import (
    build_config,
    laplacian_2d_dirichlet,
    laplacian_3d_dirichlet,
    random_banded_symmetric,
    start_block,
    tight_binding_3d_periodic,
)


def _check(A, r, ref, normA, tol=1e-10):
    assert r.converged
    assert r.eigenvalues.size == ref.size
    assert np.max(np.abs(r.eigenvalues - np.sort(ref))) <= tol * normA
    V = r.eigenvectors
    assert V.shape[1] == ref.size
    R = A.to_scipy() @ V - V * r.eigenvalues[None, :]
    assert np.max(np.linalg.norm(R, axis=0)) <= 1e-9 * normA
    assert np.max(np.abs(V.conj().T @ V - np.eye(ref.size))) < 1e-10


@pytest.mark.parametrize("block,basis", [(4, 96), (8, 128)])
def test_config1_closed_form(block, basis):
    A, (lmin, lmax), (a, b), cfg = build_config("lap2d_64")
    exact = closed_form.lap2d_eigs(64)
    exact = exact[(exact >= a) & (exact <= b)]
    assert exact.size == 40
    r = ol.filtered_lanczos(A, a, b, lmin, lmax, start_block(A.n, block, seed=0),
                            ol.LanczosOptions(degree=cfg.degree, block=block, basis=basis))
    _check(A, r, exact, max(abs(lmin), abs(lmax)))
    assert np.all((r.eigenvalues >= a) & (r.eigenvalues <= b))


def _window(A, count):
    w = np.linalg.eigvalsh(A.to_dense())
    lo = A.n // 2 - count // 2
    a = 0.5 * (w[lo - 1] + w[lo])
    b = 0.5 * (w[lo + count - 1] + w[lo + count])
    return w, a, b, w[lo: lo + count]


@pytest.mark.parametrize("case", ["lap3d", "tb", "rand"])
def test_brute_force(case):
    A = {
        "lap3d": lambda: laplacian_3d_dirichlet(12, 2.0, seed=1),
        "tb": lambda: tight_binding_3d_periodic(12, seed=1),
        "rand": lambda: random_banded_symmetric(2000, seed=1, band=16),
    }[case]()
    w, a, b, ref = _window(A, 12)
    lmin, lmax = w[0] - 1e-2, w[-1] + 1e-2
    X0 = start_block(A.n, 4, seed=3, complex_=A.is_complex)
    r = ol.filtered_lanczos(A, a, b, lmin, lmax, X0, ol.LanczosOptions(degree=200, block=4, basis=64))
    _check(A, r, ref, max(abs(lmin), abs(lmax)))


def test_window_of_double_eigenvalues():
    # a 24 x 24 Dirichlet Laplacian has double eigenvalues (i, j) and (j, i): a window
    # of six doubles, found with both copies (exact count) by blocks of four and of one
    A = laplacian_2d_dirichlet(24)
    w = np.sort(closed_form.lap2d_eigs(24))
    lo, hi = 139, 151  # six double eigenvalues, gaps of 1.5e-2 and 1.3e-2 at the ends
    a, b = 0.5 * (w[lo - 1] + w[lo]), 0.5 * (w[hi - 1] + w[hi])
    ref = w[(w >= a) & (w <= b)]
    assert ref.size == 12 and np.sum(np.diff(ref) < 1e-12) == 6
    for block in (4, 1):
        r = ol.filtered_lanczos(A, a, b, 0.0, 8.0, start_block(A.n, block, seed=1),
                                ol.LanczosOptions(degree=120, basis=64, block=block, max_cycles=30))
        _check(A, r, ref, 8.0)
