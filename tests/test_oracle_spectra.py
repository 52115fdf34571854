"""Pins of the oracle's interval eigenvalues (oracle.spectra) and of the 27^3 fixture.

The banded routine is checked against dense eigh on grids small enough to
diagonalise; the stored 27^3 window (written by tests/golden/make_golden.py from the
same routine) is checked for the properties the solver tests rely on.
"""
import os

import numpy as np
import pytest

from oracle import spectra
from workloads import build_config, laplacian_2d_dirichlet, laplacian_3d_dirichlet
from workloads.matrices import random_banded_symmetric

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("N,seed", [(5, 0), (8, 3), (9, 1)])
def test_banded_interval_matches_dense_eigh(N, seed):
    A = laplacian_3d_dirichlet(N, potential_scale=2.0, seed=seed)
    assert spectra.bandwidth(A) == N * N
    w = np.linalg.eigvalsh(A.to_scipy().toarray())
    for lo_i, hi_i in ((3, 20), (0, N ** 3 // 2), (N ** 3 // 3, N ** 3 - 1)):
        a = w[lo_i] - 0.5 * (w[lo_i] - w[lo_i - 1]) if lo_i > 0 else w[0] - 1.0
        b = w[hi_i] + 0.5 * (w[hi_i + 1] - w[hi_i]) if hi_i + 1 < w.size else w[-1] + 1.0
        got = spectra.eigenvalues_in_interval(A, a, b)
        ref = w[(w >= a) & (w <= b)]
        assert got.size == ref.size
        assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.abs(w).max())


def test_banded_interval_multiplicities_closed_form():
    """The plain 2D Laplacian has double eigenvalues (i, j) <-> (j, i): counted twice."""
    from oracle import closed_form

    A = laplacian_2d_dirichlet(12)
    w = closed_form.lap2d_eigs(12)
    a, b = 1.0, 3.0
    got = spectra.eigenvalues_in_interval(A, a, b)
    ref = w[(w >= a) & (w <= b)]
    assert got.size == ref.size
    assert np.max(np.abs(got - ref)) < 1e-12


def test_lower_band_layout_and_rejections():
    A = random_banded_symmetric(300, seed=2, band=5, per_row_band=3, per_row_random=0)
    ab = spectra.lower_band(A)
    D = A.to_scipy().toarray()
    w = spectra.bandwidth(A)
    for d in range(w + 1):
        assert np.array_equal(ab[d, : 300 - d], np.diag(D, -d))
    with pytest.raises(ValueError):
        spectra.eigenvalues_in_interval(A, 1.0, 1.0)


def _fixture():
    from tests.golden_util import lap3d27_header, lap3d27_window

    path = os.path.join(GOLDEN, "lap3d_pot_27_window.txt")
    if not os.path.exists(path):
        pytest.skip("lap3d_pot_27 fixture not generated")
    return lap3d27_window(), lap3d27_header()


def test_lap3d27_fixture_window_and_gaps():
    w, h = _fixture()
    A, (lo, hi), (a, b), cfg = build_config("lap3d_pot_27")
    # the fixture belongs to this exact workload and window
    assert (h["lo"], h["hi"], h["a"], h["b"]) == (float(lo), float(hi), float(a), float(b))
    assert w.size == 196 and cfg.p >= 1.8 * w.size
    assert np.all(np.diff(w) >= 0) and w[0] >= a and w[-1] <= b
    # both ends in gaps far wider than the FP64 tolerance (1e-10 ||A||): counts are stable
    normA = max(abs(lo), abs(hi))
    gap = min(w[0] - a, a - h["below"], b - w[-1], h["above"] - b)
    assert gap > 1e4 * 1e-10 * normA
    # density of states: ~0.1435 per site per unit energy mid-spectrum
    dos = w.size / ((b - a) * A.n)
    assert 0.12 < dos < 0.17
