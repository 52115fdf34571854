"""GPU parity of the filtered thick-restart block Lanczos (afsi_filtered_lanczos) with
the oracle (oracle/lanczos.py) on the same start block, through the C ABI.

Bar (as for the subspace-iteration solver): the count in [a, b] equals the oracle's
and the exact count (closed form or dense eigh); eigenvalues within 1e-10 ||A|| of the
oracle's and of the exact ones; residuals ||A v - lambda v|| <= 1e-9 ||A|| recomputed
on the host; returned vectors orthonormal.
"""
import numpy as np
import pytest

from oracle import closed_form
from oracle import lanczos as ol
from paper_2604_00914_amd import afsi
from tests.gpu_util import DEV, to_dev, torch
from workloads import (
    build_config,
    laplacian_2d_dirichlet,
    laplacian_3d_dirichlet,
    random_banded_symmetric,
    start_block,
    tight_binding_3d_periodic,
)

pytestmark = pytest.mark.gpu


def _gpu(A, a, b, bounds, X0, degree, block, basis, max_cycles=200, capacity=None, mixed=False):
    t = torch()
    M = afsi.Matrix(A, bounds=bounds)
    o = afsi.afsi_lanczos_options_default(degree)
    o.block, o.basis, o.max_cycles = block, basis, max_cycles
    if mixed:
        o.mixed, o.tau_c = 1, 1e-6
    cap = capacity or 2 * basis
    E = t.zeros((A.n, cap), dtype=t.complex128 if A.is_complex else t.float64, device=DEV)
    st, lam, res, r = afsi.afsi_filtered_lanczos(M.handle, a, b, o, to_dev(X0), E)
    V = E[:, : lam.size].cpu().numpy()
    M.close()
    return st, lam, res, V, r


def _check(A, st, lam, V, r, ref_exact, oracle, normA):
    assert st == 0 and r.converged
    assert lam.size == ref_exact.size == oracle.eigenvalues.size
    assert np.max(np.abs(lam - np.sort(ref_exact))) <= 1e-10 * normA
    assert np.max(np.abs(lam - oracle.eigenvalues)) <= 1e-10 * normA
    assert np.all((lam >= lam.min()) & np.isfinite(lam))
    R = A.to_scipy() @ V - V * lam[None, :]
    assert np.max(np.linalg.norm(R, axis=0)) <= 1e-9 * normA
    assert np.max(np.abs(V.conj().T @ V - np.eye(lam.size))) < 1e-10


@pytest.mark.parametrize("block,basis", [(4, 96), (8, 128)])
def test_config1_against_oracle_and_closed_form(block, basis):
    A, (lmin, lmax), (a, b), cfg = build_config("lap2d_64")
    exact = closed_form.lap2d_eigs(64)
    exact = exact[(exact >= a) & (exact <= b)]
    X0 = start_block(A.n, block, seed=0)
    orc = ol.filtered_lanczos(A, a, b, lmin, lmax, X0,
                              ol.LanczosOptions(degree=cfg.degree, block=block, basis=basis))
    st, lam, res, V, r = _gpu(A, a, b, (lmin, lmax), X0, cfg.degree, block, basis)
    _check(A, st, lam, V, r, exact, orc, max(abs(lmin), abs(lmax)))
    assert np.all((lam >= a) & (lam <= b))
    # the same work as the oracle up to rounding: within a cycle of it
    assert abs(r.cycles - orc.cycles) <= 1


def _window(A, count):
    w = np.linalg.eigvalsh(A.to_dense())
    lo = A.n // 2 - count // 2
    a = 0.5 * (w[lo - 1] + w[lo])
    b = 0.5 * (w[lo + count - 1] + w[lo + count])
    return w, a, b, w[lo: lo + count]


@pytest.mark.parametrize("case", ["lap3d", "tb", "rand"])
def test_brute_force_against_oracle(case):
    A = {
        "lap3d": lambda: laplacian_3d_dirichlet(12, 2.0, seed=1),
        "tb": lambda: tight_binding_3d_periodic(12, seed=1),
        "rand": lambda: random_banded_symmetric(2000, seed=1, band=16),
    }[case]()
    w, a, b, ref = _window(A, 12)
    lmin, lmax = w[0] - 1e-2, w[-1] + 1e-2
    X0 = start_block(A.n, 4, seed=3, complex_=A.is_complex)
    orc = ol.filtered_lanczos(A, a, b, lmin, lmax, X0, ol.LanczosOptions(degree=200, block=4, basis=64))
    st, lam, res, V, r = _gpu(A, a, b, (lmin, lmax), X0, 200, 4, 64)
    _check(A, st, lam, V, r, ref, orc, max(abs(lmin), abs(lmax)))


@pytest.mark.parametrize("block", [4, 1])
def test_window_of_double_eigenvalues(block):
    # six double eigenvalues of the 24 x 24 Dirichlet Laplacian: both copies of each
    A = laplacian_2d_dirichlet(24)
    w = np.sort(closed_form.lap2d_eigs(24))
    lo, hi = 139, 151
    a, b = 0.5 * (w[lo - 1] + w[lo]), 0.5 * (w[hi - 1] + w[hi])
    ref = w[(w >= a) & (w <= b)]
    X0 = start_block(A.n, block, seed=1)
    orc = ol.filtered_lanczos(A, a, b, 0.0, 8.0, X0,
                              ol.LanczosOptions(degree=120, basis=64, block=block, max_cycles=30))
    st, lam, res, V, r = _gpu(A, a, b, (0.0, 8.0), X0, 120, block, 64, max_cycles=30)
    _check(A, st, lam, V, r, ref, orc, 8.0)


def test_errors_and_cycle_limit():
    t = torch()
    A = laplacian_3d_dirichlet(8, 2.0, seed=1)
    M = afsi.Matrix(A, bounds=(0.0, 14.0))
    X0 = to_dev(start_block(A.n, 4, seed=1))
    E = t.zeros((A.n, 64), dtype=t.float64, device=DEV)
    o = afsi.afsi_lanczos_options_default(40)
    o.basis = 6  # below 2 * block
    with pytest.raises(afsi.AfsiError):
        afsi.afsi_filtered_lanczos(M.handle, 6.9, 7.1, o, X0, E)
    o = afsi.afsi_lanczos_options_default(40)
    o.basis, o.max_cycles = 32, 1
    st, lam, res, r = afsi.afsi_filtered_lanczos(M.handle, 6.9, 7.1, o, X0, E)
    assert r.cycles == 1 and (st == -6) == (not r.converged)  # stops at the limit
    M.close()


@pytest.mark.parametrize("case", ["config1", "tb"])
def test_mixed_form_within_tolerance(case):
    # the FP32 (complex FP32) filter with FP64 Krylov basis, Rayleigh-Ritz and residuals,
    # locking at 1e-6 ||A||: exact counts, eigenvalues within 1e-5 ||A|| of the exact ones
    # and of the FP64 oracle's, residuals <= 1e-5 ||A||
    if case == "config1":
        A, (lmin, lmax), (a, b), cfg = build_config("lap2d_64")
        ref = closed_form.lap2d_eigs(64)
        ref = ref[(ref >= a) & (ref <= b)]
        deg, block, basis = cfg.degree, 8, 128
    else:
        A = tight_binding_3d_periodic(12, seed=1)
        w, a, b, ref = _window(A, 12)
        lmin, lmax = w[0] - 1e-2, w[-1] + 1e-2
        deg, block, basis = 200, 4, 64
    normA = max(abs(lmin), abs(lmax))
    X0 = start_block(A.n, block, seed=5, complex_=A.is_complex)
    orc = ol.filtered_lanczos(A, a, b, lmin, lmax, X0, ol.LanczosOptions(degree=deg, block=block, basis=basis))
    st, lam, res, V, r = _gpu(A, a, b, (lmin, lmax), X0, deg, block, basis, mixed=True)
    assert st == 0 and r.converged and lam.size == ref.size == orc.eigenvalues.size
    assert np.max(np.abs(lam - np.sort(ref))) <= 1e-5 * normA
    assert np.max(np.abs(lam - orc.eigenvalues)) <= 1e-5 * normA
    R = A.to_scipy() @ V - V * lam[None, :]
    assert np.max(np.linalg.norm(R, axis=0)) <= 1e-5 * normA
    assert np.max(np.abs(V.conj().T @ V - np.eye(lam.size))) < 1e-8
