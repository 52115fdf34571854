"""GPU tests of afsi_estimate_eigencount (trace estimation of the filter, Section 3.4)
through the C ABI, against the oracle on the same probe blocks.

* per-probe values Re z_i^H rho(A) z_i equal the oracle's within the FP64 rounding of
  the filter, |diff| <= 2e-11 n max|rho| (real config 1 with Jackson and Lanczos
  damping; complex lattice with complex probes; 1 and 3 probes for the narrow kernels);
* full size: the 100^3 matrix (n = 10^6, degree 120) with 4 probes;
* config 1 with 256 probes estimates the closed-form tr rho(A) within 5 standard errors;
* errors: no bounds, FP32 probes, a >= b, overlapping blocks, no probe columns.
"""
import numpy as np
import pytest

from oracle import eigencount as ec
from paper_2604_00914_amd import afsi
from tests.gpu_util import to_dev, torch
from workloads import build_config, probe_block

pytestmark = pytest.mark.gpu


def _run(M, a, b, degree, Z0, damping, m_exp=0.5):
    t = torch()
    Z = to_dev(Z0)
    Y, W = t.empty_like(Z), t.empty_like(Z)
    est, per = afsi.afsi_estimate_eigencount(M.handle, a, b, degree, Z, Y, W, damping, m_exp)
    return est, per


def _check_parity(A, bounds, a, b, degree, Z0, damping):
    M = afsi.Matrix(A, bounds=bounds)
    est, per = _run(M, a, b, degree, Z0, damping)
    M.close()
    ref = ec.probe_quadratic_forms(A, Z0, bounds[0], bounds[1], a, b, degree, damping)
    tol = 2e-11 * A.n
    assert np.max(np.abs(per - ref)) <= tol, (np.max(np.abs(per - ref)), tol)
    assert abs(est - np.mean(per)) <= 1e-12 * max(1.0, abs(est))
    return est, per


@pytest.mark.parametrize("damping", ["jackson", "lanczos"])
@pytest.mark.parametrize("m", [1, 3, 32])
def test_config1_parity(damping, m):
    A, bounds, (a, b), cfg = build_config("lap2d_64")
    _check_parity(A, bounds, a, b, cfg.degree, probe_block(A.n, m, seed=7), damping)


def test_complex_lattice_parity():
    A, bounds, (a, b), cfg = build_config("tb3d_64", size=8)
    _check_parity(A, bounds, a, b, 90, probe_block(A.n, 16, seed=8, complex_=True), "lanczos")


def test_full_size_config2_four_probes():
    A, bounds, (a, b), cfg = build_config("lap3d_pot_100")
    _check_parity(A, bounds, a, b, cfg.degree, probe_block(A.n, 4, seed=9), "jackson")


def test_config1_estimate_matches_closed_form_trace():
    A, bounds, (a, b), cfg = build_config("lap2d_64")
    N = 64
    ii, jj = np.meshgrid(np.arange(1, N + 1), np.arange(1, N + 1))
    lam = (4 - 2 * np.cos(ii * np.pi / (N + 1)) - 2 * np.cos(jj * np.pi / (N + 1))).ravel()
    tr = ec.filter_trace(lam, bounds[0], bounds[1], a, b, cfg.degree, "jackson")
    M = afsi.Matrix(A, bounds=bounds)
    est, per = _run(M, a, b, cfg.degree, probe_block(A.n, 256, seed=3), "jackson")
    M.close()
    se = per.std(ddof=1) / np.sqrt(per.size)
    assert abs(est - tr) < 5 * se
    assert abs(tr - 40) < 1.0


def test_errors():
    t = torch()
    A, bounds, (a, b), cfg = build_config("lap2d_64")
    Z0 = probe_block(A.n, 4, seed=1)
    M = afsi.Matrix(A)  # no bounds yet
    with pytest.raises(afsi.AfsiError) as e:
        _run(M, a, b, 10, Z0, "jackson")
    assert e.value.status == -1
    afsi.afsi_set_spectral_bounds(M.handle, *bounds)
    Z = to_dev(Z0)
    Y, W = t.empty_like(Z), t.empty_like(Z)
    with pytest.raises(afsi.AfsiError):
        afsi.afsi_estimate_eigencount(M.handle, b, a, 10, Z, Y, W)           # a >= b
    with pytest.raises(afsi.AfsiError):
        afsi.afsi_estimate_eigencount(M.handle, a, b, 0, Z, Y, W)           # degree 0
    with pytest.raises(afsi.AfsiError):
        afsi.afsi_estimate_eigencount(M.handle, a, b, 10, Z, Z, W)          # Y overlaps Z
    Z32 = Z.to(t.float32)
    with pytest.raises(afsi.AfsiError):
        afsi.afsi_estimate_eigencount(M.handle, a, b, 10, Z32, t.empty_like(Z32), t.empty_like(Z32))
    E = t.empty((A.n, 0), dtype=t.float64, device=Z.device)
    with pytest.raises(afsi.AfsiError):
        afsi.afsi_estimate_eigencount(M.handle, a, b, 10, E, t.empty_like(E), t.empty_like(E))
    # the probe block is left unchanged
    est, per = afsi.afsi_estimate_eigencount(M.handle, a, b, 10, Z, Y, W)
    assert np.array_equal(Z.cpu().numpy(), Z0) and np.isfinite(est)
    M.close()
