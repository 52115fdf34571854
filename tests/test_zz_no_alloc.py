"""GPU test of the allocation-free residual call (afsi_residual_norms_noalloc) through
the C ABI: on two calls in a row, the second with a smaller input, it gives the same
norms as afsi_residual_norms (same kernels, same fixed-order reductions: identical
bits) and agrees with the oracle's residual norms; shapes beyond its fixed scratch are
rejected with AFSI_E_INVALID."""
import numpy as np
import pytest

from oracle import dense as odense
from paper_2604_00914_amd import afsi
from tests.gpu_util import DEV, torch
from workloads import start_block

pytestmark = pytest.mark.gpu


def _pair(n, q, cplx, seed):
    V = start_block(n, q, seed=seed, complex_=cplx)
    AV = start_block(n, q, seed=seed + 1, complex_=cplx)
    lam = np.random.default_rng(seed + 2).standard_normal(q)
    return V, AV, lam


@pytest.mark.parametrize("cplx", [False, True])
def test_noalloc_residuals_equal_allocating_call(cplx):
    t = torch()
    for n, q, ld, seed in ((200_003, 300, 304, 1), (5_001, 37, 40, 2)):
        V0, AV0, lam = _pair(n, q, cplx, seed)
        dt = t.complex128 if cplx else t.float64
        Vs = t.zeros((n, ld), dtype=dt, device=DEV)
        AVs = t.zeros((n, ld), dtype=dt, device=DEV)
        Vs[:, :q] = t.from_numpy(V0).to(DEV)
        AVs[:, :q] = t.from_numpy(AV0).to(DEV)
        V, AV = Vs[:, :q], AVs[:, :q]
        got = afsi.afsi_residual_norms_noalloc(V, AV, lam)
        ref = afsi.afsi_residual_norms(V, AV, lam)
        assert np.array_equal(got, ref), (n, q)
        oracle = odense.residual_norms(V0, AV0, lam)
        assert np.max(np.abs(got - oracle) / oracle) <= 1e-13, (n, q)
        again = afsi.afsi_residual_norms_noalloc(V, AV, lam)
        assert np.array_equal(again, got)


def test_noalloc_residuals_reject_oversized_shapes():
    t = torch()
    n, q = 1024, 30000  # 2q + partials = 60000 + 3 * 30000 doubles > 2^17
    V = t.zeros((n, q), dtype=t.float64, device=DEV)
    with pytest.raises(afsi.AfsiError) as e:
        afsi.afsi_residual_norms_noalloc(V, V, np.zeros(q))
    assert e.value.status == -1
    # an empty block is a no-op
    E = t.zeros((n, 0), dtype=t.float64, device=DEV)
    assert afsi.afsi_residual_norms_noalloc(E, E, np.zeros(0)).size == 0
