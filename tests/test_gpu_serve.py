"""GPU tests of the continuous-batching server (afsi_server_* through the C ABI).

* a slice gives bit-identical eigenpairs alone and batched with other slices of
  its matrix plus an unrelated complex matrix running on another stream;
* every slice matches dense eigendecomposition (FP64 tolerances: eigenvalues
  within 1e-10 ||A||, residuals <= 1e-9 ||A||, exact counts);
* admission by device footprint, rejection of requests that can never fit;
* the mixed form through the server; the timed stream reports latencies.
"""
import numpy as np
import pytest

from paper_2604_00914_amd import afsi, serve
from tests.gpu_util import DEV, torch
from workloads import build_config, laplacian_3d_dirichlet, random_banded_symmetric, tight_binding_3d_periodic

pytestmark = pytest.mark.gpu


def _opts(kmax, max_iter=300, dtype=afsi.R64, tau_c=1e-10):
    o = afsi.afsi_options_default(kmax)
    o.max_iter = max_iter
    o.filter_dtype = dtype
    o.tau_c = tau_c
    return o


@pytest.fixture(scope="module")
def banded():
    A = random_banded_symmetric(2000, seed=1, band=16)
    w = np.linalg.eigvalsh(A.to_dense())
    lmin, lmax = w[0] - 1e-2, w[-1] + 1e-2
    mid = A.n // 2
    slices = []
    for s in range(3):
        lo = mid - 18 + 12 * s
        a = 0.5 * (w[lo - 1] + w[lo])
        b = 0.5 * (w[lo + 11] + w[lo + 12])
        slices.append((a, b, w[lo: lo + 12]))
    return A, (lmin, lmax), slices


def _fetch_all(S, rid, n, p, cplx=False):
    t = torch()
    info = S.wait(rid, 600.0)
    assert info.state == 2, info.status
    E = t.zeros((n, p), dtype=t.complex128 if cplx else t.float64, device=DEV)
    lam, res = S.fetch(rid, p, E)
    return lam, res, E[:, : len(lam)].cpu().numpy(), info


# (filter dtype, tau_c, eigenvalue / residual tolerance relative to ||A||): the FP64
# form and the mixed form (FP32 filter, FP64 dense steps)
FORMS = {"fp64": (afsi.R64, 1e-10, 1e-10, 1e-9), "mixed": (afsi.R32, 1e-6, 1e-5, 1e-5)}


@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_slice_alone_equals_slice_in_mix(banded, form):
    # p = 64 columns: a width the grouped kernel maps (FP64 32 vectors, FP32 16), and
    # after pairs lock the filtered width is padded up to such a width, so the slices of
    # the mix share grouped-kernel launches for the whole solve
    dtype, tau_c, eig_tol, res_tol = FORMS[form]
    A, bounds, slices = banded
    M = afsi.Matrix(A, bounds=bounds)
    normA = max(abs(bounds[0]), abs(bounds[1]))
    p, k = 64, 200
    with serve.Server(hbm_budget_bytes=8 << 30) as S:
        S.set_pool_columns(M, 3 * p)
        a, b, _ = slices[1]
        rid = S.submit(M, a, b, p, _opts(k, dtype=dtype, tau_c=tau_c), seed=11)
        alone = _fetch_all(S, rid, A.n, p)
        st_alone = S.stats()
    T = tight_binding_3d_periodic(8, seed=2)
    MT = afsi.Matrix(T, bounds=(-7.0, 7.0))
    with serve.Server(hbm_budget_bytes=8 << 30) as S:
        S.set_pool_columns(M, 3 * p)
        ids = []
        for s, (a, b, _) in enumerate(slices):
            ids.append(S.submit(M, a, b, p, _opts(k, dtype=dtype, tau_c=tau_c), seed=10 + s))
        other = S.submit(MT, -0.3, 0.3, 32, _opts(120, max_iter=5, dtype=afsi.C128), seed=99)
        mixed = [_fetch_all(S, r, A.n, p) for r in ids]
        _fetch_all(S, other, T.n, 32, cplx=True)
        st = S.stats()
    # the lone slice ran every product in the grouped kernel (its widths were padded)
    assert st_alone["kernel_slices"] == st_alone["batched_groups"] == st_alone["kernel_launches"]
    # in the mix, grouped-kernel launches really carried several slices
    assert st["kernel_slices"] > 1.25 * st["kernel_launches"], st
    lam_a, res_a, V_a, info_a = alone
    lam_m, res_m, V_m, info_m = mixed[1]
    # the same bits alone and in the mix (each column's arithmetic ignores its neighbours)
    assert np.array_equal(lam_a, lam_m) and np.array_equal(res_a, res_m) and np.array_equal(V_a, V_m)
    assert info_a.iterations == info_m.iterations
    for (a, b, ref), (lam, res, V, info) in zip(slices, mixed):
        assert info.converged and lam.size == ref.size
        assert np.max(np.abs(lam - ref)) <= eig_tol * normA
        R = A.to_scipy() @ V - V * lam
        assert np.max(np.linalg.norm(R, axis=0)) <= res_tol * normA
    M.close()
    MT.close()


def test_admission_waits_for_memory():
    A1 = laplacian_3d_dirichlet(12, 2.0, seed=1)
    A2 = laplacian_3d_dirichlet(12, 2.0, seed=2)
    M1, M2 = afsi.Matrix(A1, bounds=(0.0, 14.0)), afsi.Matrix(A2, bounds=(0.0, 14.0))
    p = 32
    one = 3 * A1.n * p * 8 + A1.n * p * 8
    with serve.Server(hbm_budget_bytes=int(1.5 * one)) as S:
        r1 = S.submit(M1, 6.9, 7.1, p, _opts(60, max_iter=4), seed=1)
        r2 = S.submit(M2, 6.9, 7.1, p, _opts(60, max_iter=4), seed=2)
        i1 = S.wait(r1, 300.0)
        i2 = S.wait(r2, 300.0)
        assert i1.state == 2 and i2.state == 2
        assert i2.t_admit >= i1.t_done
        S.fetch(r1, p)
        S.fetch(r2, p)
        with pytest.raises(afsi.AfsiError) as e:
            S.submit(M1, 6.9, 7.1, 1000, _opts(60), seed=3)
        assert e.value.status == -7
    M1.close()
    M2.close()


def test_mixed_form_through_server():
    A, (lmin, lmax), (a, b), cfg = build_config("lap2d_64")
    M = afsi.Matrix(A, bounds=(lmin, lmax))
    normA = max(abs(lmin), abs(lmax))
    from tests.golden_util import lap2d_window

    ref = lap2d_window()
    with serve.Server(hbm_budget_bytes=4 << 30) as S:
        rid = S.submit(M, a, b, cfg.p, _opts(cfg.degree, dtype=afsi.R32, tau_c=1e-6), seed=5)
        lam, res, V, info = _fetch_all(S, rid, A.n, cfg.p)
    assert info.status == 0 and lam.size == 40
    assert np.max(np.abs(lam - ref)) <= 1e-5 * normA
    assert np.max(res) <= 1e-5 * normA
    M.close()


def test_timed_stream_reports_latency():
    mats = [afsi.Matrix(laplacian_3d_dirichlet(N, 2.0, seed=N), bounds=(0.0, 14.0)) for N in (10, 12, 14)]
    jobs = []
    for i in range(9):
        M = mats[i % 3]
        jobs.append((0.02 * i, M, 6.95, 7.05, 32, _opts(60, max_iter=3), 100 + i, i))
    with serve.Server(hbm_budget_bytes=4 << 30) as S:
        rep = serve.run_stream(S, jobs)
    s = rep.summary()
    assert s["requests"] == 9 and s["p99_latency_s"] >= s["p50_latency_s"] > 0
    for M in mats:
        M.close()


def test_requests_arriving_as_pools_drain_all_finish():
    # requests of a few small matrices arriving while earlier ones finish: pools empty,
    # retire and are created again; every request must finish (a request admitted into
    # a pool that is retiring must not be lost)
    mats = [afsi.Matrix(laplacian_3d_dirichlet(N, 2.0, seed=N), bounds=(0.0, 14.0)) for N in (8, 9, 10)]
    jobs = []
    for i in range(36):
        jobs.append((0.004 * i, mats[i % 3], 6.9, 7.1, 32, _opts(20 + i, max_iter=1), 300 + i, i))
    with serve.Server(hbm_budget_bytes=4 << 30) as S:
        rep = serve.run_stream(S, jobs, timeout_s=120.0)
        st = S.stats()
    assert len(rep.completed) == 36 and st["running"] == 0 and st["queued"] == 0
    assert all(c.info.get("state") == 2 for c in rep.completed)
    for M in mats:
        M.close()
