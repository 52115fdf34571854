"""CPU tests of the C ABI: the library loads, exports what include/afsi.h declares,
and its host-side logic agrees with the oracle (no GPU calls)."""
import os
import re

import numpy as np
import pytest

from oracle import coefficients as co
from oracle import solver as osolver
from oracle.degree import select_degree as oracle_select_degree
from oracle.filter import clenshaw_filter
from paper_2604_00914_amd import afsi
from workloads import random_dense_symmetric_csr, start_block

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _built():
    if not os.path.exists(afsi.LIB_PATH):
        from paper_2604_00914_amd import build

        build.build()


def _declared():
    text = open(os.path.join(ROOT, "include", "afsi.h")).read()
    return sorted(set(re.findall(r"\b(afsi_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = afsi.lib()
    names = _declared()
    assert len(names) >= 25
    for name in names:
        assert hasattr(L, name), name
    assert set(afsi.exported_symbols()) == set(names)


def test_version_and_no_device_here():
    assert "gfx950" in afsi.afsi_version()


@pytest.mark.parametrize("damping,m", [("jackson", 0.5), ("lanczos", 0.5), ("lanczos", 1.0), ("none", 0.0)])
@pytest.mark.parametrize("interval", [(0.1285, 0.2556), (-0.3, 0.3), (-9.0, -6.5), (7.9, 20.0)])
def test_coefficients_match_oracle(damping, m, interval):
    lmin, lmax = -7.0, 8.0
    a, b = interval
    got = afsi.afsi_filter_coefficients(lmin, lmax, a, b, 150, damping, m)
    ref = co.filter_coefficients(lmin, lmax, a, b, 150, damping, m)
    assert np.max(np.abs(got - ref)) < 1e-14


def test_coefficient_errors():
    with pytest.raises(afsi.AfsiError) as e:
        afsi.afsi_filter_coefficients(0.0, 1.0, 0.5, 0.4, 10)
    assert e.value.status == -1
    with pytest.raises(afsi.AfsiError):
        afsi.afsi_filter_coefficients(1.0, 1.0, 0.1, 0.4, 10)


def _emulate_schedule(A, X, coeffs, k, l1, l2):
    """Run the library's product schedule with dense numpy arithmetic (host check)."""
    P = {0: X, 1: np.zeros_like(X), 2: np.zeros_like(X)}
    for s in range(k):
        g = afsi.afsi_clenshaw_step_params(coeffs, k, s, l1, l2)
        src = P[g.src]
        out = g.sigma * (A @ src) + g.tau * src
        if g.has_v:
            out = out - P[g.dst]
        out = out + g.alpha * X
        P[g.dst] = out
    return P[1 + (k - 1) % 2]


@pytest.mark.parametrize("k", [1, 2, 3, 4, 17, 60])
def test_step_schedule_reproduces_clenshaw(k):
    Acsr = random_dense_symmetric_csr(60, 0.2, seed=2)
    D = Acsr.to_dense()
    w = np.linalg.eigvalsh(D)
    lmin, lmax = w[0] - 0.1, w[-1] + 0.1
    c = co.filter_coefficients(lmin, lmax, w[20], w[30], k, "jackson")
    l1, l2 = co.affine_map(lmin, lmax)
    X = start_block(60, 4, seed=1)
    got = _emulate_schedule(D, X, c, k, l1, l2)
    ref = clenshaw_filter(Acsr, X, c, l1, l2)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_select_degree_matches_oracle():
    rng = np.random.default_rng(7)
    lmin, lmax = -2.0, 5.0
    l1, l2 = co.affine_map(lmin, lmax)
    for trial in range(40):
        a = rng.uniform(-1.5, 3.5)
        b = a + rng.uniform(0.05, 1.0)
        damping = ["jackson", "lanczos", "none"][trial % 3]
        c = co.filter_coefficients(lmin, lmax, a, b, 120, damping, 0.5)
        ritz = np.sort(rng.uniform(lmin, lmax, size=rng.integers(3, 40)))
        inside = (ritz >= a) & (ritz <= b)
        e = int(inside.sum())
        if e == 0:
            continue
        assert afsi.afsi_select_degree(ritz, e, c, l1, l2, 1e-3) == oracle_select_degree(ritz, e, c, l1, l2, 1e-3)


def test_lock_select_matches_oracle_sequences():
    rng = np.random.default_rng(3)
    for trial in range(30):
        p = int(rng.integers(2, 12))
        a, b = 0.0, 1.0
        ritz = np.sort(rng.uniform(-0.5, 1.5, size=p))
        if not np.any((ritz >= a) & (ritz <= b)):
            ritz[0] = 0.5
            ritz = np.sort(ritz)
        st = osolver.ControlState(n_lock=int(rng.integers(0, 3)), n_check_prev=int(rng.integers(0, 4)))
        n_check_prev = st.n_check_prev
        res = 10.0 ** rng.uniform(-13, -1, size=p)
        Iidx = np.nonzero((ritz >= a) & (ritz <= b))[0]
        I_o, L_o, done_o = osolver.control_step(ritz, res[Iidx], Iidx, a, b, 1e-10, st)
        Imask = (ritz >= a) & (ritz <= b)
        I_c, L_c, done_c, ncheck = afsi.afsi_lock_select(ritz, res, Imask, a, b, 1e-10, st.n_lock, n_check_prev)
        assert list(np.nonzero(I_c)[0]) == list(I_o)
        assert list(np.nonzero(L_c)[0]) == list(L_o)
        assert done_c == done_o and ncheck == st.n_check_prev


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("p", [1, 2, 3, 5, 64, 200, 333])
def test_host_eigh_against_numpy(cplx, p):
    rng = np.random.default_rng(p)
    M = rng.standard_normal((p, p)) + (1j * rng.standard_normal((p, p)) if cplx else 0)
    B = M + M.conj().T
    w, U = afsi.afsi_host_eigh(B)
    wr = np.linalg.eigvalsh(B)
    scale = max(1.0, np.max(np.abs(wr)))
    assert np.max(np.abs(w - wr)) < 1e-12 * scale * max(1, p / 10)
    assert np.max(np.abs(U.conj().T @ U - np.eye(p))) < 1e-12 * max(1, p / 10)
    assert np.max(np.abs(B @ U - U * w)) < 1e-11 * scale * max(1, p / 10)


@pytest.mark.parametrize("cplx", [False, True])
def test_host_eigh_degenerate_and_diagonal(cplx):
    # clustered / repeated eigenvalues (the Laplacian window has double eigenvalues)
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)) + (1j * rng.standard_normal((40, 40)) if cplx else 0))
    lam = np.repeat(np.linspace(-1, 1, 10), 4)
    B = (Q * lam) @ Q.conj().T
    w, U = afsi.afsi_host_eigh(B)
    assert np.max(np.abs(w - np.sort(lam))) < 1e-13
    assert np.max(np.abs(B @ U - U * w)) < 1e-13
    w, U = afsi.afsi_host_eigh(np.diag([3.0, 1.0, 2.0]))
    assert np.allclose(w, [1, 2, 3])


def _structured_spectra(p, rng, cplx):
    """Matrices whose tridiagonal forms exercise every branch of the divide and conquer
    step: deflation by a small z entry, by two close poles, graded and zero spectra."""
    Q, _ = np.linalg.qr(rng.standard_normal((p, p)) + (1j * rng.standard_normal((p, p)) if cplx else 0))
    out = {
        "4-fold": np.repeat(rng.standard_normal(p // 4 + 1), 4)[:p],
        "cluster 1e-14": 1.0 + 1e-14 * rng.standard_normal(p),
        "graded": np.logspace(-15, 0, p),
        "converged Ritz window": np.concatenate([np.linspace(7.0, 7.1, p // 2),
                                                 1e-6 * rng.standard_normal(p - p // 2)]),
    }
    mats = {k: (Q * lam) @ Q.conj().T for k, lam in out.items()}
    mats["1D Laplacian"] = 2 * np.eye(p) - np.eye(p, k=1) - np.eye(p, k=-1)
    mats["Wilkinson"] = np.diag(np.abs(np.arange(p) - p // 2).astype(float)) + np.eye(p, k=1) + np.eye(p, k=-1)
    mats["ones"] = np.ones((p, p))
    mats["zero"] = np.zeros((p, p))
    return mats


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("p", [33, 130])
def test_host_eigh_structured_spectra(cplx, p):
    # sizes above 32 take divide and conquer: 33 one merge of two leaves, 130 two levels
    # of merges; each case against numpy and for orthogonality and residual
    for name, B in _structured_spectra(p, np.random.default_rng(p), cplx).items():
        w, U = afsi.afsi_host_eigh(B)
        wr = np.linalg.eigvalsh(B)
        scale = max(1e-300, np.max(np.abs(wr)))
        assert np.max(np.abs(w - wr)) <= 1e-13 * max(scale, 1.0) * max(1, p / 32), name
        assert np.max(np.abs(U.conj().T @ U - np.eye(p))) <= 1e-13 * max(1, p / 10), name
        assert np.max(np.abs(B @ U - U * w)) <= 1e-13 * max(scale, 1.0) * max(1, p / 32), name


@pytest.mark.parametrize("p", [40, 97, 256])
def test_host_eigh_closed_form_tridiagonal(p):
    # the 1D Dirichlet Laplacian tridiag(-1, 2, -1): eigenvalues 2 - 2 cos(j pi / (p+1)),
    # eigenvectors sin(i j pi / (p+1)) (distinct eigenvalues: unique up to sign); the
    # input is already tridiagonal, so this pins the divide and conquer step directly
    T = 2 * np.eye(p) - np.eye(p, k=1) - np.eye(p, k=-1)
    w, U = afsi.afsi_host_eigh(T)
    j = np.arange(1, p + 1)
    lam = 2 - 2 * np.cos(j * np.pi / (p + 1))
    V = np.sin(np.outer(j, j) * np.pi / (p + 1)) * np.sqrt(2 / (p + 1))
    assert np.max(np.abs(w - lam)) < 1e-14 * max(1, p / 32)
    assert np.max(np.abs(np.abs(np.sum(U * V, axis=0)) - 1)) < 1e-12


@pytest.mark.parametrize("cplx", [False, True])
def test_host_eigh_rejects_non_finite_input(cplx):
    B = np.eye(6, dtype=np.complex128 if cplx else np.float64)
    B[4, 1] = np.nan
    with pytest.raises(afsi.AfsiError) as e:
        afsi.afsi_host_eigh(B)
    assert e.value.status == -1 and "non-finite" in str(e.value)
    if cplx:
        B = np.eye(6, dtype=np.complex128)
        B[2, 3] = complex(0.0, np.inf)
        with pytest.raises(afsi.AfsiError):
            afsi.afsi_host_eigh(B)


@pytest.mark.parametrize("cplx", [False, True])
def test_host_cholesky_inverse(cplx):
    rng = np.random.default_rng(5)
    X = rng.standard_normal((300, 30)) * np.logspace(0, -6, 30)
    if cplx:
        X = X + 1j * rng.standard_normal((300, 30)) * np.logspace(0, -6, 30)
    G = X.conj().T @ X
    Ri = afsi.afsi_host_cholesky_inverse(G)
    assert np.allclose(np.tril(Ri, -1), 0)
    Q = X @ Ri
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(30))) < 1e-8
    with pytest.raises(afsi.AfsiError) as e:
        afsi.afsi_host_cholesky_inverse(np.diag([1.0, -1.0]))
    assert e.value.status == -4
    # a shift makes a singular Gram factorable
    S = np.ones((3, 3))
    Ri = afsi.afsi_host_cholesky_inverse(S, shift=1e-3)
    assert np.all(np.isfinite(Ri))


def test_invalid_csr_is_rejected_before_device_use():
    rp = np.array([0, 2, 3])
    with pytest.raises(afsi.AfsiError) as e:
        afsi.afsi_matrix_create_csr(0, 2, 3, rp, np.array([1, 0, 1]), np.ones(3), afsi.R64)  # unsorted
    assert e.value.status == -1
    with pytest.raises(afsi.AfsiError):
        afsi.afsi_matrix_create_csr(0, 2, 3, rp, np.array([0, 2, 1]), np.ones(3), afsi.R64)  # out of range
    with pytest.raises(afsi.AfsiError):
        afsi.afsi_matrix_create_csr(0, 2, 3, np.array([0, 2, 4]), np.array([0, 1, 1]), np.ones(3), afsi.R64)


def test_block_size_from_count():
    # Section 3.4: p = ceil(mu * e~), Section 4's mu = 1.8; clipped to [1, n]
    assert afsi.afsi_block_size(196.59, 1.8, 19683) == 354   # 353.862 rounds up
    assert afsi.afsi_block_size(200.0, 1.8, 10 ** 6) == 360  # exact product, no round-up
    assert afsi.afsi_block_size(40.7, 1.8, 4096) == 74
    assert afsi.afsi_block_size(-3.0, 1.8, 100) == 1
    assert afsi.afsi_block_size(0.0, 1.8, 100) == 1
    assert afsi.afsi_block_size(1e9, 1.8, 4096) == 4096
    for bad in ((10.0, 0.0, 100), (10.0, -1.0, 100), (float("nan"), 1.8, 100), (10.0, 1.8, 0)):
        with pytest.raises(afsi.AfsiError) as e:
            afsi.afsi_block_size(*bad)
        assert e.value.status == -1
