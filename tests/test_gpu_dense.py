"""GPU parity of the FP64 dense steps (Gram/projection, block update, Cholesky QR,
Rayleigh-Ritz, residual norms, casts, gathers) through the C ABI."""
import numpy as np
import pytest

from oracle import dense as odense
from paper_2604_00914_amd import afsi
from tests.gpu_util import DEV, to_dev, torch
from workloads import build_config, random_dense_symmetric_csr, start_block, tight_binding_3d_periodic

pytestmark = pytest.mark.gpu


def _rand(n, p, cplx, seed):
    return start_block(n, p, seed=seed, complex_=cplx)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n,p,q", [(1, 1, 1), (5, 3, 7), (1001, 17, 70), (4096, 64, 64), (20000, 256, 256), (3000, 130, 5)])
def test_block_inner(n, p, q, cplx):
    t = torch()
    X, Y = _rand(n, p, cplx, 1), _rand(n, q, cplx, 2)
    G = t.empty((p, q), dtype=t.complex128 if cplx else t.float64, device=DEV)
    afsi.afsi_block_inner(to_dev(X), to_dev(Y), G)
    ref = X.conj().T @ Y
    got = G.cpu().numpy()
    scale = np.sqrt(n) * max(1.0, np.abs(ref).max())
    assert np.max(np.abs(got - ref)) <= 1e-14 * scale * 10


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n,p", [(1, 1), (7, 5), (1001, 70), (20000, 256), (3000, 300)])
def test_block_inner_same_block_is_exactly_hermitian(n, p, cplx):
    """X^H X through the symmetric path (one block passed twice): upper tiles only,
    lower triangle mirrored; must match X^H X and be exactly Hermitian."""
    t = torch()
    X = _rand(n, p, cplx, 11)
    Xd = to_dev(X)
    G = t.empty((p, p), dtype=t.complex128 if cplx else t.float64, device=DEV)
    afsi.afsi_block_inner(Xd, Xd, G)
    got = G.cpu().numpy()
    ref = X.conj().T @ X
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.sqrt(n) * max(1.0, np.abs(ref).max())
    assert np.array_equal(got, got.conj().T)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n,p,q,beta", [(1, 1, 1, 0.0), (1001, 17, 70, 0.0), (5000, 64, 64, 1.0), (3000, 256, 250, -0.5)])
def test_block_gemm(n, p, q, beta, cplx):
    t = torch()
    X, Mh, Y0 = _rand(n, p, cplx, 3), _rand(p, q, cplx, 4), _rand(n, q, cplx, 5)
    Y = to_dev(Y0)
    afsi.afsi_block_gemm(to_dev(X), to_dev(Mh), beta, Y)
    ref = X @ Mh + beta * Y0
    assert np.max(np.abs(Y.cpu().numpy() - ref)) <= 1e-13 * np.sqrt(p) * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("p", [48, 200, 300])
def test_orthonormalize_with_locked(cplx, p):
    """p > 128 spans several column tiles of the triangular X R^{-1} product."""
    t = torch()
    n, k = 3000, 10
    L, _ = np.linalg.qr(_rand(n, k, cplx, 6))
    X0 = _rand(n, p, cplx, 7)
    X = to_dev(X0)
    W = t.empty_like(X)
    afsi.afsi_orthonormalize(to_dev(L), X, W)
    Q = X.cpu().numpy()
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(p))) < 1e-13
    assert np.max(np.abs(L.conj().T @ Q)) < 1e-13
    # same span as the oracle's Householder result
    Qo = odense.orthonormalize(X0, L)
    assert np.linalg.norm(Q - Qo @ (Qo.conj().T @ Q)) < 1e-11


def test_orthonormalize_ill_conditioned_uses_shift():
    t = torch()
    n, p = 4000, 32
    X0 = _rand(n, p, False, 8)
    X0[:, -1] = X0[:, 0] + 1e-14 * X0[:, 1]  # numerically rank deficient
    X = to_dev(X0)
    W = t.empty_like(X)
    afsi.afsi_orthonormalize(None, X, W)
    Q = X.cpu().numpy()
    assert np.all(np.isfinite(Q))
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(p))) < 1e-10


@pytest.mark.parametrize("name", ["lap2d_64", "tb3d_64"])
def test_rayleigh_ritz_matches_oracle(name):
    t = torch()
    size = 64 if name == "lap2d_64" else 10
    A, (lmin, lmax), _, cfg = build_config(name, size=size)
    cplx = A.is_complex
    Q0, _ = np.linalg.qr(_rand(A.n, 40, cplx, 9))
    M = afsi.Matrix(A, bounds=(lmin, lmax))
    Q = to_dev(Q0)
    V, AV = t.empty_like(Q), t.empty_like(Q)
    ritz = afsi.afsi_rayleigh_ritz(M.handle, Q, V, AV)
    w, Vo, AVo = odense.rayleigh_ritz(A, Q0)
    assert np.max(np.abs(ritz - w)) < 1e-12 * max(abs(lmin), abs(lmax))
    Vg, AVg = V.cpu().numpy(), AV.cpu().numpy()
    assert np.max(np.abs(Vg.conj().T @ Vg - np.eye(40))) < 1e-12
    assert np.max(np.abs(A.to_scipy() @ Vg - AVg)) < 1e-12
    res = afsi.afsi_residual_norms(V, AV, ritz)
    assert np.max(np.abs(res - odense.residual_norms(Vg, AVg, ritz))) < 1e-12
    M.close()


@pytest.mark.parametrize("graded", [False, True])
@pytest.mark.parametrize("name", ["lap2d_64", "tb3d_64"])
def test_orthonormalize_rayleigh_ritz_matches_oracle(name, graded):
    # the fused call (the basis Q of Cholesky QR left implicit) against the oracle's
    # Householder QR followed by its Rayleigh-Ritz, on a raw (not orthonormal) block;
    # graded columns (norms 1 .. 1e-6) make the first Cholesky pass visibly inexact
    t = torch()
    size = 64 if name == "lap2d_64" else 10
    A, (lmin, lmax), _, cfg = build_config(name, size=size)
    cplx = A.is_complex
    p = 40
    X0 = _rand(A.n, p, cplx, 11)
    if graded:
        X0 = X0 * np.logspace(0, -6, p)[None, :]
    normA = max(abs(lmin), abs(lmax))
    w, Vo, AVo = odense.rayleigh_ritz(A, odense.orthonormalize(X0))
    M = afsi.Matrix(A, bounds=(lmin, lmax))
    X = to_dev(X0)
    W, V = t.empty_like(X), t.empty_like(X)
    ritz = afsi.afsi_orthonormalize_rayleigh_ritz(M.handle, X, W, V, W)   # AV in the work block
    assert np.max(np.abs(ritz - w)) < 1e-12 * normA
    Vg, AVg = V.cpu().numpy(), W.cpu().numpy()
    assert np.max(np.abs(Vg.conj().T @ Vg - np.eye(p))) < 1e-12
    assert np.max(np.abs(A.to_scipy() @ Vg - AVg)) < 1e-12 * normA
    # same Ritz vectors (up to a unit factor) where the Ritz values are apart
    gap = np.minimum(np.r_[np.inf, np.diff(w)], np.r_[np.diff(w), np.inf])
    sep = gap > 1e-6 * normA
    assert np.all(np.abs(np.abs(np.sum(Vo.conj() * Vg, axis=0))[sep] - 1) < 1e-8)
    M.close()


def test_orthonormalize_rayleigh_ritz_rejects_overlap():
    t = torch()
    A, (lmin, lmax), _, cfg = build_config("lap2d_64", size=16)
    M = afsi.Matrix(A, bounds=(lmin, lmax))
    X = to_dev(_rand(A.n, 8, False, 1))
    W = t.empty_like(X)
    with pytest.raises(afsi.AfsiError):
        afsi.afsi_orthonormalize_rayleigh_ritz(M.handle, X, W, W, X)   # V on the work block
    M.close()


def test_convert_and_gather():
    t = torch()
    X0 = _rand(777, 13, True, 10)
    X = to_dev(X0)
    X32 = t.empty((777, 13), dtype=t.complex64, device=DEV)
    afsi.afsi_convert_block(X, X32)
    assert np.array_equal(X32.cpu().numpy(), X0.astype(np.complex64))
    back = t.empty_like(X)
    afsi.afsi_convert_block(X32, back)
    assert np.array_equal(back.cpu().numpy(), X0.astype(np.complex64).astype(np.complex128))
    cols = [12, 0, 5, 5]
    G = t.empty((777, 4), dtype=t.complex128, device=DEV)
    afsi.afsi_gather_columns(X, cols, G)
    assert np.array_equal(G.cpu().numpy(), X0[:, cols])
