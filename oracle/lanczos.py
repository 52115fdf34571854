"""Filtered thick-restart block Lanczos for the eigenpairs in [a, b].

Test infrastructure only.

The paper designs its filter for subspace iteration and notes that the same filter
suits thick-restart Lanczos (Section 3.1, and Section 5 names filtered Lanczos as the
next framework); it defines no such method.  This oracle states the method the
library builds, in plain steps:

* the operator is B = rho(A), the damped step filter of eq. (AdaPolySI) at a fixed
  degree, applied by the Clenshaw recurrence (Algorithm 2);  B has eigenvalues
  rho(lambda_i): close to one for lambda_i in [a, b] and close to zero away from it;
* a block Krylov basis V (s columns per block) is grown by V_{j+1} = orth((I - V V^H
  - L L^H) B V_j), projected out twice (full reorthogonalisation against the basis
  and the locked vectors L); W = B V is kept beside V;
* once V has m columns: H = V^H W (symmetrised), H = Y diag(theta) Y^H with theta
  descending; Ritz vectors U = V Y, and B U = W Y;
* a Ritz pair is *wanted* when theta >= eta = min(rho(a), rho(b)) (the filter's value
  at the interval's ends: eigenvalues inside [a, b] lie above it, those outside
  below, for the positive-kernel dampings);  its A-side Rayleigh quotient is
  lambda = u^H A u and its residual ||A u - lambda u||;
* wanted pairs with ||A u - lambda u|| < tau_c ||A|| are locked (deflated from the
  basis); those with lambda in [a, b] are results, the others are dropped;
* the cycle ends done when no wanted pair is left unlocked and the largest unlocked
  Ritz value, widened by its B-residual ||B u - theta u||, stays below eta (the
  remaining space has no eigenvalue of B above eta);
* otherwise the basis restarts thick: the unlocked Ritz vectors with the largest
  theta (n_keep = min(wanted unlocked + s, m / 2)) and, for the Krylov continuation,
  the next block orth((I - V V^H - L L^H) B V_last);  W follows by W Y for the kept
  vectors and one filter of the continuation block.

Readings (the paper is silent): block size s (a block finds eigenvalues of
multiplicity up to s, which a single vector does not), basis size m, threshold eta
and the stopping test above, the kept count, tau_c relative to ||A|| =
max(|lmin|, |lmax|) as in Algorithm 4, a cycle limit.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import coefficients as co
from . import native
from .filter import clenshaw_filter


@dataclass
class LanczosOptions:
    degree: int = 60
    damping: str = "jackson"
    m_exp: float = 0.5
    block: int = 4          # s
    basis: int = 128        # m
    tau_c: float = 1e-10
    max_cycles: int = 200


@dataclass
class LanczosResult:
    eigenvalues: np.ndarray
    eigenvectors: np.ndarray
    residuals: np.ndarray
    cycles: int
    filter_columns: int     # columns the filter was applied to (each: `degree` products)
    converged: bool
    locked_outside: int = 0
    history: list = field(default_factory=list)


def _project_out(Z, *bases):
    for _ in range(2):
        for Q in bases:
            if Q is not None and Q.shape[1]:
                Z = Z - Q @ (Q.conj().T @ Z)
    return Z


def _orth(Z):
    Q, _ = np.linalg.qr(Z, mode="reduced")
    return Q


def filtered_lanczos(A, a: float, b: float, lmin: float, lmax: float, V0: np.ndarray,
                     opts: LanczosOptions) -> LanczosResult:
    coeffs = co.filter_coefficients(lmin, lmax, a, b, opts.degree, opts.damping, opts.m_exp)
    l1, l2 = co.affine_map(lmin, lmax)
    eta = float(min(co.filter_value(a, coeffs, lmin, lmax), co.filter_value(b, coeffs, lmin, lmax)))
    tau_abs = opts.tau_c * max(abs(lmin), abs(lmax))
    s, m = opts.block, opts.basis
    cplx = np.iscomplexobj(V0) or np.iscomplexobj(A.val)
    dt = np.complex128 if cplx else np.float64

    def B(Z):
        return clenshaw_filter(A, Z, coeffs, l1, l2)

    L = np.zeros((A.n, 0), dtype=dt)
    lam_out, res_out = [], []
    outside = 0
    filtered = 0
    V = _orth(np.asarray(V0, dtype=dt))
    W = B(V)
    filtered += V.shape[1]
    history = []
    for cycle in range(1, opts.max_cycles + 1):
        # grow the block Krylov basis to m columns
        while V.shape[1] < m:
            Z = _orth(_project_out(W[:, -s:], V, L))
            V = np.concatenate([V, Z], axis=1)
            W = np.concatenate([W, B(Z)], axis=1)
            filtered += Z.shape[1]
        H = V.conj().T @ W
        H = 0.5 * (H + H.conj().T)
        theta, Y = np.linalg.eigh(H)
        order = np.argsort(-theta, kind="stable")
        theta, Y = theta[order], Y[:, order]
        U, BU = V @ Y, W @ Y
        rB = np.linalg.norm(BU - U * theta[None, :], axis=0)
        AU = native.spmm(A, U)
        lam = np.real(np.sum(U.conj() * AU, axis=0))
        rA = np.linalg.norm(AU - U * lam[None, :], axis=0)
        wanted = theta >= eta
        lock = wanted & (rA < tau_abs)
        for i in np.nonzero(lock)[0]:
            if a <= lam[i] <= b:
                lam_out.append(float(lam[i]))
                res_out.append(float(rA[i]))
            else:
                outside += 1
        L = np.concatenate([L, U[:, lock]], axis=1)
        free = np.nonzero(~lock)[0]
        n_want = int(np.sum(wanted & ~lock))
        top = free[0] if free.size else None
        history.append({"cycle": cycle, "locked": int(lock.sum()), "wanted_left": n_want,
                        "theta_top": float(theta[top]) if top is not None else None})
        if n_want == 0 and (top is None or theta[top] + rB[top] < eta):
            return _result(lam_out, res_out, L, cycle, filtered, True, outside, history, A, a, b)
        # thick restart: kept Ritz vectors plus the Krylov continuation block
        keep = free[: max(1, min(n_want + s, m // 2))]
        Z = _orth(_project_out(W[:, -s:], V, L))
        V = np.concatenate([U[:, keep], Z], axis=1)
        W = np.concatenate([BU[:, keep], B(Z)], axis=1)
        filtered += Z.shape[1]
    return _result(lam_out, res_out, L, opts.max_cycles, filtered, False, outside, history, A, a, b)


def _result(lam, res, L, cycles, filtered, converged, outside, history, A, a, b):
    lam = np.asarray(lam, dtype=np.float64)
    # the locked vectors in [a, b]: recompute their quotients to pick them out of L
    AL = native.spmm(A, L) if L.shape[1] else L
    q = np.real(np.sum(L.conj() * AL, axis=0)) if L.shape[1] else np.zeros(0)
    inside = np.nonzero((q >= a) & (q <= b))[0]
    Vin = L[:, inside]
    order = np.argsort(lam, kind="stable")
    vorder = np.argsort(q[inside], kind="stable")
    return LanczosResult(lam[order], Vin[:, vorder], np.asarray(res)[order] if len(res) else np.zeros(0),
                         cycles, filtered, converged, outside, history)
