"""Adaptive filtered subspace iteration with locking (Algorithm 4).

Test infrastructure only.

Per iteration i:
  1. X_hat = rho_{k^(i),k}(A) V_hat            (filter, Algorithm 2, eq. (AdaPolySI))
  2. Q = X_hat orthonormalised against the locked V      (orth step)
  3. (V_hat, Lambda_hat) = Rayleigh-Ritz(A, Q)
  4. I = {j : Lambda_hat_jj in [a, b]}, e = |I|; if e = 0 go on to i + 1
  5. k^(i+1) by Algorithm 3 (adaptive mode only)
  6. residuals ||r_j|| for j in I
  7. tau_s = min_{j in I} dist(lambda_hat_j, {a, b})                  eq. (tau_s)
  8. C = {j in I : ||r_j|| < tau_s};  n_check = |C| + n_lock;
     if n_check > 0 and n_check equals the previous n_check: I = C
  9. L = {j in I : ||r_j|| < tau_c ||A||}; lock L, drop it from V_hat
 10. stop when I \\ L is empty.

Readings (the paper is silent or ambiguous):
* the locking test is relative, ||r|| < tau_c ||A|| with ||A|| = max(|lmin|, |lmax|),
  matching the convergence criterion of Section 4;
* the columns kept after orth([V, X_hat]) are those of X_hat made orthogonal to
  the locked V (keeping the first p - n_lock columns would keep V itself);
* the previous n_check starts at 0 and is left unchanged by iterations with e = 0;
* an iteration limit is added (the printed loop has none); reaching it returns
  the locked pairs found so far with converged = False.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import coefficients as co
from . import dense
from .degree import select_degree
from .filter import clenshaw_filter


@dataclass
class Options:
    kmax: int = 60
    damping: str = "jackson"
    m_exp: float = 0.5
    adaptive: bool = False
    k_init: int | None = None   # default: kmax (fixed) or eq. (compute_k_1) (adaptive)
    tau_a: float = 1e-3
    tau_c: float = 1e-10
    C: float = 1.4
    max_iter: int = 200


@dataclass
class Result:
    eigenvalues: np.ndarray
    eigenvectors: np.ndarray
    residuals: np.ndarray
    iterations: int
    spmv: int
    degrees: list = field(default_factory=list)
    converged: bool = True

    @property
    def avg_degree(self) -> float:
        return float(np.mean(self.degrees)) if self.degrees else 0.0


@dataclass
class ControlState:
    n_lock: int = 0
    n_check_prev: int = 0


def control_step(ritz: np.ndarray, res_I: np.ndarray, I: np.ndarray, a: float, b: float,
                 tau_c_abs: float, state: ControlState):
    """Steps 7-10 above on one iteration's Ritz values.

    ``I`` holds indices into ``ritz`` (all inside [a, b], non-empty); ``res_I`` the
    residual norms in the same order.  Returns (I_final, L, done) as index arrays
    into ``ritz`` and updates ``state.n_check_prev`` (``state.n_lock`` is updated by
    the caller after locking).
    """
    I = np.asarray(I, dtype=np.int64)
    res = dict(zip(I.tolist(), np.asarray(res_I, dtype=np.float64).tolist()))
    tau_s = min(min(abs(ritz[j] - a), abs(ritz[j] - b)) for j in I)
    C = np.array([j for j in I if res[j] < tau_s], dtype=np.int64)
    n_check = len(C) + state.n_lock
    if n_check > 0 and n_check == state.n_check_prev:
        I = C
    state.n_check_prev = n_check
    L = np.array([j for j in I if res[j] < tau_c_abs], dtype=np.int64)
    done = len(set(I.tolist()) - set(L.tolist())) == 0
    return I, L, done


def solve(A, a: float, b: float, lmin: float, lmax: float, X0: np.ndarray, opts: Options) -> Result:
    l1, l2 = co.affine_map(lmin, lmax)
    coeffs = co.filter_coefficients(lmin, lmax, a, b, opts.kmax, opts.damping, opts.m_exp)
    if opts.k_init is not None:
        k_cur = opts.k_init
    elif opts.adaptive:
        alpha, beta = co.interval_angles(a, b, lmin, lmax)
        k_cur = min(max(1, co.initial_degree(alpha, beta, opts.C)), opts.kmax)
    else:
        k_cur = opts.kmax
    normA = max(abs(lmin), abs(lmax))
    tau_abs = opts.tau_c * normA

    Vh = dense.orthonormalize(X0)
    cplx = np.iscomplexobj(X0) or np.iscomplexobj(A.val)
    lam_locked: list = []
    res_locked: list = []
    V_locked = np.zeros((A.n, 0), dtype=np.complex128 if cplx else np.float64)
    state = ControlState()
    spmv = 0
    degrees = []
    for it in range(1, opts.max_iter + 1):
        Xh = clenshaw_filter(A, Vh, coeffs, l1, l2, k_cur)
        spmv += k_cur * Vh.shape[1]
        degrees.append(k_cur)
        Q = dense.orthonormalize(Xh, V_locked)
        w, V, AV = dense.rayleigh_ritz(A, Q)
        spmv += Q.shape[1]
        I = np.nonzero((w >= a) & (w <= b))[0]
        Vh = V
        if I.size == 0:
            continue
        if opts.adaptive:
            k_cur = select_degree(w, I.size, coeffs, l1, l2, opts.tau_a)
        res_I = dense.residual_norms(V[:, I], AV[:, I], w[I])
        res_all = dict(zip(I.tolist(), res_I.tolist()))
        I_fin, L, done = control_step(w, res_I, I, a, b, tau_abs, state)
        if L.size:
            lam_locked.extend(w[L].tolist())
            res_locked.extend(res_all[j] for j in L.tolist())
            V_locked = np.concatenate([V_locked, V[:, L]], axis=1)
            keep = np.setdiff1d(np.arange(V.shape[1]), L)
            Vh = V[:, keep]
            state.n_lock += L.size
        if done:
            return _result(lam_locked, V_locked, res_locked, it, spmv, degrees, True)
    return _result(lam_locked, V_locked, res_locked, opts.max_iter, spmv, degrees, False)


def _result(lams, V, res, it, spmv, degrees, converged):
    lams = np.asarray(lams, dtype=np.float64)
    order = np.argsort(lams, kind="stable")
    return Result(lams[order], V[:, order], np.asarray(res)[order] if len(res) else np.zeros(0),
                  it, spmv, degrees, converged)
