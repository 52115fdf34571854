"""Spectral interval estimate by a few Lanczos steps (Section 3.4, setup phase).

Test infrastructure only.  The paper says only that lambda_min and lambda_max
are estimated with "a few" Lanczos iterations.  Reading used here: k_L steps
with full reorthogonalisation from a seeded start vector; the extreme Ritz
values of the tridiagonal T are widened by the Ritz-pair residual bound
|beta_k s_k| (last eigenvector component times the last beta) plus a relative
margin, so that the returned interval encloses the spectrum in practice.
"""
from __future__ import annotations

import numpy as np

from . import native


def lanczos_bounds(A, steps: int = 40, seed: int = 0, margin: float = 1e-3):
    n = A.n
    steps = min(steps, n)
    rng = np.random.default_rng(seed)
    cplx = np.iscomplexobj(A.val)
    q = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
    q = q / np.linalg.norm(q)
    Qs = [q]
    alphas, betas = [], []
    beta = 0.0
    for j in range(steps):
        w = native.spmm(A, Qs[-1])
        alpha = float(np.real(np.vdot(Qs[-1], w)))
        w = w - alpha * Qs[-1] - (beta * Qs[-2] if j > 0 else 0)
        Qm = np.stack(Qs, axis=1)
        for _ in range(2):
            w = w - Qm @ (Qm.conj().T @ w)
        alphas.append(alpha)
        beta = float(np.linalg.norm(w))
        if j == steps - 1 or beta == 0.0:
            break
        betas.append(beta)
        Qs.append(w / beta)
    T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
    th, S = np.linalg.eigh(T)
    r_lo = abs(beta * S[-1, 0])
    r_hi = abs(beta * S[-1, -1])
    span = th[-1] - th[0]
    return th[0] - r_lo - margin * span, th[-1] + r_hi + margin * span
