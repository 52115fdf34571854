"""CPU oracle for adaptive Chebyshev-filtered subspace iteration.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, independently
written reference that the HIP library is checked against.  Only the test
suite, the package smoke check and the benchmark's CPU-baseline leg may
import it; the library itself never does, and the two share no code.

Everything is float64 / complex128.  Each function cites the passage of
"Adaptive Polynomial Filtering for Hermitian Interior Eigenproblems:
Convergence Analysis" (Xu, Ni, Li, Zhang) that it follows.

Modules
-------
coefficients  affine map l(x), step-function Chebyshev coefficients, damping
theory        J(theta), C_m and the pointwise error bounds (Section 3.2)
native        plain C CSR sparse x dense-block product (OpenMP over rows)
filter        Clenshaw evaluation of rho(l(A)) X and the forward recurrence
dense         orthonormalisation, Rayleigh-Ritz, residual norms
degree        initial degree rule and adaptive degree selection
solver        the full adaptive filtered subspace iteration with locking
closed_form   grid-Laplacian spectra (definition-level results)
spectra       eigenvalues of a banded real symmetric matrix inside an interval
bounds        Lanczos estimate of the spectral interval
eigencount    eigenvalue count in [a, b] by trace estimation of the filter
"""
