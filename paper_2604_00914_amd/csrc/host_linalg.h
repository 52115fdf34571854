// Host dense Hermitian linear algebra (FP64), independent of HIP.
#pragma once

#include <cstdint>

namespace afsi {

// Overwrite G (p x p Hermitian, row-major, ld) with R^{-1}, where R^H R = G + shift I
// and R is upper triangular (strictly lower part set to zero).  The factorisation
// runs on the unit-diagonal scaling D (G + shift I) D.  Returns false, with G
// unchanged, on a non-positive or non-finite pivot.
bool host_cholesky_inverse(int64_t p, bool cplx, double *G, int64_t ld, double shift);

// B (p x p Hermitian, row-major, ldb) = U diag(w) U^H with w ascending and U unitary
// (row-major, ldu).  Returns false if the tridiagonal eigensolver does not converge.
bool host_eigh(int64_t p, bool cplx, const double *B, int64_t ldb, double *w, double *U,
               int64_t ldu);

}  // namespace afsi
