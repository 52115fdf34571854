// Run-time choice between the generic and the AVX2/FMA builds of host_linalg.cpp.
#include "host_linalg.h"

namespace afsi {
namespace generic {
bool host_cholesky_inverse(int64_t p, bool cplx, double *G, int64_t ld, double shift);
bool host_eigh(int64_t p, bool cplx, const double *B, int64_t ldb, double *w, double *U, int64_t ldu);
}  // namespace generic
namespace avx2 {
bool host_cholesky_inverse(int64_t p, bool cplx, double *G, int64_t ld, double shift);
bool host_eigh(int64_t p, bool cplx, const double *B, int64_t ldb, double *w, double *U, int64_t ldu);
}  // namespace avx2

static bool cpu_has_avx2() {
    static const bool v = __builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma");
    return v;
}

bool host_cholesky_inverse(int64_t p, bool cplx, double *G, int64_t ld, double shift) {
    return cpu_has_avx2() ? avx2::host_cholesky_inverse(p, cplx, G, ld, shift)
                          : generic::host_cholesky_inverse(p, cplx, G, ld, shift);
}

bool host_eigh(int64_t p, bool cplx, const double *B, int64_t ldb, double *w, double *U,
               int64_t ldu) {
    return cpu_has_avx2() ? avx2::host_eigh(p, cplx, B, ldb, w, U, ldu)
                          : generic::host_eigh(p, cplx, B, ldb, w, U, ldu);
}

}  // namespace afsi
