// Host-side choice of the Clenshaw-step kernel variant for one element type.
#pragma once

#include "clenshaw_kernels.h"
#include "internal.h"

namespace afsi {

template <class Tr, int VN, int L, bool HV, bool HX>
void launch_exact(const MatView &A, const void *src, const void *X, void *dst, int64_t ldv,
                  double sigma, double tau, double alpha, hipStream_t s) {
    using vec = typename Tr::vec;
    using scal = typename Tr::scal;
    constexpr int U = VN <= 2 ? 8 : (VN <= 4 ? 4 : 2);
    constexpr int rows_per_block = 4 * (64 / L);
    const int64_t grid = (A.n + rows_per_block - 1) / rows_per_block;
    hipLaunchKernelGGL((clenshaw_step_kernel<Tr, VN, L, HV, HX, U>), dim3((unsigned)grid), dim3(256),
                       0, s, (int)A.n, A.rp, A.ci, (const typename Tr::val *)A.val,
                       (const vec *)src, (const vec *)X, (vec *)dst, ldv, (scal)sigma, (scal)tau,
                       (scal)alpha);
}

template <class Tr, int VN, bool HV, bool HX>
void launch_masked(const MatView &A, const void *src, const void *X, void *dst, int64_t ldv,
                   int p16, double sigma, double tau, double alpha, hipStream_t s) {
    using vec = typename Tr::vec;
    using scal = typename Tr::scal;
    constexpr int U = VN <= 2 ? 8 : 4;
    const int64_t grid = (A.n + 3) / 4;
    hipLaunchKernelGGL((clenshaw_step_masked_kernel<Tr, VN, HV, HX, U>), dim3((unsigned)grid),
                       dim3(256), 0, s, (int)A.n, A.rp, A.ci, (const typename Tr::val *)A.val,
                       (const vec *)src, (const vec *)X, (vec *)dst, ldv, p16, (scal)sigma,
                       (scal)tau, (scal)alpha);
}

template <class Tr, bool HV, bool HX>
void dispatch_flags(const MatView &A, const void *src, const void *X, void *dst, int p16,
                    int64_t ldv, double sg, double ta, double al, hipStream_t s) {
#define AFSI_EXACT(VN_, L_)                                                                         \
    if (p16 == (VN_) * (L_)) return launch_exact<Tr, VN_, L_, HV, HX>(A, src, X, dst, ldv, sg, ta, al, s)
    AFSI_EXACT(1, 64); AFSI_EXACT(2, 64); AFSI_EXACT(3, 64); AFSI_EXACT(4, 64);
    AFSI_EXACT(5, 64); AFSI_EXACT(6, 64); AFSI_EXACT(8, 64);
    AFSI_EXACT(1, 32); AFSI_EXACT(3, 32); AFSI_EXACT(5, 32);
    AFSI_EXACT(1, 16); AFSI_EXACT(3, 16);
#undef AFSI_EXACT
    if (p16 <= 64) return launch_masked<Tr, 1, HV, HX>(A, src, X, dst, ldv, p16, sg, ta, al, s);
    if (p16 <= 128) return launch_masked<Tr, 2, HV, HX>(A, src, X, dst, ldv, p16, sg, ta, al, s);
    return launch_masked<Tr, 4, HV, HX>(A, src, X, dst, ldv, p16, sg, ta, al, s);
}

template <class Tr>
void dispatch_step(const MatView &A, const void *src, const void *X, void *dst, int p16,
                   int64_t ldv, bool has_v, bool has_x, double sg, double ta, double al,
                   hipStream_t s) {
    if (has_v) {
        if (has_x) dispatch_flags<Tr, true, true>(A, src, X, dst, p16, ldv, sg, ta, al, s);
        else dispatch_flags<Tr, true, false>(A, src, X, dst, p16, ldv, sg, ta, al, s);
    } else {
        if (has_x) dispatch_flags<Tr, false, true>(A, src, X, dst, p16, ldv, sg, ta, al, s);
        else dispatch_flags<Tr, false, false>(A, src, X, dst, p16, ldv, sg, ta, al, s);
    }
}

template <class Tr>
void dispatch_batched(const MatView &A, const void *X, void *P0, void *P1, int p16, int64_t ldv,
                      const BatchArgs &args, hipStream_t s) {
    using vec = typename Tr::vec;
    const int64_t grid = (A.n + 3) / 4;
    if (p16 <= 128) {
        hipLaunchKernelGGL((clenshaw_batched_kernel<Tr, 2, 4>), dim3((unsigned)grid), dim3(256), 0, s,
                           (int)A.n, A.rp, A.ci, (const typename Tr::val *)A.val, (const vec *)X,
                           (vec *)P0, (vec *)P1, ldv, p16, args);
    } else {
        hipLaunchKernelGGL((clenshaw_batched_kernel<Tr, 4, 4>), dim3((unsigned)grid), dim3(256), 0, s,
                           (int)A.n, A.rp, A.ci, (const typename Tr::val *)A.val, (const vec *)X,
                           (vec *)P0, (vec *)P1, ldv, p16, args);
    }
}

template <class Sr>
void dispatch_scalar(const MatView &A, const void *src, const void *X, void *dst, int p,
                     int64_t ld, bool hv, bool hx, double sg, double ta, double al, hipStream_t s) {
    using vec = typename Sr::vec;
    using scal = typename Sr::scal;
    const int64_t grid = (A.n + 3) / 4;
    hipLaunchKernelGGL((clenshaw_step_scalar_kernel<Sr, 4, 4>), dim3((unsigned)grid), dim3(256), 0, s,
                       (int)A.n, A.rp, A.ci, (const typename Sr::val *)A.val, (const vec *)src,
                       (const vec *)X, (vec *)dst, ld, p, (int)hv, (int)hx, (scal)sg, (scal)ta,
                       (scal)al);
}

}  // namespace afsi

#define AFSI_DEFINE_STEP_ENTRY(NAME, TR, SR)                                                            \
    namespace afsi {                                                                                \
    void NAME##_step(const MatView &A, const void *src, const void *X, void *dst, int p16,          \
                     int64_t ldv, bool hv, bool hx, double sg, double ta, double al,               \
                     hipStream_t s) {                                                               \
        dispatch_step<TR>(A, src, X, dst, p16, ldv, hv, hx, sg, ta, al, s);                         \
    }                                                                                               \
    void NAME##_batched(const MatView &A, const void *X, void *P0, void *P1, int p16, int64_t ldv,  \
                        const BatchArgs &args, hipStream_t s) {                                     \
        dispatch_batched<TR>(A, X, P0, P1, p16, ldv, args, s);                                      \
    }                                                                                               \
    void NAME##_scalar(const MatView &A, const void *src, const void *X, void *dst, int p,          \
                       int64_t ld, bool hv, bool hx, double sg, double ta, double al,              \
                       hipStream_t s) {                                                             \
        dispatch_scalar<SR>(A, src, X, dst, p, ld, hv, hx, sg, ta, al, s);                          \
    }                                                                                               \
    }
