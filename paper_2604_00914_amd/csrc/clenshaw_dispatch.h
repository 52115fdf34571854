// Host-side choice of the Clenshaw-step kernel variant for one element type.
#pragma once

#include <algorithm>

#include "clenshaw_kernels.h"
#include "internal.h"

namespace afsi {

// XCD-aware grid: every XCD processes runs of `group` consecutive workgroups,
// about `run_rows` rows (default 4096), and the grid is padded to a multiple of 8 * group.
struct Grid {
    int group;
    int nblocks;
    int64_t grid;
};
inline Grid xcd_grid(int64_t n, int rows_per_block, int64_t run_rows = 4096) {
    Grid g;
    g.nblocks = (int)((n + rows_per_block - 1) / rows_per_block);
    int grp = std::max(1, (int)(run_rows / rows_per_block));
    const int per_xcd = (g.nblocks + 7) / 8;
    grp = std::min(grp, std::max(1, per_xcd));
    g.group = grp;
    g.grid = grp <= 1 ? g.nblocks : ((int64_t)g.nblocks + 8 * grp - 1) / (8 * grp) * (8 * grp);
    return g;
}

// Rows per XCD run for rows of row_bytes: a banded matrix whose entries reach `band`
// rows away (A.band, the median over rows) gets runs of band / 8 rows when three such
// runs of source rows fit one XCD's 4 MB L2, so that a row's +-band neighbours are
// processed by the same XCD 8 runs apart, while the rows between are still cached
// (FP32 rows of 1 KB on the 100^3 stencil: 814 -> 787 us per product; the 2 KB FP64 rows
// do not fit and keep 4096-row runs); otherwise 4096 rows.
inline int64_t run_rows_for(const MatView &A, int64_t row_bytes, int rows_per_block) {
    const int64_t r = A.band / 8 / rows_per_block * rows_per_block;
    if (r >= rows_per_block && r < 4096 && 3 * r * row_bytes <= (int64_t(4) << 20)) return r;
    return 4096;
}

template <class Tr, int VN, int L, bool HV, bool HX>
void launch_exact(const MatView &A, const void *src, const void *X, void *dst, int64_t ldv,
                  double sigma, double tau, double alpha, hipStream_t s) {
    using vec = typename Tr::vec;
    using scal = typename Tr::scal;
    constexpr int U = VN <= 4 ? 8 : 4;
    const Grid g = xcd_grid(A.n, 4 * (64 / L), run_rows_for(A, VN * L * 16, 4 * (64 / L)));
    if constexpr (VN <= 3 && L == 64) {
        if (A.stage_near) {
            hipLaunchKernelGGL((clenshaw_step_staged_kernel<Tr, VN, L, HV, HX, U>),
                               dim3((unsigned)g.grid), dim3(256), 0, s, (int)A.n, A.rp, A.ci,
                               (const typename Tr::val *)A.val, (const vec *)src, (const vec *)X,
                               (vec *)dst, ldv, (scal)sigma, (scal)tau, (scal)alpha, g.group,
                               g.nblocks);
            return;
        }
    }
    hipLaunchKernelGGL((clenshaw_step_kernel<Tr, VN, L, HV, HX, U>), dim3((unsigned)g.grid),
                       dim3(256), 0, s, (int)A.n, A.rp, A.ci, (const typename Tr::val *)A.val,
                       (const vec *)src, (const vec *)X, (vec *)dst, ldv, (scal)sigma, (scal)tau,
                       (scal)alpha, g.group, g.nblocks);
}

template <class Tr, int VN, bool HV, bool HX>
void launch_masked(const MatView &A, const void *src, const void *X, void *dst, int64_t ldv,
                   int p16, double sigma, double tau, double alpha, hipStream_t s) {
    using vec = typename Tr::vec;
    using scal = typename Tr::scal;
    constexpr int U = VN <= 2 ? 8 : 4;
    const Grid g = xcd_grid(A.n, 4);
    hipLaunchKernelGGL((clenshaw_step_masked_kernel<Tr, VN, HV, HX, U>), dim3((unsigned)g.grid),
                       dim3(256), 0, s, (int)A.n, A.rp, A.ci, (const typename Tr::val *)A.val,
                       (const vec *)src, (const vec *)X, (vec *)dst, ldv, p16, (scal)sigma,
                       (scal)tau, (scal)alpha, g.group, g.nblocks);
}

template <class Tr, bool HV, bool HX>
void dispatch_flags(const MatView &A, const void *src, const void *X, void *dst, int p16,
                    int64_t ldv, double sg, double ta, double al, hipStream_t s) {
    // exact fits, preferred order (where two fit, the first was measured faster on the
    // 100^3 stencil: 2 x 64 over 4 x 32 at 128 vectors, 2 x 32 over 1 x 64 at 64)
#define AFSI_EXACT(VN_, L_)                                                                         \
    if (p16 == (VN_) * (L_)) return launch_exact<Tr, VN_, L_, HV, HX>(A, src, X, dst, ldv, sg, ta, al, s)
    // with near-diagonal entries one row per wave takes the LDS-staged kernel, which at
    // 64 vectors per row (FP32 p = 256) beats two rows per wave: 810 against 847 us on
    // the 100^3 stencil
    if (A.stage_near) { AFSI_EXACT(1, 64); }
    AFSI_EXACT(2, 64); AFSI_EXACT(4, 32); AFSI_EXACT(4, 64); AFSI_EXACT(3, 64); AFSI_EXACT(5, 64);
    AFSI_EXACT(3, 32); AFSI_EXACT(5, 32); AFSI_EXACT(2, 32);
    AFSI_EXACT(6, 64); AFSI_EXACT(8, 64); AFSI_EXACT(1, 64); AFSI_EXACT(1, 32);
    AFSI_EXACT(3, 16); AFSI_EXACT(1, 16);
    AFSI_EXACT(3, 8);  // 24 vectors: the FP32 slice width p = 96
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

template <class Sr, int P>
void launch_narrow(const MatView &A, const void *src, const void *X, void *dst, int64_t ld,
                   bool hv, bool hx, double sg, double ta, double al, hipStream_t s) {
    using vec = typename Sr::vec;
    using scal = typename Sr::scal;
    constexpr int U = P <= 2 ? 8 : (P <= 4 ? 4 : 2);
    const Grid g = xcd_grid(A.n, 256);
    hipLaunchKernelGGL((clenshaw_step_narrow_kernel<Sr, P, U>), dim3((unsigned)g.grid), dim3(256), 0,
                       s, (int)A.n, A.rp, A.ci, (const typename Sr::val *)A.val, (const vec *)src,
                       (const vec *)X, (vec *)dst, ld, (int)hv, (int)hx, (scal)sg, (scal)ta,
                       (scal)al, g.group, g.nblocks);
}

template <class Sr>
void dispatch_narrow(const MatView &A, const void *src, const void *X, void *dst, int p,
                     int64_t ld, bool hv, bool hx, double sg, double ta, double al, hipStream_t s) {
    switch (p) {
#define AFSI_NARROW(P_)                                                                             \
    case P_: return launch_narrow<Sr, P_>(A, src, X, dst, ld, hv, hx, sg, ta, al, s);
    AFSI_NARROW(1) AFSI_NARROW(2) AFSI_NARROW(3) AFSI_NARROW(4) AFSI_NARROW(5) AFSI_NARROW(6)
    AFSI_NARROW(7) AFSI_NARROW(8) AFSI_NARROW(9) AFSI_NARROW(10) AFSI_NARROW(11) AFSI_NARROW(12)
    AFSI_NARROW(13) AFSI_NARROW(14) AFSI_NARROW(15) AFSI_NARROW(16)
#undef AFSI_NARROW
    }
}

template <class Sr>
void dispatch_scalar(const MatView &A, const void *src, const void *X, void *dst, int p,
                     int64_t ld, bool hv, bool hx, double sg, double ta, double al, hipStream_t s) {
    using vec = typename Sr::vec;
    using scal = typename Sr::scal;
    if (p <= kNarrowMax) return dispatch_narrow<Sr>(A, src, X, dst, p, ld, hv, hx, sg, ta, al, s);
    const Grid g = xcd_grid(A.n, 4);
    hipLaunchKernelGGL((clenshaw_step_scalar_kernel<Sr, 4, 4>), dim3((unsigned)g.grid), dim3(256), 0,
                       s, (int)A.n, A.rp, A.ci, (const typename Sr::val *)A.val, (const vec *)src,
                       (const vec *)X, (vec *)dst, ld, p, (int)hv, (int)hx, (scal)sg, (scal)ta,
                       (scal)al, g.group, g.nblocks);
}

}  // namespace afsi

#define AFSI_DEFINE_STEP_ENTRY(NAME, TR, SR)                                                        \
    namespace afsi {                                                                                \
    void NAME##_step(const MatView &A, const void *src, const void *X, void *dst, int p16,          \
                     int64_t ldv, bool hv, bool hx, double sg, double ta, double al,               \
                     hipStream_t s) {                                                               \
        dispatch_step<TR>(A, src, X, dst, p16, ldv, hv, hx, sg, ta, al, s);                         \
    }                                                                                               \
    void NAME##_scalar(const MatView &A, const void *src, const void *X, void *dst, int p,          \
                       int64_t ld, bool hv, bool hx, double sg, double ta, double al,              \
                       hipStream_t s) {                                                             \
        dispatch_scalar<SR>(A, src, X, dst, p, ld, hv, hx, sg, ta, al, s);                          \
    }                                                                                               \
    }
