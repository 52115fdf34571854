// Batched Clenshaw step for spectrum slices of one matrix (several filters advanced
// by one launch, the matrix read once).  Kept apart from the single-block kernels.
#pragma once

#include "clenshaw_dispatch.h"

namespace afsi {

// Each wave owns one (row, chunk) item: the chunk is 64 * VN consecutive 16-byte
// vectors of the concatenated row, lane `lane` owning vectors v * 64 + lane.  No
// wave loops over chunks, which keeps U * VN row gathers in flight per lane as in
// the single-block kernel; a row's nonzeros are read once per chunk (from cache).
// A vector belongs to the group whose [vec0, vec1) holds it; vectors outside every
// active group are left untouched (their products are computed and discarded, so
// that the gather loop is the same for every lane).  At least 4 waves per SIMD.
// SAME_SRC: every active group reads the same source block (the host checks), so the
// gathers use one wave-uniform base address instead of a per-lane pointer, which the
// address unit handles as a scalar base plus a 32-bit lane offset (16 slices x 96
// columns of the 100^3 matrix: 13.2 against 14.8 ms per step).
template <class Tr, int VN, int U, bool SAME_SRC>
__global__ __launch_bounds__(256, 4) void clenshaw_batched_kernel(
    int n, const int *__restrict__ rp, const int *__restrict__ ci,
    const typename Tr::val *__restrict__ va, const typename Tr::vec *__restrict__ X,
    typename Tr::vec *P0, typename Tr::vec *P1, int64_t ldv, int p16, int nchunks, int group,
    int nblocks, const BatchArgs args) {
    using vec = typename Tr::vec;
    using scal = typename Tr::scal;
    const int lb = xcd_block(blockIdx.x, group, nblocks);
    if (lb < 0) return;
    const int lane = threadIdx.x & 63;
    // items are column-chunk-major: the grid sweeps every row of one 64 * VN-vector
    // panel before the next, so the rows a banded matrix gathers again (up to its
    // bandwidth away) stay within the memory-side cache even for wide blocks
    const int64_t item = (int64_t)lb * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (item >= (int64_t)n * nchunks) return;
    const int row = __builtin_amdgcn_readfirstlane((int)(item % n));
    const int c0 = __builtin_amdgcn_readfirstlane((int)(item / n)) * 64 * VN;
    const int start = rp[row], end = rp[row + 1];
    // per vector: its group, its source block and a load index that is always a whole
    // vector inside the block (a vector outside every group is read at the first
    // vector of group 0 and its product discarded), so the gather loop has no
    // lane-dependent branches
    int grp[VN], vix[VN];
    const vec *sp[VN];
    int live = 0;
#pragma unroll
    for (int v = 0; v < VN; ++v) {
        const int vi = c0 + v * 64 + lane;
        grp[v] = -1;
        for (int g = 0; g < args.ngroups; ++g)
            if (vi >= args.vec0[g] && vi < args.vec1[g]) grp[v] = g;
        const int s = SAME_SRC ? args.src[0] : (grp[v] >= 0 ? args.src[grp[v]] : 0);
        sp[v] = s == 0 ? X : (s == 1 ? P0 : P1);
        vix[v] = grp[v] >= 0 ? vi : args.vec0[0];
        live |= (grp[v] >= 0) << v;
    }
    if (__ballot(live != 0) == 0) return;  // no lane of this wave has a live vector
    vec acc[VN];
#pragma unroll
    for (int v = 0; v < VN; ++v) acc[v] = Tr::zero();
    for (int e0 = start; e0 < end; e0 += U) {
        // the tail gathers the clamped entry with a zero coefficient, so that nothing
        // in the chunk is conditional and every gather is issued before the first
        // wait (16 slices x 96 columns of the 100^3 matrix: 11.9 ms per step, against
        // 13.2 ms with the multiply-add predicated and 13.7 ms with the tail gathers
        // skipped)
        int c[U];
        typename Tr::val a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = e0 + u < end;
            const int e = ok ? e0 + u : end - 1;
            c[u] = ci[e];
            a[u] = ok ? va[e] : Tr::val_zero();
        }
        vec w[U][VN];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int v = 0; v < VN; ++v) w[u][v] = sp[v][(int64_t)c[u] * ldv + vix[v]];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int v = 0; v < VN; ++v) acc[v] = Tr::fma_val(a[u], w[u][v], acc[v]);
    }
#pragma unroll
    for (int v = 0; v < VN; ++v) {
        if (live & (1 << v)) {
            const int g = grp[v];
            const int64_t idx = (int64_t)row * ldv + c0 + v * 64 + lane;
            vec *dp = args.dst[g] == 1 ? P0 : P1;
            vec r = clenshaw_combine<Tr>((scal)args.sigma[g], (scal)args.tau[g], acc[v], sp[v][idx]);
            if (args.has_v[g]) r = Tr::sub(r, nt_load(dp + idx));
            if (args.alpha[g] != 0.0) r = Tr::axpy((scal)args.alpha[g], nt_load(X + idx), r);
            nt_store(r, dp + idx);
        }
    }
}

template <class Tr, int VN, bool SAME_SRC>
void launch_batched(const MatView &A, const void *X, void *P0, void *P1, int p16, int64_t ldv,
                    const BatchArgs &args, hipStream_t s) {
    using vec = typename Tr::vec;
    const int nchunks = (p16 + 64 * VN - 1) / (64 * VN);
    const int64_t items = A.n * (int64_t)nchunks;
    AFSI_REQUIRE(items < (1LL << 31), "batched step: rows x column chunks too large");
    const Grid g = xcd_grid(items, 4);  // 4 items (waves) per workgroup
    hipLaunchKernelGGL((clenshaw_batched_kernel<Tr, VN, 8, SAME_SRC>), dim3((unsigned)g.grid),
                       dim3(256), 0, s, (int)A.n, A.rp, A.ci, (const typename Tr::val *)A.val,
                       (const vec *)X, (vec *)P0, (vec *)P1, ldv, p16, nchunks, g.group, g.nblocks,
                       args);
}

// 2 vectors per lane (2 KB chunks of an FP64 row): on 16 slices x 96 columns of the
// 100^3 matrix, 14.8 ms per step against 18.0 ms with 4 vectors per lane
template <class Tr>
void dispatch_batched(const MatView &A, const void *X, void *P0, void *P1, int p16, int64_t ldv,
                      const BatchArgs &args, hipStream_t s) {
    bool same = true;
    for (int g = 1; g < args.ngroups; ++g) same = same && args.src[g] == args.src[0];
    if (same) launch_batched<Tr, 2, true>(A, X, P0, P1, p16, ldv, args, s);
    else launch_batched<Tr, 2, false>(A, X, P0, P1, p16, ldv, args, s);
}

}  // namespace afsi

#define AFSI_DEFINE_BATCHED_ENTRY(NAME, TR)                                                         \
    namespace afsi {                                                                                \
    void NAME##_batched(const MatView &A, const void *X, void *P0, void *P1, int p16, int64_t ldv,  \
                        const BatchArgs &args, hipStream_t s) {                                     \
        dispatch_batched<TR>(A, X, P0, P1, p16, ldv, args, s);                                      \
    }                                                                                               \
    }
