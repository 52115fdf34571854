// Fused Clenshaw step over a CSR matrix and row-major dense blocks (gfx950).
//
// One product of Clenshaw's recurrence (Algorithm 2, division-free form):
//
//     dst[i, :] = sigma * sum_e A[i, col_e] * src[col_e, :] + tau * src[i, :]
//                 - dst[i, :]            (HAS_V: the block b_{j+2}, read in place)
//                 + alpha * X[i, :]      (HAS_X)
//
// Mapping: a group of L lanes owns one row; the row's p columns are split into
// 16-byte vectors and lane `sub` of the group owns vectors v*L + sub, v < VN, so
// each load instruction of the group reads L*16 contiguous bytes of a row.  The
// row's (column, value) pairs are the same for every lane of the group (scalar
// registers when L = 64).  U nonzeros are fetched together so that U*VN row
// gathers are in flight per lane; in the tail of a row the index is clamped (never
// reading past the row) and the entry contributes nothing (gather_accumulate says
// how, per lane mapping).
// MASKED variants use L = 64 and loop over chunks of 64*VN vectors with a bounds
// test, for any width.
//
// Memory behaviour (the kernel is HBM-bound):
//  * src rows are gathered through the caches (each is reused by every row that
//    references it); dst, the in-place b_{j+2} and X are streamed with
//    non-temporal accesses so that they do not evict those rows.
//  * Workgroups are dispatched round-robin over the 8 XCDs, each with its own
//    L2.  xcd_block() renumbers them so that every XCD works on a contiguous run
//    of `group` workgroups (a few thousand rows) while all XCDs advance through
//    the matrix together: neighbouring rows share an L2, and the far neighbours of
//    a banded matrix are still in the shared memory-side cache when reused.
//  * With one row per wave the in-place b_{j+2} and X are loaded after the
//    gathers: issuing them before the row's CSR entries (kept there by a compiler
//    barrier) needs 96 VGPRs at 2 vectors per lane, 5 waves per SIMD instead of 8,
//    and measured 2.5% slower on the 100^3 stencil.  With several rows per wave and
//    at most 3 vectors per lane they are issued before the CSR entries.
#pragma once

#include "vec_types.h"

namespace afsi {

// Logical workgroup index for hardware index b, or -1 for padding workgroups.
// The grid is a multiple of 8 * group; hardware workgroup b runs on XCD b % 8.
__device__ inline int xcd_block(int b, int group, int nblocks) {
    if (group <= 1) return b < nblocks ? b : -1;
    const int x = b & 7, slot = b >> 3;
    const int lb = ((slot / group) * 8 + x) * group + slot % group;
    return lb < nblocks ? lb : -1;
}

// WAVE_ROW: every lane of the wave works on the same row (L = 64), so the tail
// test is wave-uniform.  Then a tail gather is skipped by a uniform branch and its
// vector left at zero, while the multiply-adds stay unconditional; predicating the
// multiply-add instead lets the compiler move each gather into that branch, next to
// its wait, and only one nonzero's gathers are in flight at a time.  With several
// rows per wave (L < 64) the tail test differs between lanes, the gathers are
// issued together under the execution mask either way, and the predicated
// multiply-add is the faster form.
template <class Tr, int VN, int U, bool WAVE_ROW>
__device__ inline void gather_accumulate(int start, int end, const int *__restrict__ ci,
                                         const typename Tr::val *__restrict__ va,
                                         const typename Tr::vec *__restrict__ src, int64_t ldv,
                                         int64_t off, int stride, int nvalid,
                                         typename Tr::vec (&acc)[VN]) {
    using vec = typename Tr::vec;
    using val = typename Tr::val;
    for (int e0 = start; e0 < end; e0 += U) {
        int c[U];
        val a[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ok[u] = e0 + u < end;
            const int e = ok[u] ? e0 + u : end - 1;
            c[u] = ci[e];
            a[u] = va[e];
        }
        vec w[U][VN];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const vec *rowp = src + (int64_t)c[u] * ldv + off;
#pragma unroll
            for (int v = 0; v < VN; ++v) {
                if (WAVE_ROW) {
                    w[u][v] = Tr::zero();
                    if (ok[u] && v < nvalid) w[u][v] = rowp[v * stride];
                } else if (v < nvalid) {
                    w[u][v] = rowp[v * stride];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (WAVE_ROW || ok[u]) {
#pragma unroll
                for (int v = 0; v < VN; ++v)
                    if (v < nvalid) acc[v] = Tr::fma_val(a[u], w[u][v], acc[v]);
            }
        }
    }
}

template <class Tr, int VN, int L, bool HAS_V, bool HAS_X, int U>
__global__ __launch_bounds__(256) void clenshaw_step_kernel(
    int n, const int *__restrict__ rp, const int *__restrict__ ci,
    const typename Tr::val *__restrict__ va, const typename Tr::vec *__restrict__ src,
    const typename Tr::vec *__restrict__ X, typename Tr::vec *dst, int64_t ldv,
    typename Tr::scal sigma, typename Tr::scal tau, typename Tr::scal alpha, int group,
    int nblocks) {
    using vec = typename Tr::vec;
    constexpr int RW = 64 / L;
    const int lb = xcd_block(blockIdx.x, group, nblocks);
    if (lb < 0) return;
    const int lane = threadIdx.x & 63;
    const int sub = lane % L;
    int row = (lb * (int)(blockDim.x / 64) + (int)(threadIdx.x >> 6)) * RW + lane / L;
    if (L == 64) row = __builtin_amdgcn_readfirstlane(row);
    if (row >= n) return;
    constexpr bool EARLY = L < 64 && VN <= 3;
    const int64_t base = (int64_t)row * ldv + sub;
    vec vin[VN], xin[VN];
    if (EARLY) {
#pragma unroll
        for (int v = 0; v < VN; ++v) {
            if (HAS_V) vin[v] = nt_load(dst + base + v * L);
            if (HAS_X) xin[v] = nt_load(X + base + v * L);
        }
    }
    const int start = rp[row], end = rp[row + 1];
    vec acc[VN];
#pragma unroll
    for (int v = 0; v < VN; ++v) acc[v] = Tr::zero();
    gather_accumulate<Tr, VN, U, L == 64>(start, end, ci, va, src, ldv, sub, L, VN, acc);
#pragma unroll
    for (int v = 0; v < VN; ++v) {
        const int64_t idx = base + v * L;
        vec r = clenshaw_combine<Tr>(sigma, tau, acc[v], src[idx]);
        if (HAS_V) r = Tr::sub(r, EARLY ? vin[v] : nt_load(dst + idx));
        if (HAS_X) r = Tr::axpy(alpha, EARLY ? xin[v] : nt_load(X + idx), r);
        nt_store(r, dst + idx);
    }
}

// Rows of the source block staged in LDS.  A workgroup's 4 * (64 / L) rows are
// consecutive (the row mapping of clenshaw_step_kernel), so src rows r0 - 1 .. r0 + TR
// are copied to LDS once and every entry whose column falls among them, and the
// tau * src_i term, read LDS instead of gathering through L1/L2.  The stencil's
// diagonal and +-1 entries (3 of 7 per row) take this path: 1664 -> 1598 us per
// product on the 100^3 stencil at p = 256 FP64, 684 -> 628 us on the 64^3 complex
// lattice at p = 192; four rows per workgroup measured faster than 2, 8 or 16 at one
// row per wave.  The staging loads are issued first and the gathers from global
// memory of a row's first U entries before the barrier, so both are in flight
// together; entries past the first U follow in gather_accumulate (no LDS).  The
// multiply-adds run in entry order, as in gather_accumulate, so a column's bits do
// not depend on the kernel.  Staging passes through registers: used for VN <= 3, and
// at one row per wave only (the routine handles narrower lane groups, but staged they
// measured slower: 3 x 32 complex FP32 361 -> 384 us, the 3 x 16 grouped slice step
// 11.2 -> 14.5 ms).
template <class Tr, int VN, int L>
struct Staged {
    static constexpr int RW = 64 / L;        // rows per wave
    static constexpr int TR = 4 * RW;        // rows per workgroup
    static constexpr int RV = VN * L;        // vectors per row
    static constexpr int NSV = (TR + 2) * RV;  // staged vectors
    static constexpr int NS = (NSV + 255) / 256;
};

// One workgroup of staged_step: rows rb .. rb + TR - 1 of an n-row block (rb >= 0).
// Every thread of the workgroup must call it (it holds a barrier).
template <class Tr, int VN, int L, int U>
__device__ __forceinline__ void staged_step(int n, int rb, const int *__restrict__ rp,
                                   const int *__restrict__ ci,
                                   const typename Tr::val *__restrict__ va,
                                   const typename Tr::vec *__restrict__ src,
                                   const typename Tr::vec *__restrict__ X, typename Tr::vec *dst,
                                   int64_t ldv, typename Tr::scal sigma, typename Tr::scal tau,
                                   typename Tr::scal alpha, bool hv, bool hx,
                                   typename Tr::vec *tile) {
    using vec = typename Tr::vec;
    using val = typename Tr::val;
    using S = Staged<Tr, VN, L>;
    const int lane = threadIdx.x & 63;
    const int sub = lane % L;
    const int wlo = rb - 1;  // first staged row
    vec stage[S::NS];
#pragma unroll
    for (int j = 0; j < S::NS; ++j) {
        const int k = (int)threadIdx.x + 256 * j;
        const int rr = wlo + k / S::RV;
        stage[j] = Tr::zero();
        if (k < S::NSV && rr >= 0 && rr < n) stage[j] = src[(int64_t)rr * ldv + k % S::RV];
    }
    int row = rb + (int)(threadIdx.x >> 6) * S::RW + lane / L;
    if (L == 64) row = __builtin_amdgcn_readfirstlane(row);
    const bool live = row < n;
    const int start = live ? rp[row] : 0, end = live ? rp[row + 1] : 0;
    vec acc[VN];
#pragma unroll
    for (int v = 0; v < VN; ++v) acc[v] = Tr::zero();
    int c[U];
    val a[U];
    bool near[U];
    vec w[U][VN];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const bool ok = start + u < end;
        c[u] = ok ? ci[start + u] : 0;
        a[u] = ok ? va[start + u] : Tr::val_zero();
        near[u] = ok && c[u] >= wlo && c[u] <= wlo + S::TR + 1;
#pragma unroll
        for (int v = 0; v < VN; ++v) {
            w[u][v] = Tr::zero();
            if (ok && !near[u]) w[u][v] = src[(int64_t)c[u] * ldv + sub + v * L];
        }
    }
#pragma unroll
    for (int j = 0; j < S::NS; ++j) {
        const int k = (int)threadIdx.x + 256 * j;
        if (k < S::NSV) tile[k] = stage[j];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int v = 0; v < VN; ++v)
            if (near[u]) w[u][v] = tile[(c[u] - wlo) * S::RV + sub + v * L];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int v = 0; v < VN; ++v) acc[v] = Tr::fma_val(a[u], w[u][v], acc[v]);
    gather_accumulate<Tr, VN, U, L == 64>(start + U, end, ci, va, src, ldv, sub, L, VN, acc);
    if (!live) return;
    const int64_t base = (int64_t)row * ldv + sub;
#pragma unroll
    for (int v = 0; v < VN; ++v) {
        const int64_t idx = base + v * L;
        vec r = clenshaw_combine<Tr>(sigma, tau, acc[v], tile[(row - wlo) * S::RV + sub + v * L]);
        if (hv) r = Tr::sub(r, nt_load(dst + idx));
        if (hx) r = Tr::axpy(alpha, nt_load(X + idx), r);
        nt_store(r, dst + idx);
    }
}

template <class Tr, int VN, int L, bool HAS_V, bool HAS_X, int U>
__global__ __launch_bounds__(256) void clenshaw_step_staged_kernel(
    int n, const int *__restrict__ rp, const int *__restrict__ ci,
    const typename Tr::val *__restrict__ va, const typename Tr::vec *__restrict__ src,
    const typename Tr::vec *__restrict__ X, typename Tr::vec *dst, int64_t ldv,
    typename Tr::scal sigma, typename Tr::scal tau, typename Tr::scal alpha, int group,
    int nblocks) {
    __shared__ typename Tr::vec tile[Staged<Tr, VN, L>::NSV];
    const int lb = xcd_block(blockIdx.x, group, nblocks);
    if (lb < 0) return;  // the whole workgroup: before the barrier
    staged_step<Tr, VN, L, U>(n, lb * Staged<Tr, VN, L>::TR, rp, ci, va, src, X, dst, ldv, sigma,
                              tau, alpha, HAS_V, HAS_X, tile);
}

// Any width: L = 64 lanes per row, chunks of 64*VN vectors, bounds-tested.
template <class Tr, int VN, bool HAS_V, bool HAS_X, int U>
__global__ __launch_bounds__(256) void clenshaw_step_masked_kernel(
    int n, const int *__restrict__ rp, const int *__restrict__ ci,
    const typename Tr::val *__restrict__ va, const typename Tr::vec *__restrict__ src,
    const typename Tr::vec *__restrict__ X, typename Tr::vec *dst, int64_t ldv, int p16,
    typename Tr::scal sigma, typename Tr::scal tau, typename Tr::scal alpha, int group,
    int nblocks) {
    using vec = typename Tr::vec;
    const int lb = xcd_block(blockIdx.x, group, nblocks);
    if (lb < 0) return;
    const int lane = threadIdx.x & 63;
    int row = lb * (int)(blockDim.x / 64) + (int)(threadIdx.x >> 6);
    row = __builtin_amdgcn_readfirstlane(row);
    if (row >= n) return;
    const int start = rp[row], end = rp[row + 1];
    for (int c0 = 0; c0 < p16; c0 += 64 * VN) {
        // vectors c0 + v*64 + lane that exist in this row
        const int left = p16 - c0 - lane;
        const int nvalid = left <= 0 ? 0 : (left + 63) / 64;
        vec acc[VN];
#pragma unroll
        for (int v = 0; v < VN; ++v) acc[v] = Tr::zero();
        gather_accumulate<Tr, VN, U, true>(start, end, ci, va, src, ldv, c0 + lane, 64, nvalid, acc);
        const int64_t base = (int64_t)row * ldv + c0 + lane;
#pragma unroll
        for (int v = 0; v < VN; ++v) {
            if (v < nvalid) {
                const int64_t idx = base + v * 64;
                vec r = clenshaw_combine<Tr>(sigma, tau, acc[v], src[idx]);
                if (HAS_V) r = Tr::sub(r, nt_load(dst + idx));
                if (HAS_X) r = Tr::axpy(alpha, nt_load(X + idx), r);
                nt_store(r, dst + idx);
            }
        }
    }
}

// Narrow blocks (p <= 16 elements per row, any alignment): one lane per row, holding
// all P elements of it, 64 rows per wave.  The row's entries are taken in entry order
// with U of them fetched together, each contributing P multiply-adds, so every column
// gets the same bits as from the wider mappings.  A wave's rows are consecutive, so the
// gathers of neighbouring rows' nearby columns fall on neighbouring addresses.  Used
// for the bounds estimate's single vectors (P = 1), narrow Krylov blocks and narrow
// columns views, where a lane group per row would leave most lanes idle.
template <class Sr, int P, int U>
__global__ __launch_bounds__(256) void clenshaw_step_narrow_kernel(
    int n, const int *__restrict__ rp, const int *__restrict__ ci,
    const typename Sr::val *__restrict__ va, const typename Sr::vec *__restrict__ src,
    const typename Sr::vec *__restrict__ X, typename Sr::vec *dst, int64_t ld, int has_v,
    int has_x, typename Sr::scal sigma, typename Sr::scal tau, typename Sr::scal alpha, int group,
    int nblocks) {
    using vec = typename Sr::vec;
    using val = typename Sr::val;
    const int lb = xcd_block(blockIdx.x, group, nblocks);
    if (lb < 0) return;
    const int row = lb * (int)blockDim.x + (int)threadIdx.x;
    if (row >= n) return;
    const int start = rp[row], end = rp[row + 1];
    vec acc[P];
#pragma unroll
    for (int j = 0; j < P; ++j) acc[j] = Sr::zero();
    for (int e0 = start; e0 < end; e0 += U) {
        int c[U];
        val a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u < end ? e0 + u : end - 1;
            c[u] = ci[e];
            a[u] = va[e];
        }
        vec w[U][P];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const vec *rowp = src + (int64_t)c[u] * ld;
#pragma unroll
            for (int j = 0; j < P; ++j) w[u][j] = rowp[j];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (e0 + u < end) {
#pragma unroll
                for (int j = 0; j < P; ++j) acc[j] = Sr::fma_val(a[u], w[u][j], acc[j]);
            }
    }
    const int64_t base = (int64_t)row * ld;
#pragma unroll
    for (int j = 0; j < P; ++j) {
        vec r = clenshaw_combine<Sr>(sigma, tau, acc[j], src[base + j]);
        if (has_v) r = Sr::sub(r, dst[base + j]);
        if (has_x) r = Sr::axpy(alpha, X[base + j], r);
        dst[base + j] = r;
    }
}

// Unaligned rows: one wave per row, one element per lane per 64 columns.
template <class Tr, int VN, int U>
__global__ __launch_bounds__(256) void clenshaw_step_scalar_kernel(
    int n, const int *__restrict__ rp, const int *__restrict__ ci,
    const typename Tr::val *__restrict__ va, const typename Tr::vec *__restrict__ src,
    const typename Tr::vec *__restrict__ X, typename Tr::vec *dst, int64_t ld, int p, int has_v,
    int has_x, typename Tr::scal sigma, typename Tr::scal tau, typename Tr::scal alpha, int group,
    int nblocks) {
    using vec = typename Tr::vec;
    const int lb = xcd_block(blockIdx.x, group, nblocks);
    if (lb < 0) return;
    const int lane = threadIdx.x & 63;
    int row = lb * (int)(blockDim.x / 64) + (int)(threadIdx.x >> 6);
    row = __builtin_amdgcn_readfirstlane(row);
    if (row >= n) return;
    const int start = rp[row], end = rp[row + 1];
    for (int c0 = 0; c0 < p; c0 += 64 * VN) {
        const int left = p - c0 - lane;
        const int nvalid = left <= 0 ? 0 : (left + 63) / 64;
        vec acc[VN];
#pragma unroll
        for (int v = 0; v < VN; ++v) acc[v] = Tr::zero();
        gather_accumulate<Tr, VN, U, true>(start, end, ci, va, src, ld, c0 + lane, 64, nvalid, acc);
        const int64_t base = (int64_t)row * ld + c0 + lane;
#pragma unroll
        for (int v = 0; v < VN; ++v) {
            if (v < nvalid) {
                const int64_t idx = base + v * 64;
                vec r = clenshaw_combine<Tr>(sigma, tau, acc[v], src[idx]);
                if (has_v) r = Tr::sub(r, dst[idx]);
                if (has_x) r = Tr::axpy(alpha, X[idx], r);
                dst[idx] = r;
            }
        }
    }
}

}  // namespace afsi
