// Grouped Clenshaw step: one launch advances several spectrum slices of one matrix by
// one product each, where every slice keeps its own row-major blocks X, P0, P1.
//
// The launch's rows are the slices' rows one after another: slice g owns logical rows
// [g * npad, g * npad + n), npad being n rounded up to whole workgroups, so a
// workgroup never spans two slices and the slice index, its pointers and its product
// parameters are wave-uniform (scalar loads, one base address per gather).  Inside a
// slice the lane mapping, the gathers and the fused epilogue are those of the
// single-block kernel, so every column gets the same bits as from afsi_filter_block.
// Unlike the batched kernel over concatenated blocks, each gather reads a whole row
// segment of one contiguous block instead of 2 KB out of a row of every slice.
#pragma once

#include "clenshaw_dispatch.h"

namespace afsi {

// STEADY: every slice of the launch subtracts its b_{j+2} and adds alpha X (the steady
// products of a filter), known at compile time as in the single-block kernel; otherwise
// each slice's flags are read at run time.
template <class Tr, int VN, int L, int U, bool STAGE, bool STEADY>
__global__ __launch_bounds__(256) void clenshaw_grouped_kernel(
    int n, const int *__restrict__ rp, const int *__restrict__ ci,
    const typename Tr::val *__restrict__ va, int group, int nblocks, const GroupArgs args) {
    using vec = typename Tr::vec;
    using scal = typename Tr::scal;
    constexpr int RW = 64 / L;
    const int lb = xcd_block(blockIdx.x, group, nblocks);
    if (lb < 0) return;
    const int64_t r0 = (int64_t)lb * (4 * RW);
    const int g = __builtin_amdgcn_readfirstlane((int)(r0 / args.npad));
    if (g >= args.ngroups) return;
    if constexpr (STAGE) {  // the slice's rows of its source block in LDS (staged_step)
        __shared__ vec tile[Staged<Tr, VN, L>::NSV];
        const int s = args.src[g];
        const vec *X = (const vec *)args.X[g];
        vec *P0 = (vec *)args.P0[g], *P1 = (vec *)args.P1[g];
        staged_step<Tr, VN, L, U>(n, (int)(r0 - (int64_t)g * args.npad), rp, ci, va,
                                  s == 0 ? X : (s == 1 ? P0 : P1), X, args.dst[g] == 1 ? P0 : P1,
                                  args.ldv[g], (scal)args.sigma[g], (scal)args.tau[g],
                                  (scal)args.alpha[g], args.has_v[g] != 0, args.alpha[g] != 0.0,
                                  tile);
        return;
    }
    const int lane = threadIdx.x & 63;
    const int sub = lane % L;
    int row = (int)(r0 - (int64_t)g * args.npad) + (int)(threadIdx.x >> 6) * RW + lane / L;
    if (L == 64) row = __builtin_amdgcn_readfirstlane(row);
    if (row >= n) return;
    const vec *X = (const vec *)args.X[g];
    vec *P0 = (vec *)args.P0[g], *P1 = (vec *)args.P1[g];
    const int s = args.src[g];
    const vec *src = s == 0 ? X : (s == 1 ? P0 : P1);
    vec *dst = args.dst[g] == 1 ? P0 : P1;
    const int64_t ldv = args.ldv[g];
    const bool hv = STEADY || args.has_v[g] != 0;
    const scal alpha = (scal)args.alpha[g];
    const bool hx = STEADY || args.alpha[g] != 0.0;
    constexpr bool EARLY = L < 64 && VN <= 3;  // as in clenshaw_step_kernel
    const int64_t base = (int64_t)row * ldv + sub;
    vec vin[VN], xin[VN];
    if (EARLY) {
#pragma unroll
        for (int v = 0; v < VN; ++v) {
            if (hv) vin[v] = nt_load(dst + base + v * L);
            if (hx) xin[v] = nt_load(X + base + v * L);
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
        vec r = clenshaw_combine<Tr>((scal)args.sigma[g], (scal)args.tau[g], acc[v], src[idx]);
        if (hv) r = Tr::sub(r, EARLY ? vin[v] : nt_load(dst + idx));
        if (hx) r = Tr::axpy(alpha, EARLY ? xin[v] : nt_load(X + idx), r);
        nt_store(r, dst + idx);
    }
}

template <class Tr, int VN, int L>
void launch_grouped(const MatView &A, GroupArgs &args, hipStream_t s) {
    constexpr int U = VN <= 4 ? 8 : 4;
    const int rows_per_block = 4 * (64 / L);
    args.npad = (A.n + rows_per_block - 1) / rows_per_block * rows_per_block;
    const int64_t rows = args.npad * args.ngroups;
    AFSI_REQUIRE(rows / rows_per_block < (1LL << 31), "grouped step: too many rows");
    const Grid g = xcd_grid(rows, rows_per_block, run_rows_for(A, VN * L * 16, rows_per_block));
    if constexpr (VN <= 3 && L == 64) {
        if (A.stage_near) {
            hipLaunchKernelGGL((clenshaw_grouped_kernel<Tr, VN, L, U, true, false>),
                               dim3((unsigned)g.grid), dim3(256), 0, s, (int)A.n, A.rp, A.ci,
                               (const typename Tr::val *)A.val, g.group, g.nblocks, args);
            return;
        }
    }
    bool steady = true;
    for (int k = 0; k < args.ngroups; ++k) steady = steady && args.has_v[k] && args.alpha[k] != 0.0;
    if (steady)
        hipLaunchKernelGGL((clenshaw_grouped_kernel<Tr, VN, L, U, false, true>), dim3((unsigned)g.grid),
                           dim3(256), 0, s, (int)A.n, A.rp, A.ci, (const typename Tr::val *)A.val,
                           g.group, g.nblocks, args);
    else
        hipLaunchKernelGGL((clenshaw_grouped_kernel<Tr, VN, L, U, false, false>), dim3((unsigned)g.grid),
                           dim3(256), 0, s, (int)A.n, A.rp, A.ci, (const typename Tr::val *)A.val,
                           g.group, g.nblocks, args);
}

// true if p16 has an exact lane mapping (the single-block kernel's table, same order)
template <class Tr>
bool dispatch_grouped(const MatView &A, int p16, GroupArgs &args, hipStream_t s) {
#define AFSI_GROUPED(VN_, L_)                                                                       \
    if (p16 == (VN_) * (L_)) return launch_grouped<Tr, VN_, L_>(A, args, s), true;
    if (A.stage_near) { AFSI_GROUPED(1, 64) }  // as in dispatch_flags
    AFSI_GROUPED_MAPPINGS(AFSI_GROUPED)
#undef AFSI_GROUPED
    return false;
}

}  // namespace afsi

#define AFSI_DEFINE_GROUPED_ENTRY(NAME, TR)                                                         \
    namespace afsi {                                                                                \
    bool NAME##_grouped(const MatView &A, int p16, GroupArgs &args, hipStream_t s) {                \
        return dispatch_grouped<TR>(A, p16, args, s);                                               \
    }                                                                                               \
    }
