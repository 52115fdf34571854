// FP64 matrix-core kernels for the dense steps (gfx950, v_mfma_f64_16x16x4f64).
//
// gram : G = X^T Y for tall n x p X and n x q Y (Cholesky-QR Gram X^H X, the
//        Rayleigh-Ritz projection Q^H (A Q), the locked projection L^H X).  A
//        256-thread block owns a 64 x 128 tile of G and a chunk of rows; its four
//        waves own 32 x 64 sub-tiles (2 x 4 MFMA accumulators).  Rows are consumed
//        16 at a time through double-buffered LDS tiles filled by coalesced loads.
//        Each chunk's partial tile goes to scratch; a second kernel adds the chunks
//        in chunk order (no atomics: bitwise reproducible for fixed n, p, q).  The
//        chunk count is a multiple of 8 sized so that each XCD runs its tiles in
//        one resident round.
// gemm : Y = alpha X M + beta Y for n x p X and small p x q M (X R^{-1}, Q U,
//        (A Q) U, the locked-vector update).  Same 64 x 128 tiles over (rows of Y,
//        columns of Y), the reduction over p runs through the same LDS pipeline with
//        X stored transposed so operand reads are conflict-free.  Column tiles of a
//        row tile are adjacent in the grid, so X rows are reused from cache.  For an
//        upper-triangular M (R^{-1}) a column tile stops at its last column's row.
// A Gram product with X == Y computes only the tiles that reach the diagonal or above
// it and takes its lower triangle from the upper one in the chunk reduction, so the
// Cholesky-QR Gram is exactly Hermitian.
// Complex Hermitian blocks use real views: a complex n x p block with leading
// dimension ld is a real n x 2p block with leading dimension 2 ld, and
//   X^H Y = (Gr[2i,2j] + Gr[2i+1,2j+1]) + i (Gr[2i,2j+1] - Gr[2i+1,2j])  with Gr = Xr^T Yr,
//   X M   = Xr Mr  with Mr[2k,2j] = Re M, Mr[2k,2j+1] = Im M, Mr[2k+1,2j] = -Im M,
//           Mr[2k+1,2j+1] = Re M.
#include "internal.h"

namespace afsi {

typedef double d4 __attribute__((ext_vector_type(4)));

// Operand layout of the 16x16x4 f64 MFMA: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator element e of lane l is D[l / 16 + 4 e][l % 16].
__device__ inline d4 mfma16x16x4(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int BM = 64, BN = 128, BK = 16;
constexpr int PADM = BM + 2, PADN = BN + 4;  // LDS row padding (rows stay 16-byte aligned)

// Tile loads: consecutive lanes read consecutive 16-byte pairs, so one load
// instruction of a wave covers whole rows of the tile.
//  VEC (16-byte aligned rows and base, even column count, at least one row): the pair
//   address is clamped into the matrix and the raw pair is kept; pairs that matter and
//   fall outside (the reduction tail) are zeroed only when the tile is stashed, on the
//   one tile that has a tail.  The prefetch of the next tile therefore overlaps the
//   MFMAs of the current one.  Pairs outside in a free dimension feed only outputs
//   that are never stored.
//  otherwise: two guarded scalars, zero outside.
template <bool VEC>
__device__ inline double2 load_pair(const double *__restrict__ base, int64_t row, int64_t nrows,
                                    int64_t ld, int col, int ncols) {
    if (VEC) {
        const int64_t r = row < nrows ? row : nrows - 1;
        const int c = col < ncols ? col : ncols - 2;
        return *reinterpret_cast<const double2 *>(base + r * ld + c);
    }
    if (row >= nrows) return make_double2(0.0, 0.0);
    const double *ptr = base + row * ld + col;
    return make_double2(col < ncols ? ptr[0] : 0.0, col + 1 < ncols ? ptr[1] : 0.0);
}

__device__ inline double2 zero_unless(bool keep, double2 v) {
    return make_double2(keep ? v.x : 0.0, keep ? v.y : 0.0);
}

template <bool VEC>
__global__ __launch_bounds__(256) void gram_f64_kernel(const double *__restrict__ X, int64_t ldx,
                                                       const double *__restrict__ Y, int64_t ldy,
                                                       int64_t n, int p, int q,
                                                       int64_t rows_per_chunk, int nchunks,
                                                       bool upper_only, double *__restrict__ ws) {
    __shared__ __align__(16) double Xs[2][BK][PADM];
    __shared__ __align__(16) double Ys[2][BK][PADN];
    const int tiles_i = (p + BM - 1) / BM, tiles_j = (q + BN - 1) / BN;
    // upper_only: only tiles holding an entry on or above the diagonal (row tile ti
    // with ti BM < (tj + 1) BN), column tile by column tile
    auto col_tiles = [&](int tj) { return upper_only ? min(tiles_i, ((tj + 1) * BN + BM - 1) / BM) : tiles_i; };
    int tiles = 0;
    for (int tj = 0; tj < tiles_j; ++tj) tiles += col_tiles(tj);
    // workgroup b runs on XCD b % 8: all tiles of one row chunk go to the same XCD
    // (consecutive slots there), so the chunk's rows come from HBM once and the other
    // tiles read them from that XCD's L2
    const int slot = blockIdx.x >> 3;
    const int chunk = (slot / tiles) * 8 + (blockIdx.x & 7);
    if (chunk >= nchunks) return;
    int ti = slot % tiles, tj = 0;
    while (ti >= col_tiles(tj)) ti -= col_tiles(tj++);
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int wr = w >> 1, wc = w & 1;
    const int i0 = ti * BM, j0 = tj * BN;
    const int lk = lane >> 4, lc = lane & 15;
    const int64_t r0 = (int64_t)chunk * rows_per_chunk;
    const int64_t r1 = min(n, r0 + rows_per_chunk);
    // X tile 16 rows x 64 columns = 512 pairs (2 per thread), Y tile 16 x 128 = 1024
    // pairs (4 per thread); pair e sits at row e / (width / 2), column 2 (e % (width / 2))
    double2 xa[2], ya[4];
    auto fetch = [&](int64_t rb) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int e = tid + 256 * t;
            xa[t] = load_pair<VEC>(X, rb + (e >> 5), r1, ldx, i0 + 2 * (e & 31), p);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int e = tid + 256 * t;
            ya[t] = load_pair<VEC>(Y, rb + (e >> 6), r1, ldy, j0 + 2 * (e & 63), q);
        }
    };
    // rb: first row of the tile being stashed; rows past the chunk end are zeroed
    auto stash = [&](int buf, int64_t rb) {
        if (VEC && rb + BK > r1) {
#pragma unroll
            for (int t = 0; t < 2; ++t) xa[t] = zero_unless(rb + ((tid + 256 * t) >> 5) < r1, xa[t]);
#pragma unroll
            for (int t = 0; t < 4; ++t) ya[t] = zero_unless(rb + ((tid + 256 * t) >> 6) < r1, ya[t]);
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int e = tid + 256 * t;
            *reinterpret_cast<double2 *>(&Xs[buf][e >> 5][2 * (e & 31)]) = xa[t];
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int e = tid + 256 * t;
            *reinterpret_cast<double2 *>(&Ys[buf][e >> 6][2 * (e & 63)]) = ya[t];
        }
    };
    d4 acc[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = d4{0, 0, 0, 0};
    const int64_t ntiles = (r1 - r0 + BK - 1) / BK;
    if (ntiles > 0) {
        fetch(r0);
        stash(0, r0);
    }
    __syncthreads();
    for (int64_t kt = 0; kt < ntiles; ++kt) {
        const int buf = (int)(kt & 1);
        if (kt + 1 < ntiles) fetch(r0 + (kt + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
            const int kr = kk * 4 + lk;
            double av[2], bv[4];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = Xs[buf][kr][wr * 32 + a * 16 + lc];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = Ys[buf][kr][wc * 64 + b * 16 + lc];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = mfma16x16x4(av[a], bv[b], acc[a][b]);
        }
        if (kt + 1 < ntiles) stash(buf ^ 1, r0 + (kt + 1) * BK);
        __syncthreads();
    }
    double *out = ws + (int64_t)chunk * p * q;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int gj = j0 + wc * 64 + b * 16 + lc;
            if (gj >= q) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gi = i0 + wr * 32 + a * 16 + lk + 4 * e;
                if (gi < p) out[(int64_t)gi * q + gj] = acc[a][b][e];
            }
        }
}

// G = sum of the chunk partials in chunk order; with `sym` (p == q) entries below the
// diagonal are taken from their mirror above it, so G is exactly symmetric.
__global__ void reduce_chunks_kernel(const double *__restrict__ ws, int nchunks, int p, int q,
                                     bool sym, double *__restrict__ G, int64_t ldg) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)p * q) return;
    const int i = (int)(idx / q), j = (int)(idx % q);
    const int64_t src = (sym && i > j) ? (int64_t)j * q + i : idx;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += ws[(int64_t)c * p * q + src];
    G[(int64_t)i * ldg + j] = s;
}

template <bool VEC>
__global__ __launch_bounds__(256) void gemm_f64_kernel(const double *__restrict__ X, int64_t ldx,
                                                       const double *__restrict__ M, int64_t ldm,
                                                       int64_t n, int p, int q, double alpha,
                                                       double beta, bool upper,
                                                       double *__restrict__ Y, int64_t ldy) {
    __shared__ __align__(16) double Xt[2][BK][PADM];  // X tile transposed: [k][row]
    __shared__ __align__(16) double Ms[2][BK][PADN];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int wr = w >> 1, wc = w & 1;
    // workgroup b runs on XCD b % 8: the column tiles of one row tile go to the same
    // XCD in consecutive slots, so X rows come from HBM once
    const int tiles_q = (q + BN - 1) / BN;
    const int64_t slot = blockIdx.x >> 3;
    const int64_t rtile = (slot / tiles_q) * 8 + (blockIdx.x & 7);
    if (rtile * BM >= n) return;
    const int64_t r0 = rtile * BM;
    const int c0 = (int)(slot % tiles_q) * BN;
    const int lk = lane >> 4, lc = lane & 15;
    // X tile 64 rows x 16 k = 512 pairs (2 per thread, pair e: row e / 8, k 2 (e % 8));
    // M tile 16 k x 128 columns = 1024 pairs (4 per thread, pair e: k e / 64, column
    // 2 (e % 64))
    double2 xa[2], ma[4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int e = tid + 256 * t;
            xa[t] = load_pair<VEC>(X, r0 + (e >> 3), n, ldx, k0 + 2 * (e & 7), p);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int e = tid + 256 * t;
            ma[t] = load_pair<VEC>(M, k0 + (e >> 6), p, ldm, c0 + 2 * (e & 63), q);
        }
    };
    // k0: first reduction index of the tile being stashed; indices >= p are zeroed in
    // both operands
    auto stash = [&](int buf, int k0) {
        if (VEC && k0 + BK > p) {
#pragma unroll
            for (int t = 0; t < 2; ++t) xa[t] = zero_unless(k0 + 2 * ((tid + 256 * t) & 7) < p, xa[t]);
#pragma unroll
            for (int t = 0; t < 4; ++t) ma[t] = zero_unless(k0 + ((tid + 256 * t) >> 6) < p, ma[t]);
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int e = tid + 256 * t;
            const int r = e >> 3, k = 2 * (e & 7);
            Xt[buf][k][r] = xa[t].x;
            Xt[buf][k + 1][r] = xa[t].y;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int e = tid + 256 * t;
            *reinterpret_cast<double2 *>(&Ms[buf][e >> 6][2 * (e & 63)]) = ma[t];
        }
    };
    d4 acc[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = d4{0, 0, 0, 0};
    // upper-triangular M (M[k][c] = 0 for k > c): rows past this column tile add zeros
    const int kend = upper ? min(p, c0 + BN) : p;
    const int ntiles = (kend + BK - 1) / BK;
    if (ntiles > 0) {
        fetch(0);
        stash(0, 0);
    }
    __syncthreads();
    for (int kt = 0; kt < ntiles; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < ntiles) fetch((kt + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
            const int kr = kk * 4 + lk;
            double av[2], bv[4];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = Xt[buf][kr][wr * 32 + a * 16 + lc];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = Ms[buf][kr][wc * 64 + b * 16 + lc];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = mfma16x16x4(av[a], bv[b], acc[a][b]);
        }
        if (kt + 1 < ntiles) stash(buf ^ 1, (kt + 1) * BK);
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int gj = c0 + wc * 64 + b * 16 + lc;
            if (gj >= q) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t gi = r0 + wr * 32 + a * 16 + lk + 4 * e;
                if (gi < n) {
                    double *yp = Y + gi * ldy + gj;
                    double v = alpha * acc[a][b][e];
                    if (beta != 0.0) v = __builtin_fma(beta, *yp, v);
                    *yp = v;
                }
            }
        }
}

__global__ void gram_combine_c128_kernel(const double *__restrict__ Gr, int p, int q,
                                         double *__restrict__ G, int64_t ldg) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)p * q) return;
    const int i = (int)(idx / q), j = (int)(idx % q);
    const int64_t q2 = 2 * (int64_t)q;
    const double rr = Gr[(2 * i) * q2 + 2 * j], ii = Gr[(2 * i + 1) * q2 + 2 * j + 1];
    const double ri = Gr[(2 * i) * q2 + 2 * j + 1], ir = Gr[(2 * i + 1) * q2 + 2 * j];
    G[2 * ((int64_t)i * ldg + j)] = rr + ii;
    G[2 * ((int64_t)i * ldg + j) + 1] = ri - ir;
}

__global__ void expand_c128_kernel(const double *__restrict__ M, int64_t ldm, int p, int q,
                                   double *__restrict__ Mr) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)p * q) return;
    const int k = (int)(idx / q), j = (int)(idx % q);
    const double re = M[2 * ((int64_t)k * ldm + j)], im = M[2 * ((int64_t)k * ldm + j) + 1];
    const int64_t q2 = 2 * (int64_t)q;
    Mr[(2 * k) * q2 + 2 * j] = re;
    Mr[(2 * k) * q2 + 2 * j + 1] = im;
    Mr[(2 * k + 1) * q2 + 2 * j] = -im;
    Mr[(2 * k + 1) * q2 + 2 * j + 1] = re;
}

// ---------------------------------------------------------------- host launchers

// Gram workgroups resident at once on one XCD: 32 CUs x 3 (LDS-bound: ~51 KB each).
constexpr int64_t kGramResidentPerXcd = 96;

// the branch-free pair loads apply: every row of the row-major rows x cols matrix
// starts on a 16-byte boundary, the column count is even and there is a row
static bool aligned_pairs(const double *base, int64_t ld, int64_t rows, int64_t cols) {
    return (reinterpret_cast<uintptr_t>(base) & 15) == 0 && (ld & 1) == 0 && (cols & 1) == 0 &&
           rows > 0 && cols > 0;
}

static void gram_raw(const double *X, int64_t ldx, const double *Y, int64_t ldy, int64_t n,
                     int64_t p, int64_t q, double *G, int64_t ldg, int slot, hipStream_t s) {
    // X == Y: tiles strictly below the diagonal are skipped and the reduction mirrors
    // the upper triangle, so that G is exactly Hermitian; the chunks are sized by the
    // tiles that run, so every XCD still holds one full resident round
    const bool sym = X == Y && ldx == ldy && p == q;
    const int64_t ti = (p + BM - 1) / BM, tj = (q + BN - 1) / BN;
    int64_t tiles = 0;
    for (int64_t j = 0; j < tj; ++j) tiles += sym ? std::min(ti, ((j + 1) * BN + BM - 1) / BM) : ti;
    // chunks: a multiple of 8 (one per XCD in turn) with at most one resident round
    // of workgroups per XCD, and at least 512 rows each
    const int64_t per_xcd = std::max<int64_t>(1, kGramResidentPerXcd / tiles);
    int64_t want = 8 * per_xcd;
    want = std::min(want, std::max<int64_t>(1, (n + 511) / 512));
    int64_t rows = (n + want - 1) / want;
    rows = std::max<int64_t>(BK, (rows + BK - 1) / BK * BK);
    const int64_t nchunks = std::max<int64_t>(1, (n + rows - 1) / rows);
    double *ws = (double *)workspace(s).dev_reserve(slot, sizeof(double) * nchunks * p * q);
    const int64_t grid = tiles * ((nchunks + 7) / 8 * 8);
    AFSI_REQUIRE(grid < (1LL << 31), "Gram product too large");
    const bool vec = aligned_pairs(X, ldx, n, p) && aligned_pairs(Y, ldy, n, q);
    hipLaunchKernelGGL(vec ? gram_f64_kernel<true> : gram_f64_kernel<false>, dim3((unsigned)grid),
                       dim3(256), 0, s, X, ldx, Y, ldy, n, (int)p, (int)q, rows, (int)nchunks, sym,
                       ws);
    hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)((p * q + 255) / 256)), dim3(256), 0, s,
                       ws, (int)nchunks, (int)p, (int)q, sym, G, ldg);
    AFSI_HIP(hipGetLastError());
}

void gram_f64(const double *X, int64_t ldx, const double *Y, int64_t ldy, int64_t n, int64_t p,
              int64_t q, double *G, int64_t ldg, hipStream_t s) {
    if (p == 0 || q == 0) return;
    gram_raw(X, ldx, Y, ldy, n, p, q, G, ldg, SLOT_PARTIAL, s);
}

void gemm_f64(const double *X, int64_t ldx, const double *M, int64_t ldm, int64_t n, int64_t p,
              int64_t q, double alpha, double beta, double *Y, int64_t ldy, hipStream_t s,
              bool upper) {
    if (n == 0 || q == 0) return;
    const int64_t blocks = ((q + BN - 1) / BN) * (((n + BM - 1) / BM + 7) / 8 * 8);
    AFSI_REQUIRE(blocks < (1LL << 31), "block product too large");
    const bool vec = aligned_pairs(X, ldx, n, p) && aligned_pairs(M, ldm, p, q);
    hipLaunchKernelGGL(vec ? gemm_f64_kernel<true> : gemm_f64_kernel<false>, dim3((unsigned)blocks),
                       dim3(256), 0, s, X, ldx, M, ldm, n, (int)p, (int)q, alpha, beta, upper, Y,
                       ldy);
    AFSI_HIP(hipGetLastError());
}

void gram_c128(const double *X, int64_t ldx, const double *Y, int64_t ldy, int64_t n, int64_t p,
               int64_t q, double *G, int64_t ldg, hipStream_t s) {
    if (p == 0 || q == 0) return;
    double *Gr = (double *)workspace(s).dev_reserve(SLOT_REALVIEW, sizeof(double) * 4 * p * q);
    // the real view of X^H X is symmetric too: gram_raw sees X == Y and mirrors
    gram_raw(X, 2 * ldx, Y, 2 * ldy, n, 2 * p, 2 * q, Gr, 2 * q, SLOT_PARTIAL, s);
    hipLaunchKernelGGL(gram_combine_c128_kernel, dim3((unsigned)((p * q + 255) / 256)), dim3(256), 0,
                       s, Gr, (int)p, (int)q, G, ldg);
    AFSI_HIP(hipGetLastError());
}

void gemm_c128(const double *X, int64_t ldx, const double *M, int64_t ldm, int64_t n, int64_t p,
               int64_t q, double alpha, double beta, double *Y, int64_t ldy, hipStream_t s,
               bool upper) {
    if (n == 0 || q == 0) return;
    double *Mr = (double *)workspace(s).dev_reserve(SLOT_REALVIEW, sizeof(double) * 4 * p * q);
    if (p > 0)
        hipLaunchKernelGGL(expand_c128_kernel, dim3((unsigned)((p * q + 255) / 256)), dim3(256), 0,
                           s, M, ldm, (int)p, (int)q, Mr);
    // complex upper-triangular M has a real view with Mr[kr][jr] = 0 once kr / 2 > jr / 2,
    // so the column-tile bound of the real kernel (BN even) still holds
    gemm_f64(X, 2 * ldx, Mr, 2 * q, n, 2 * p, 2 * q, alpha, beta, Y, 2 * ldy, s, upper);
}

}  // namespace afsi
