// FP64 matrix-core kernels for the dense steps (gfx950, v_mfma_f64_16x16x4f64).
//
// gram : G = X^T Y for tall n x p X and n x q Y (Cholesky-QR Gram X^H X, the
//        Rayleigh-Ritz projection Q^H (A Q), the locked projection L^H X).  A
//        256-thread block owns a 64 x 128 tile of G and a chunk of rows; its four
//        waves own 32 x 64 sub-tiles (2 x 4 MFMA accumulators).  Rows are consumed
//        16 at a time through double-buffered LDS tiles filled by coalesced loads.
//        Each chunk's partial tile goes to scratch; a second kernel adds the chunks
//        in chunk order (no atomics: bitwise reproducible for fixed n, p, q).
// gemm : Y = alpha X M + beta Y for n x p X and small p x q M (X R^{-1}, Q U,
//        (A Q) U, the locked-vector update).  Same 64 x 128 tiles over (rows of Y,
//        columns of Y), the reduction over p runs through the same LDS pipeline with
//        X stored transposed so operand reads are conflict-free.  Column tiles of a
//        row tile are adjacent in the grid, so X rows are reused from cache.
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
constexpr int PADM = BM + 4, PADN = BN + 4;  // LDS row padding

__global__ __launch_bounds__(256) void gram_f64_kernel(const double *__restrict__ X, int64_t ldx,
                                                       const double *__restrict__ Y, int64_t ldy,
                                                       int64_t n, int p, int q,
                                                       int64_t rows_per_chunk,
                                                       double *__restrict__ ws) {
    __shared__ double Xs[2][BK][PADM];
    __shared__ double Ys[2][BK][PADN];
    const int tiles_j = (q + BN - 1) / BN;
    const int ti = blockIdx.x / tiles_j, tj = blockIdx.x % tiles_j;
    const int chunk = blockIdx.y;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int wr = w >> 1, wc = w & 1;
    const int i0 = ti * BM, j0 = tj * BN;
    const int lk = lane >> 4, lc = lane & 15;
    const int64_t r0 = (int64_t)chunk * rows_per_chunk;
    const int64_t r1 = min(n, r0 + rows_per_chunk);
    // global -> register staging: X tile 16 x 64 (4 per thread), Y tile 16 x 128 (8 per thread)
    const int xr = tid >> 4, xc = (tid & 15) * 4;
    const int yr = tid >> 4, yc = (tid & 15) * 8;
    double xa[4], ya[8];
    auto fetch = [&](int64_t rb) {
        const int64_t rx = rb + xr, ry = rb + yr;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int c = i0 + xc + t;
            xa[t] = (rx < r1 && c < p) ? X[rx * ldx + c] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int c = j0 + yc + t;
            ya[t] = (ry < r1 && c < q) ? Y[ry * ldy + c] : 0.0;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int t = 0; t < 4; ++t) Xs[buf][xr][xc + t] = xa[t];
#pragma unroll
        for (int t = 0; t < 8; ++t) Ys[buf][yr][yc + t] = ya[t];
    };
    d4 acc[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = d4{0, 0, 0, 0};
    const int64_t ntiles = (r1 - r0 + BK - 1) / BK;
    if (ntiles > 0) {
        fetch(r0);
        stash(0);
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
        if (kt + 1 < ntiles) stash(buf ^ 1);
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

__global__ void reduce_chunks_kernel(const double *__restrict__ ws, int nchunks, int p, int q,
                                     double *__restrict__ G, int64_t ldg) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)p * q) return;
    const int i = (int)(idx / q), j = (int)(idx % q);
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += ws[(int64_t)c * p * q + idx];
    G[(int64_t)i * ldg + j] = s;
}

__global__ __launch_bounds__(256) void gemm_f64_kernel(const double *__restrict__ X, int64_t ldx,
                                                       const double *__restrict__ M, int64_t ldm,
                                                       int64_t n, int p, int q, double alpha,
                                                       double beta, double *__restrict__ Y,
                                                       int64_t ldy) {
    __shared__ double Xt[2][BK][PADM];  // X tile transposed: [k][row]
    __shared__ double Ms[2][BK][PADN];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int wr = w >> 1, wc = w & 1;
    const int tiles_q = (q + BN - 1) / BN;  // column tiles of one row tile are adjacent
    const int64_t r0 = (int64_t)(blockIdx.x / tiles_q) * BM;
    const int c0 = (int)(blockIdx.x % tiles_q) * BN;
    const int lk = lane >> 4, lc = lane & 15;
    // X tile 64 rows x 16 k: thread -> row tid/4, k (tid%4)*4 .. +3
    const int xr = tid >> 2, xk = (tid & 3) * 4;
    // M tile 16 k x 128 cols: thread -> k tid/16, cols (tid%16)*8 .. +7
    const int mk = tid >> 4, mc = (tid & 15) * 8;
    double xa[4], ma[8];
    const int64_t row = r0 + xr;
    auto fetch = [&](int k0) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = k0 + xk + t;
            xa[t] = (row < n && k < p) ? X[row * ldx + k] : 0.0;
        }
        const int km = k0 + mk;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int c = c0 + mc + t;
            ma[t] = (km < p && c < q) ? M[(int64_t)km * ldm + c] : 0.0;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int t = 0; t < 4; ++t) Xt[buf][xk + t][xr] = xa[t];
#pragma unroll
        for (int t = 0; t < 8; ++t) Ms[buf][mk][mc + t] = ma[t];
    };
    d4 acc[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = d4{0, 0, 0, 0};
    const int ntiles = (p + BK - 1) / BK;
    if (ntiles > 0) {
        fetch(0);
        stash(0);
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
        if (kt + 1 < ntiles) stash(buf ^ 1);
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

// Split n rows into chunks so that tiles * chunks is about `target_blocks`; chunk
// sizes depend only on (n, tiles), which keeps reductions reproducible.
static void chunking(int64_t n, int64_t tiles, int64_t gran, int64_t target_blocks, int64_t &rows,
                     int64_t &nchunks) {
    int64_t want = (target_blocks + tiles - 1) / tiles;
    const int64_t maxc = (n + 511) / 512;
    if (want > maxc) want = maxc;
    if (want < 1) want = 1;
    rows = (n + want - 1) / want;
    rows = (rows + gran - 1) / gran * gran;
    if (rows < gran) rows = gran;
    nchunks = (n + rows - 1) / rows;
    if (nchunks < 1) nchunks = 1;
}

static void gram_raw(const double *X, int64_t ldx, const double *Y, int64_t ldy, int64_t n,
                     int64_t p, int64_t q, double *G, int64_t ldg, int slot, hipStream_t s) {
    const int64_t tiles = ((p + BM - 1) / BM) * ((q + BN - 1) / BN);
    int64_t rows, nchunks;
    chunking(n, tiles, BK, 1024, rows, nchunks);
    double *ws = (double *)workspace(s).dev_reserve(slot, sizeof(double) * nchunks * p * q);
    hipLaunchKernelGGL(gram_f64_kernel, dim3((unsigned)tiles, (unsigned)nchunks), dim3(256), 0, s,
                       X, ldx, Y, ldy, n, (int)p, (int)q, rows, ws);
    hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)((p * q + 255) / 256)), dim3(256), 0, s,
                       ws, (int)nchunks, (int)p, (int)q, G, ldg);
    AFSI_HIP(hipGetLastError());
}

void gram_f64(const double *X, int64_t ldx, const double *Y, int64_t ldy, int64_t n, int64_t p,
              int64_t q, double *G, int64_t ldg, hipStream_t s) {
    if (p == 0 || q == 0) return;
    gram_raw(X, ldx, Y, ldy, n, p, q, G, ldg, SLOT_PARTIAL, s);
}

void gemm_f64(const double *X, int64_t ldx, const double *M, int64_t ldm, int64_t n, int64_t p,
              int64_t q, double alpha, double beta, double *Y, int64_t ldy, hipStream_t s) {
    if (n == 0 || q == 0) return;
    const int64_t blocks = ((q + BN - 1) / BN) * ((n + BM - 1) / BM);
    AFSI_REQUIRE(blocks < (1LL << 31), "block product too large");
    hipLaunchKernelGGL(gemm_f64_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, ldx, M, ldm, n,
                       (int)p, (int)q, alpha, beta, Y, ldy);
    AFSI_HIP(hipGetLastError());
}

void gram_c128(const double *X, int64_t ldx, const double *Y, int64_t ldy, int64_t n, int64_t p,
               int64_t q, double *G, int64_t ldg, hipStream_t s) {
    if (p == 0 || q == 0) return;
    double *Gr = (double *)workspace(s).dev_reserve(SLOT_REALVIEW, sizeof(double) * 4 * p * q);
    gram_raw(X, 2 * ldx, Y, 2 * ldy, n, 2 * p, 2 * q, Gr, 2 * q, SLOT_PARTIAL, s);
    hipLaunchKernelGGL(gram_combine_c128_kernel, dim3((unsigned)((p * q + 255) / 256)), dim3(256), 0,
                       s, Gr, (int)p, (int)q, G, ldg);
    AFSI_HIP(hipGetLastError());
}

void gemm_c128(const double *X, int64_t ldx, const double *M, int64_t ldm, int64_t n, int64_t p,
               int64_t q, double alpha, double beta, double *Y, int64_t ldy, hipStream_t s) {
    if (n == 0 || q == 0) return;
    double *Mr = (double *)workspace(s).dev_reserve(SLOT_REALVIEW, sizeof(double) * 4 * p * q);
    if (p > 0)
        hipLaunchKernelGGL(expand_c128_kernel, dim3((unsigned)((p * q + 255) / 256)), dim3(256), 0,
                           s, M, ldm, (int)p, (int)q, Mr);
    gemm_f64(X, 2 * ldx, Mr, 2 * q, n, 2 * p, 2 * q, alpha, beta, Y, 2 * ldy, s);
}

}  // namespace afsi
