// Dense FP64 kernels for orthonormalisation, Rayleigh-Ritz and residuals (gfx950).
//
// gram_f64 : G = X^T Y for tall n x p, n x q blocks.  Each 256-thread block owns a
//            64 x 64 tile of G and a chunk of rows; its four waves own 32 x 32
//            sub-tiles computed with v_mfma_f64_16x16x4f64 (a 2 x 2 grid of 16 x 16
//            accumulators per wave).  Chunk partials go to scratch and are summed
//            in chunk order by a second kernel: no atomics, bitwise reproducible.
// gemm_f64 : Y = X M + beta Y with M small (p x q); same tile shape, the MFMA
//            reduction runs over p.
// Complex Hermitian blocks use real views: a complex n x p block with leading
// dimension ld is a real n x 2p block with leading dimension 2 ld, and
//   X^H Y  = (Gr[2i,2j] + Gr[2i+1,2j+1]) + i (Gr[2i,2j+1] - Gr[2i+1,2j])  with Gr = Xr^T Yr,
//   X M    = Xr Mr  with Mr[2k,2j] = Re M, Mr[2k,2j+1] = Im M, Mr[2k+1,2j] = -Im M,
//            Mr[2k+1,2j+1] = Re M.
#include "internal.h"

namespace afsi {

typedef double d4 __attribute__((ext_vector_type(4)));

// MFMA 16x16x4 f64 operand layout: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16];
// accumulator element e of lane l is D[l / 16 + 4 e][l % 16] (rows interleaved by 4).
__device__ inline d4 mfma16x16x4(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(256) void gram_f64_kernel(const double *__restrict__ X, int64_t ldx,
                                                       const double *__restrict__ Y, int64_t ldy,
                                                       int64_t n, int p, int q,
                                                       int64_t rows_per_chunk,
                                                       double *__restrict__ ws) {
    const int tiles_j = (q + 63) / 64;
    const int ti = blockIdx.x / tiles_j, tj = blockIdx.x % tiles_j;
    const int chunk = blockIdx.y;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i0 = ti * 64 + (w >> 1) * 32, j0 = tj * 64 + (w & 1) * 32;
    const int lk = lane >> 4, lc = lane & 15;
    const int64_t r0 = (int64_t)chunk * rows_per_chunk;
    const int64_t r1 = min(n, r0 + rows_per_chunk);
    const int ca0 = i0 + lc, ca1 = i0 + 16 + lc, cb0 = j0 + lc, cb1 = j0 + 16 + lc;
    const bool va0 = ca0 < p, va1 = ca1 < p, vb0 = cb0 < q, vb1 = cb1 < q;
    d4 acc00 = {0, 0, 0, 0}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
#pragma unroll 4
    for (int64_t r = r0; r < r1; r += 4) {
        const int64_t row = r + lk;
        const bool rv = row < r1;
        const double *xr = X + row * ldx;
        const double *yr = Y + row * ldy;
        const double a0 = (rv && va0) ? xr[ca0] : 0.0;
        const double a1 = (rv && va1) ? xr[ca1] : 0.0;
        const double b0 = (rv && vb0) ? yr[cb0] : 0.0;
        const double b1 = (rv && vb1) ? yr[cb1] : 0.0;
        acc00 = mfma16x16x4(a0, b0, acc00);
        acc01 = mfma16x16x4(a0, b1, acc01);
        acc10 = mfma16x16x4(a1, b0, acc10);
        acc11 = mfma16x16x4(a1, b1, acc11);
    }
    double *out = ws + (int64_t)chunk * p * q;
    const d4 accs[4] = {acc00, acc01, acc10, acc11};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int gi0 = i0 + (t >> 1) * 16 + lk;
        const int gj = j0 + (t & 1) * 16 + lc;
        if (gj >= q) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (gi0 + 4 * e < p) out[(int64_t)(gi0 + 4 * e) * q + gj] = accs[t][e];
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
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t r0 = (int64_t)blockIdx.x * 64 + (w >> 1) * 32;
    const int c0 = blockIdx.y * 64 + (w & 1) * 32;
    const int lk = lane >> 4, lc = lane & 15;
    const int64_t ra0 = r0 + lc, ra1 = r0 + 16 + lc;
    const bool va0 = ra0 < n, va1 = ra1 < n;
    const int cb0 = c0 + lc, cb1 = c0 + 16 + lc;
    const bool vb0 = cb0 < q, vb1 = cb1 < q;
    const double *x0 = X + ra0 * ldx, *x1 = X + ra1 * ldx;
    d4 acc00 = {0, 0, 0, 0}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
#pragma unroll 4
    for (int k = 0; k < p; k += 4) {
        const int kk = k + lk;
        const bool kv = kk < p;
        const double a0 = (kv && va0) ? x0[kk] : 0.0;
        const double a1 = (kv && va1) ? x1[kk] : 0.0;
        const double *mr = M + (int64_t)kk * ldm;
        const double b0 = (kv && vb0) ? mr[cb0] : 0.0;
        const double b1 = (kv && vb1) ? mr[cb1] : 0.0;
        acc00 = mfma16x16x4(a0, b0, acc00);
        acc01 = mfma16x16x4(a0, b1, acc01);
        acc10 = mfma16x16x4(a1, b0, acc10);
        acc11 = mfma16x16x4(a1, b1, acc11);
    }
    const d4 accs[4] = {acc00, acc01, acc10, acc11};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int64_t gi0 = r0 + (t >> 1) * 16 + lk;
        const int gj = c0 + (t & 1) * 16 + lc;
        if (gj >= q) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t gi = gi0 + 4 * e;
            if (gi < n) {
                double *yp = Y + gi * ldy + gj;
                double v = alpha * accs[t][e];
                if (beta != 0.0) v = __builtin_fma(beta, *yp, v);
                *yp = v;
            }
        }
    }
}

// Complex helpers for the real-view formulation.
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

// Column sums of |AV - lambda V|^2 over a chunk of rows (V may be null: |AV|^2).
template <bool CPLX>
__global__ __launch_bounds__(256) void colsq_partial_kernel(const double *__restrict__ V, int64_t ldv,
                                                            const double *__restrict__ AV,
                                                            int64_t ldav,
                                                            const double *__restrict__ lam,
                                                            int64_t n, int q, int64_t rows_per_chunk,
                                                            double *__restrict__ ws) {
    __shared__ double red[4][64];
    const int r = threadIdx.x >> 6, c = threadIdx.x & 63;
    const int col = blockIdx.y * 64 + c;
    const int64_t i0 = (int64_t)blockIdx.x * rows_per_chunk;
    const int64_t i1 = min(n, i0 + rows_per_chunk);
    double s = 0.0;
    if (col < q) {
        const double l = lam ? lam[col] : 0.0;
        for (int64_t i = i0 + r; i < i1; i += 4) {
            if (CPLX) {
                const double *av = AV + 2 * (i * ldav + col);
                double dr = av[0], di = av[1];
                if (V) {
                    const double *v = V + 2 * (i * ldv + col);
                    dr = __builtin_fma(-l, v[0], dr);
                    di = __builtin_fma(-l, v[1], di);
                }
                s = __builtin_fma(dr, dr, s);
                s = __builtin_fma(di, di, s);
            } else {
                double d = AV[i * ldav + col];
                if (V) d = __builtin_fma(-l, V[i * ldv + col], d);
                s = __builtin_fma(d, d, s);
            }
        }
    }
    red[r][c] = s;
    __syncthreads();
    if (r == 0 && col < q) ws[(int64_t)blockIdx.x * q + col] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

__global__ void colsq_finalize_kernel(const double *__restrict__ ws, int nchunks, int q,
                                      bool take_sqrt, double *__restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += ws[(int64_t)c * q + j];
    out[j] = take_sqrt ? sqrt(s) : s;
}

__global__ void sum_kernel(const double *__restrict__ v, int q, double *__restrict__ out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double s = 0.0;
        for (int j = 0; j < q; ++j) s += v[j];
        out[0] = s;
    }
}

// ---------------------------------------------------------------- host launchers

static void chunking(int64_t n, int64_t tiles, int64_t gran, int64_t target_blocks, int64_t &rows,
                     int64_t &nchunks) {
    int64_t want = (target_blocks + tiles - 1) / tiles;
    const int64_t maxc = (n + 255) / 256;
    if (want > maxc) want = maxc;
    if (want < 1) want = 1;
    rows = (n + want - 1) / want;
    rows = (rows + gran - 1) / gran * gran;
    if (rows < gran) rows = gran;
    nchunks = (n + rows - 1) / rows;
    if (nchunks < 1) nchunks = 1;
}

void gram_f64(const double *X, int64_t ldx, const double *Y, int64_t ldy, int64_t n, int64_t p,
              int64_t q, double *G, int64_t ldg, hipStream_t s) {
    if (p == 0 || q == 0) return;
    const int64_t tiles = ((p + 63) / 64) * ((q + 63) / 64);
    int64_t rows, nchunks;
    chunking(n, tiles, 16, 2048, rows, nchunks);
    if (n == 0) nchunks = 1, rows = 16;
    double *ws = (double *)workspace(s).dev_reserve(SLOT_PARTIAL, sizeof(double) * nchunks * p * q);
    hipLaunchKernelGGL(gram_f64_kernel, dim3((unsigned)tiles, (unsigned)nchunks), dim3(256), 0, s,
                       X, ldx, Y, ldy, n, (int)p, (int)q, rows, ws);
    const int64_t tot = p * q;
    hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       ws, (int)nchunks, (int)p, (int)q, G, ldg);
    AFSI_HIP(hipGetLastError());
}

void gemm_f64(const double *X, int64_t ldx, const double *M, int64_t ldm, int64_t n, int64_t p,
              int64_t q, double alpha, double beta, double *Y, int64_t ldy, hipStream_t s) {
    if (n == 0 || q == 0) return;
    hipLaunchKernelGGL(gemm_f64_kernel, dim3((unsigned)((n + 63) / 64), (unsigned)((q + 63) / 64)),
                       dim3(256), 0, s, X, ldx, M, ldm, n, (int)p, (int)q, alpha, beta, Y, ldy);
    AFSI_HIP(hipGetLastError());
}

void gram_c128(const double *X, int64_t ldx, const double *Y, int64_t ldy, int64_t n, int64_t p,
               int64_t q, double *G, int64_t ldg, hipStream_t s) {
    if (p == 0 || q == 0) return;
    // real Gram of the real views into the top of a dedicated region, then combine
    const int64_t tiles = ((2 * p + 63) / 64) * ((2 * q + 63) / 64);
    int64_t rows, nchunks;
    chunking(n, tiles, 16, 2048, rows, nchunks);
    double *Gr = (double *)workspace(s).dev_reserve(SLOT_REALVIEW, sizeof(double) * 4 * p * q);
    double *ws = (double *)workspace(s).dev_reserve(SLOT_PARTIAL, sizeof(double) * nchunks * 4 * p * q);
    hipLaunchKernelGGL(gram_f64_kernel, dim3((unsigned)tiles, (unsigned)nchunks), dim3(256), 0, s,
                       X, 2 * ldx, Y, 2 * ldy, n, (int)(2 * p), (int)(2 * q), rows, ws);
    hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)((4 * p * q + 255) / 256)), dim3(256),
                       0, s, ws, (int)nchunks, (int)(2 * p), (int)(2 * q), Gr, 2 * q);
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

static void colsq(int dtype, const void *V, int64_t ldv, const void *AV, int64_t ldav,
                  const double *d_lambda, int64_t n, int64_t q, bool take_sqrt, double *d_out,
                  hipStream_t s) {
    if (q == 0) return;
    const int64_t ctiles = (q + 63) / 64;
    int64_t rows, nchunks;
    chunking(n, ctiles, 4, 1024, rows, nchunks);
    double *ws = (double *)workspace(s).dev_reserve(SLOT_PARTIAL, sizeof(double) * nchunks * q);
    const bool cplx = dtype == AFSI_C128;
    auto kern = cplx ? colsq_partial_kernel<true> : colsq_partial_kernel<false>;
    hipLaunchKernelGGL(kern, dim3((unsigned)nchunks, (unsigned)ctiles), dim3(256), 0, s,
                       (const double *)V, ldv, (const double *)AV, ldav, d_lambda, n, (int)q, rows,
                       ws);
    hipLaunchKernelGGL(colsq_finalize_kernel, dim3((unsigned)((q + 255) / 256)), dim3(256), 0, s, ws,
                       (int)nchunks, (int)q, take_sqrt, d_out);
    AFSI_HIP(hipGetLastError());
}

void residual_norms_dev(int dtype, const void *V, int64_t ldv, const void *AV, int64_t ldav,
                        const double *d_lambda, int64_t n, int64_t q, double *d_norms,
                        hipStream_t s) {
    colsq(dtype, V, ldv, AV, ldav, d_lambda, n, q, true, d_norms, s);
}

void frob2_dev(int dtype, const void *X, int64_t ldx, int64_t n, int64_t q, double *d_out,
               hipStream_t s) {
    // column sums of squares into d_out[1..q], total into d_out[0]
    colsq(dtype, nullptr, 0, X, ldx, nullptr, n, q, false, d_out + 1, s);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(64), 0, s, d_out + 1, (int)q, d_out);
    AFSI_HIP(hipGetLastError());
}

}  // namespace afsi
