// Column reductions for the residual step (Algorithm 4), the shifted Cholesky QR and
// the eigenvalue-count estimate (Section 3.4).
//
// colsq: per column j, sum_i |AV[i, j] - lambda_j V[i, j]|^2 (V may be absent: |AV|^2).
// Each block owns 64 columns and a chunk of rows; its 4 row-lanes are combined in a
// fixed order in LDS, and the chunk partials are added in chunk order by a second
// kernel, so results are reproducible for fixed (n, q).
#include "internal.h"

namespace afsi {

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
    if (r == 0 && col < q)
        ws[(int64_t)blockIdx.x * q + col] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

// coldot: per column j, Re sum_i conj(Z[i, j]) Y[i, j]; same chunking and fixed-order
// combination as colsq.
template <bool CPLX>
__global__ __launch_bounds__(256) void coldot_partial_kernel(const double *__restrict__ Z, int64_t ldz,
                                                             const double *__restrict__ Y, int64_t ldy,
                                                             int64_t n, int q, int64_t rows_per_chunk,
                                                             double *__restrict__ ws) {
    __shared__ double red[4][64];
    const int r = threadIdx.x >> 6, c = threadIdx.x & 63;
    const int col = blockIdx.y * 64 + c;
    const int64_t i0 = (int64_t)blockIdx.x * rows_per_chunk;
    const int64_t i1 = min(n, i0 + rows_per_chunk);
    double s = 0.0;
    if (col < q) {
        for (int64_t i = i0 + r; i < i1; i += 4) {
            if (CPLX) {
                const double *z = Z + 2 * (i * ldz + col);
                const double *y = Y + 2 * (i * ldy + col);
                s = __builtin_fma(z[0], y[0], s);
                s = __builtin_fma(z[1], y[1], s);
            } else {
                s = __builtin_fma(Z[i * ldz + col], Y[i * ldy + col], s);
            }
        }
    }
    red[r][c] = s;
    __syncthreads();
    if (r == 0 && col < q)
        ws[(int64_t)blockIdx.x * q + col] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
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

// Partial sums colsq needs for (n, q): nchunks * q doubles.
static int64_t colsq_partials(int64_t n, int64_t q) {
    int64_t rows, nchunks;
    chunking(n, (q + 63) / 64, 4, 1024, rows, nchunks);
    return nchunks * q;
}

// colsq with its chunk partials in `ws` (colsq_partials(n, q) doubles, or NULL: the
// stream's workspace).
static void colsq(int dtype, const void *V, int64_t ldv, const void *AV, int64_t ldav,
                  const double *d_lambda, int64_t n, int64_t q, bool take_sqrt, double *d_out,
                  hipStream_t s, double *ws = nullptr) {
    if (q == 0) return;
    const int64_t ctiles = (q + 63) / 64;
    int64_t rows, nchunks;
    chunking(n, ctiles, 4, 1024, rows, nchunks);
    if (!ws) ws = (double *)workspace(s).dev_reserve(SLOT_PARTIAL, sizeof(double) * nchunks * q);
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

// ---------------------------------------------------------------- allocation-free residuals
//
// Device memory of afsi_residual_norms_noalloc: the eigenvalues, the chunk partials and
// the norms of one call, kNoallocDoubles doubles in all.  Each device holds its own copy
// of this array from the library's load until the process ends; host code must address
// it through the pointer hipGetSymbolAddress returns on that device, never by its name.
constexpr int64_t kNoallocDoubles = int64_t(1) << 17;  // 1 MiB
static __device__ __align__(256) double scratch[kNoallocDoubles];

static std::mutex g_scratch_mu;
static double *g_scratch_ptr[256];  // per device ordinal, set on first use

static double *scratch_ptr(int dev) {
    AFSI_REQUIRE(dev >= 0 && dev < 256, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        AFSI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        AFSI_REQUIRE(p != nullptr, "no device address for the residual scratch");
        g_scratch_ptr[dev] = (double *)p;
    }
    return g_scratch_ptr[dev];
}

int64_t residual_noalloc_need(int64_t n, int64_t q) { return 2 * q + colsq_partials(n, q); }
int64_t residual_noalloc_capacity() { return kNoallocDoubles; }

void residual_norms_noalloc(int dtype, const void *V, int64_t ldv, const void *AV, int64_t ldav,
                            const double *lambda, int64_t n, int64_t q, double *out,
                            hipStream_t s) {
    if (q == 0) return;
    const int64_t need = residual_noalloc_need(n, q);
    AFSI_REQUIRE(need <= kNoallocDoubles,
                 "%lld columns of %lld rows need %lld doubles of scratch; the allocation-free "
                 "residual call holds %lld", (long long)q, (long long)n, (long long)need,
                 (long long)kNoallocDoubles);
    int dev = 0;
    AFSI_HIP(hipGetDevice(&dev));
    double *d_lam = scratch_ptr(dev), *d_out = d_lam + q, *ws = d_lam + 2 * q;
    AFSI_HIP(hipMemcpyAsync(d_lam, lambda, sizeof(double) * q, hipMemcpyHostToDevice, s));
    colsq(dtype, V, ldv, AV, ldav, d_lam, n, q, true, d_out, s, ws);
    AFSI_HIP(hipMemcpyAsync(out, d_out, sizeof(double) * q, hipMemcpyDeviceToHost, s));
    AFSI_HIP(hipStreamSynchronize(s));
}

void column_dots_dev(int dtype, const void *Z, int64_t ldz, const void *Y, int64_t ldy, int64_t n,
                     int64_t q, double *d_out, hipStream_t s) {
    if (q == 0) return;
    const int64_t ctiles = (q + 63) / 64;
    int64_t rows, nchunks;
    chunking(n, ctiles, 4, 1024, rows, nchunks);
    double *ws = (double *)workspace(s).dev_reserve(SLOT_PARTIAL, sizeof(double) * nchunks * q);
    auto kern = dtype == AFSI_C128 ? coldot_partial_kernel<true> : coldot_partial_kernel<false>;
    hipLaunchKernelGGL(kern, dim3((unsigned)nchunks, (unsigned)ctiles), dim3(256), 0, s,
                       (const double *)Z, ldz, (const double *)Y, ldy, n, (int)q, rows, ws);
    hipLaunchKernelGGL(colsq_finalize_kernel, dim3((unsigned)((q + 255) / 256)), dim3(256), 0, s, ws,
                       (int)nchunks, (int)q, false, d_out);
    AFSI_HIP(hipGetLastError());
}

void frob2_dev(int dtype, const void *X, int64_t ldx, int64_t n, int64_t q, double *d_out,
               hipStream_t s) {
    // column sums of squares into d_out[1..q], total into d_out[0]
    colsq(dtype, nullptr, 0, X, ldx, nullptr, n, q, false, d_out + 1, s);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(64), 0, s, d_out + 1, (int)q, d_out);
    AFSI_HIP(hipGetLastError());
}

}  // namespace afsi
