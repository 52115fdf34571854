/* Plain CSR sparse-matrix x dense-block product for the CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY: part of the oracle that the HIP library is checked
 * against.  Computes C = A * B for a square CSR matrix A (n x n) and a row-major
 * dense block B (n x p, leading dimension p); the textbook row-wise CSR product
 * that Section 3.3.1 takes as its starting point.  One OpenMP loop over rows,
 * no blocking, no reordering of the per-row sum.  Small products run on one thread
 * (a team costs more than it saves there, and far more on a loaded host); the
 * threading never changes a result.
 */
#include <stdint.h>

void oracle_spmm_f64(int64_t n, const int64_t *row_ptr, const int32_t *col,
                     const double *val, const double *B, int64_t p, double *C)
{
    #pragma omp parallel for schedule(static) if (n * p >= 65536)
    for (int64_t i = 0; i < n; ++i) {
        double *c = C + i * p;
        for (int64_t t = 0; t < p; ++t) c[t] = 0.0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const double a = val[e];
            const double *b = B + (int64_t)col[e] * p;
            for (int64_t t = 0; t < p; ++t) c[t] += a * b[t];
        }
    }
}

/* Complex version: val, B and C hold interleaved (re, im) pairs. */
void oracle_spmm_c128(int64_t n, const int64_t *row_ptr, const int32_t *col,
                      const double *val, const double *B, int64_t p, double *C)
{
    #pragma omp parallel for schedule(static) if (n * p >= 32768)
    for (int64_t i = 0; i < n; ++i) {
        double *c = C + 2 * i * p;
        for (int64_t t = 0; t < 2 * p; ++t) c[t] = 0.0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const double ar = val[2 * e], ai = val[2 * e + 1];
            const double *b = B + 2 * (int64_t)col[e] * p;
            for (int64_t t = 0; t < p; ++t) {
                const double br = b[2 * t], bi = b[2 * t + 1];
                c[2 * t] += ar * br - ai * bi;
                c[2 * t + 1] += ar * bi + ai * br;
            }
        }
    }
}

int oracle_num_threads(void)
{
    int nt = 1;
    #pragma omp parallel
    {
        #pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            nt = omp_get_num_threads();
#endif
        }
    }
    return nt;
}

/* Thread count of the products above (measurement only: single-thread baselines). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}
