// Bandwidth kernels: precision conversion of blocks and matrix values, column gather,
// row permutation.
#include "internal.h"

namespace afsi {

template <class S, class D>
__global__ void convert_kernel(const S *__restrict__ src, int64_t lds, D *__restrict__ dst,
                               int64_t ldd, int64_t rows, int64_t cols) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * cols) return;
    const int64_t i = idx / cols, j = idx % cols;
    dst[i * ldd + j] = (D)src[i * lds + j];
}

template <class T>
__global__ void gather_kernel(const T *__restrict__ src, int64_t lds, const int32_t *__restrict__ cols,
                              int64_t count, int comp, T *__restrict__ dst, int64_t ldd, int64_t rows) {
    // comp = scalars per element (1 real, 2 complex)
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per_row = count * comp;
    if (idx >= rows * per_row) return;
    const int64_t i = idx / per_row, r = idx % per_row;
    const int64_t t = r / comp, c = r % comp;
    dst[(i * ldd + t) * comp + c] = src[(i * lds + cols[t]) * comp + c];
}

// Row permutation: dst row i = src row perm[i] (gather) or dst row perm[i] = src row i
// (inverse: scatter), U the widest unit that divides every row, ld and base.
template <class U>
__global__ void permute_rows_kernel(const U *__restrict__ src, int64_t lds, U *__restrict__ dst,
                                    int64_t ldd, const int64_t *__restrict__ perm, int inverse,
                                    int64_t rows, int64_t units) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * units) return;
    const int64_t i = idx / units, c = idx % units;
    const int64_t pi = perm[i];
    const int64_t si = inverse ? i : pi, di = inverse ? pi : i;
    dst[di * ldd + c] = src[si * lds + c];
}

__global__ void to_f32_kernel(const double *__restrict__ src, float *__restrict__ dst, int64_t count) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < count) dst[idx] = (float)src[idx];
}

__global__ void scale_strided_kernel(double *__restrict__ x, int64_t n, int64_t ld, int comp,
                                     double s) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * comp) return;
    const int64_t i = idx / comp, c = idx % comp;
    x[i * ld * comp + c] *= s;
}

static unsigned blocks_for(int64_t count) { return (unsigned)((count + 255) / 256); }

// splitmix64 finaliser (Steele, Lea, Flood 2014) used as a counter-based generator.
__device__ inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
__device__ inline double unit_open(uint64_t r) { return ((r >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

// N(0,1) entries for element (i, j) of an n x p block, from counter (i * p + j): the
// value depends only on (seed, i, j, p), not on where the block is stored.
__global__ void fill_normal_kernel(double *__restrict__ x, int64_t n, int64_t p, int64_t ld,
                                   int comp, uint64_t seed) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * p) return;
    const int64_t i = idx / p, j = idx % p;
    const uint64_t base = mix64(seed) ^ (uint64_t)(idx * 4);
    for (int c = 0; c < comp; ++c) {
        const double u1 = unit_open(mix64(base + 2 * c)), u2 = unit_open(mix64(base + 2 * c + 1));
        double g = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
        if (comp == 2) g *= 0.7071067811865476;
        x[(i * ld + j) * comp + c] = g;
    }
}

void launch_fill_normal(double *x, int64_t n, int64_t p, int64_t ld, int comp, uint64_t seed,
                        hipStream_t st) {
    if (n * p == 0) return;
    hipLaunchKernelGGL(fill_normal_kernel, dim3((unsigned)((n * p + 255) / 256)), dim3(256), 0, st, x,
                       n, p, ld, comp, seed);
    AFSI_HIP(hipGetLastError());
}

// x[i * ld + 0..comp) *= s for i < n (one strided column; comp = 2 for complex).
void launch_scale(double *x, int64_t n, int64_t ld, int comp, double s, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(scale_strided_kernel, dim3(blocks_for(n * comp)), dim3(256), 0, st, x, n, ld,
                       comp, s);
    AFSI_HIP(hipGetLastError());
}

void launch_convert(const afsi_block &src, const afsi_block &dst, hipStream_t s) {
    const int comp = is_complex(src.dtype) ? 2 : 1;
    const int64_t rows = src.rows, cols = src.cols * comp;
    const int64_t lds = src.ld * comp, ldd = dst.ld * comp;
    if (rows * cols == 0) return;
    const bool s64 = is_fp64(src.dtype), d64 = is_fp64(dst.dtype);
    const unsigned g = blocks_for(rows * cols);
    if (s64 && d64)
        hipLaunchKernelGGL((convert_kernel<double, double>), dim3(g), dim3(256), 0, s,
                           (const double *)src.ptr, lds, (double *)dst.ptr, ldd, rows, cols);
    else if (s64 && !d64)
        hipLaunchKernelGGL((convert_kernel<double, float>), dim3(g), dim3(256), 0, s,
                           (const double *)src.ptr, lds, (float *)dst.ptr, ldd, rows, cols);
    else if (!s64 && d64)
        hipLaunchKernelGGL((convert_kernel<float, double>), dim3(g), dim3(256), 0, s,
                           (const float *)src.ptr, lds, (double *)dst.ptr, ldd, rows, cols);
    else
        hipLaunchKernelGGL((convert_kernel<float, float>), dim3(g), dim3(256), 0, s,
                           (const float *)src.ptr, lds, (float *)dst.ptr, ldd, rows, cols);
    AFSI_HIP(hipGetLastError());
}

void launch_gather_columns(const afsi_block &src, const int32_t *d_cols, int64_t count,
                           const afsi_block &dst, hipStream_t s) {
    const int comp = is_complex(src.dtype) ? 2 : 1;
    const int64_t tot = src.rows * count * comp;
    if (tot == 0) return;
    if (is_fp64(src.dtype))
        hipLaunchKernelGGL((gather_kernel<double>), dim3(blocks_for(tot)), dim3(256), 0, s,
                           (const double *)src.ptr, src.ld, d_cols, count, comp, (double *)dst.ptr,
                           dst.ld, src.rows);
    else
        hipLaunchKernelGGL((gather_kernel<float>), dim3(blocks_for(tot)), dim3(256), 0, s,
                           (const float *)src.ptr, src.ld, d_cols, count, comp, (float *)dst.ptr,
                           dst.ld, src.rows);
    AFSI_HIP(hipGetLastError());
}

void launch_permute_rows(const afsi_block &src, const int64_t *d_perm, bool inverse,
                         const afsi_block &dst, hipStream_t s) {
    const int64_t eb = elem_bytes(src.dtype);
    const int64_t row = src.cols * eb, lds = src.ld * eb, ldd = dst.ld * eb;
    if (src.rows == 0 || row == 0) return;
    const uintptr_t a = reinterpret_cast<uintptr_t>(src.ptr) | reinterpret_cast<uintptr_t>(dst.ptr);
    auto fits = [&](int64_t u) { return row % u == 0 && lds % u == 0 && ldd % u == 0 && a % u == 0; };
    const int64_t u = fits(16) ? 16 : (fits(8) ? 8 : 4);
    const int64_t units = row / u, tot = src.rows * units;
    if (u == 16)
        hipLaunchKernelGGL((permute_rows_kernel<uint4>), dim3(blocks_for(tot)), dim3(256), 0, s,
                           (const uint4 *)src.ptr, lds / 16, (uint4 *)dst.ptr, ldd / 16, d_perm,
                           (int)inverse, src.rows, units);
    else if (u == 8)
        hipLaunchKernelGGL((permute_rows_kernel<uint2>), dim3(blocks_for(tot)), dim3(256), 0, s,
                           (const uint2 *)src.ptr, lds / 8, (uint2 *)dst.ptr, ldd / 8, d_perm,
                           (int)inverse, src.rows, units);
    else
        hipLaunchKernelGGL((permute_rows_kernel<uint32_t>), dim3(blocks_for(tot)), dim3(256), 0, s,
                           (const uint32_t *)src.ptr, lds / 4, (uint32_t *)dst.ptr, ldd / 4, d_perm,
                           (int)inverse, src.rows, units);
    AFSI_HIP(hipGetLastError());
}

void launch_to_f32(const double *src, float *dst, int64_t count, hipStream_t s) {
    if (count == 0) return;
    hipLaunchKernelGGL(to_f32_kernel, dim3(blocks_for(count)), dim3(256), 0, s, src, dst, count);
    AFSI_HIP(hipGetLastError());
}

}  // namespace afsi
