// Internal declarations shared by the library's translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>

#include "../../include/afsi.h"
#include "host_linalg.h"

namespace afsi {

// ---------------------------------------------------------------- errors

void set_error(const char *fmt, ...);

struct Error {
    int status;
};

#define AFSI_REQUIRE(cond, ...)                                                                     \
    do {                                                                                            \
        if (!(cond)) {                                                                              \
            ::afsi::set_error(__VA_ARGS__);                                                         \
            throw ::afsi::Error{AFSI_E_INVALID};                                                    \
        }                                                                                           \
    } while (0)

#define AFSI_HIP(expr)                                                                              \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) {                                                                     \
            ::afsi::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__,     \
                              __LINE__);                                                            \
            throw ::afsi::Error{e_ == hipErrorOutOfMemory ? AFSI_E_NOMEM : AFSI_E_HIP};            \
        }                                                                                           \
    } while (0)

#define AFSI_FAIL(status, ...)                                                                      \
    do {                                                                                            \
        ::afsi::set_error(__VA_ARGS__);                                                             \
        throw ::afsi::Error{status};                                                                \
    } while (0)

// Runs `body` and converts errors into a status code.
template <class F>
int guarded(F &&body) {
    try {
        body();
        return AFSI_OK;
    } catch (const Error &e) {
        return e.status;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return AFSI_E_NOMEM;
    } catch (...) {
        set_error("unexpected C++ exception");
        return AFSI_E_HIP;
    }
}

// ---------------------------------------------------------------- dtypes

inline int elem_bytes(int dt) {
    switch (dt) {
    case AFSI_R64: return 8;
    case AFSI_R32: return 4;
    case AFSI_C128: return 16;
    case AFSI_C64: return 8;
    }
    return 0;
}
inline bool is_complex(int dt) { return dt == AFSI_C128 || dt == AFSI_C64; }
inline bool is_fp64(int dt) { return dt == AFSI_R64 || dt == AFSI_C128; }

// ---------------------------------------------------------------- matrix

struct MatView {
    int64_t n;
    const int *rp;   // n + 1
    const int *ci;   // nnz
    const void *val; // nnz values of the requested precision
    // at least one entry per two rows lies within one column of the diagonal: the
    // Clenshaw step stages each workgroup's rows of the source block in LDS
    bool stage_near = false;
    // column-block width (bytes) of a product's passes over the dense block: 0 = whole
    // rows in one pass (see afsi_matrix_set_column_block)
    int64_t seg_bytes = 0;
    // median over rows of the largest |column - row| (the reach of a banded matrix)
    int64_t band = 0;
};

}  // namespace afsi

struct afsi_matrix_s {
    int device = 0;
    int64_t n = 0, nnz = 0;
    int32_t dtype = AFSI_R64;  // AFSI_R64 or AFSI_C128
    int *d_rp = nullptr;
    int *d_ci = nullptr;
    void *d_val64 = nullptr;
    void *d_val32 = nullptr;
    int64_t near_nnz = 0;  // entries with |column - row| <= 1
    int64_t seg_bytes = 0; // column-block width of the products (0 = whole rows)
    int64_t band = 0;      // median over rows of the largest |column - row|
    double lmin = 0, lmax = 0;
    bool has_bounds = false;
    std::mutex mu;
};

namespace afsi {

// Device values matching a block dtype (creates the FP32 copy on first use).
MatView matrix_view(afsi_matrix_t A, int block_dtype, hipStream_t stream);

// RAII: make `dev` current for the scope.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
};

// ---------------------------------------------------------------- scratch

// Per-(device, stream) growable device scratch and pinned host staging.  Slots
// are independent regions: kernel-internal partial sums (SLOT_PARTIAL), complex
// real-view temporaries (SLOT_REALVIEW), small matrices of an API call
// (SLOT_SMALL) and vectors (SLOT_VEC).  Growing a slot synchronises the stream.
enum { SLOT_PARTIAL = 0, SLOT_REALVIEW = 1, SLOT_SMALL = 2, SLOT_VEC = 3, SLOT_GATHER = 4,
       NUM_DEV_SLOTS = 5 };
struct Workspace {
    hipStream_t stream = nullptr;
    void *dev[NUM_DEV_SLOTS] = {};
    size_t dev_bytes[NUM_DEV_SLOTS] = {};
    void *host[2] = {};
    size_t host_bytes[2] = {};
    void *dev_reserve(int slot, size_t bytes);
    void *host_reserve(int slot, size_t bytes);
};
Workspace &workspace(hipStream_t stream);

// ---------------------------------------------------------------- kernels (clenshaw_*.hip)

// Batched step arguments: column groups with their own source block, flags and
// scalars (group g owns 16-byte row vectors [vec0, vec1)).
struct BatchArgs {
    int ngroups;
    int vec0[64], vec1[64];   // group g owns row vectors [vec0, vec1)
    int src[64], dst[64];     // 0 = X, 1 = P0, 2 = P1
    int has_v[64];
    double sigma[64], tau[64], alpha[64];
};

// Lane mappings of the grouped step kernel, in the order they are tried: X(VN, L) is
// VN 16-byte vectors per lane and L lanes per row, a row of VN * L vectors.  (A
// matrix with near-diagonal entries tries X(1, 64) first.)
#define AFSI_GROUPED_MAPPINGS(X)                                                                    \
    X(2, 64) X(4, 32) X(4, 64) X(3, 64) X(5, 64) X(3, 32) X(5, 32) X(2, 32) X(6, 64) X(8, 64)      \
    X(1, 64) X(1, 32) X(3, 16) X(1, 16) X(3, 8) X(1, 8) X(1, 4)


// Smallest row width, in 16-byte vectors, of at least p16 that the grouped kernel
// maps exactly, or -1 if p16 is wider than every mapping.
inline int64_t grouped_width_at_least(int64_t p16) {
    int64_t best = -1;
#define AFSI_GW(VN_, L_)                                                                            \
    if ((VN_) * (L_) >= p16 && (best < 0 || (VN_) * (L_) < best)) best = (VN_) * (L_);
    AFSI_GROUPED_MAPPINGS(AFSI_GW)
#undef AFSI_GW
    return best;
}

// Blocks of at most kNarrowMax elements per row that have no exact lane mapping run the
// one-lane-per-row kernel (the *_scalar entries take it for p <= kNarrowMax).
constexpr int kNarrowMax = 16;

// Grouped step: up to kGroupedMax slices with their own blocks, one launch.
constexpr int kGroupedMax = 32;
struct GroupArgs {
    int ngroups;
    int64_t npad;  // rows per slice rounded up to whole workgroups (set by the launcher)
    const void *X[kGroupedMax];
    void *P0[kGroupedMax], *P1[kGroupedMax];
    int64_t ldv[kGroupedMax];  // leading dimension in 16-byte vectors
    int src[kGroupedMax], dst[kGroupedMax], has_v[kGroupedMax];
    double sigma[kGroupedMax], tau[kGroupedMax], alpha[kGroupedMax];
};

#define AFSI_DECLARE_STEP_ENTRY(NAME)                                                               \
    void NAME##_step(const MatView &A, const void *src, const void *X, void *dst, int p16,          \
                     int64_t ldv, bool hv, bool hx, double sg, double ta, double al,               \
                     hipStream_t s);                                                                \
    void NAME##_batched(const MatView &A, const void *X, void *P0, void *P1, int p16, int64_t ldv,  \
                        const BatchArgs &args, hipStream_t s);                                      \
    void NAME##_scalar(const MatView &A, const void *src, const void *X, void *dst, int p,          \
                       int64_t ld, bool hv, bool hx, double sg, double ta, double al, hipStream_t s); \
    bool NAME##_grouped(const MatView &A, int p16, GroupArgs &args, hipStream_t s);
AFSI_DECLARE_STEP_ENTRY(clenshaw_r64)
AFSI_DECLARE_STEP_ENTRY(clenshaw_r32)
AFSI_DECLARE_STEP_ENTRY(clenshaw_c128)
AFSI_DECLARE_STEP_ENTRY(clenshaw_c64)

// ---------------------------------------------------------------- kernels (util.hip)

void launch_convert(const afsi_block &src, const afsi_block &dst, hipStream_t s);
void launch_gather_columns(const afsi_block &src, const int32_t *d_cols, int64_t count,
                           const afsi_block &dst, hipStream_t s);
void launch_to_f32(const double *src, float *dst, int64_t count, hipStream_t s);
// dst row i = src row d_perm[i], or with `inverse` dst row d_perm[i] = src row i (d_perm a
// device permutation of src.rows rows; same dtype and shape).
void launch_permute_rows(const afsi_block &src, const int64_t *d_perm, bool inverse,
                         const afsi_block &dst, hipStream_t s);

// ---------------------------------------------------------------- kernels (dense.hip)

// Real FP64: G (p x q, ldg) = X^T Y; scratch from workspace.  X == Y (same ld, p == q)
// takes the symmetric path: upper tiles only, lower triangle mirrored.
void gram_f64(const double *X, int64_t ldx, const double *Y, int64_t ldy, int64_t n, int64_t p,
              int64_t q, double *G, int64_t ldg, hipStream_t s);
// Real FP64: Y = alpha X M + beta Y.  upper: M is upper triangular (zeros below the
// diagonal are skipped, not read).
void gemm_f64(const double *X, int64_t ldx, const double *M, int64_t ldm, int64_t n, int64_t p,
              int64_t q, double alpha, double beta, double *Y, int64_t ldy, hipStream_t s,
              bool upper = false);
// Complex via real views.
void gram_c128(const double *X, int64_t ldx, const double *Y, int64_t ldy, int64_t n, int64_t p,
               int64_t q, double *G, int64_t ldg, hipStream_t s);
void gemm_c128(const double *X, int64_t ldx, const double *M, int64_t ldm, int64_t n, int64_t p,
               int64_t q, double alpha, double beta, double *Y, int64_t ldy, hipStream_t s,
               bool upper = false);
// norms[j] = || AV[:, j] - lambda[j] V[:, j] ||_2, device output (q doubles).
void residual_norms_dev(int dtype, const void *V, int64_t ldv, const void *AV, int64_t ldav,
                        const double *d_lambda, int64_t n, int64_t q, double *d_norms,
                        hipStream_t s);
// As residual_norms_host, with every device buffer in the library's fixed per-device
// scratch array (no allocation); rejects shapes that need more than it holds.
void residual_norms_noalloc(int dtype, const void *V, int64_t ldv, const void *AV, int64_t ldav,
                            const double *lambda, int64_t n, int64_t q, double *out,
                            hipStream_t s);
int64_t residual_noalloc_need(int64_t n, int64_t q);  // doubles of scratch for (n, q)
int64_t residual_noalloc_capacity();                   // doubles the scratch holds
// d_out[j] = Re sum_i conj(Z[i, j]) Y[i, j], device output (q doubles).  R64 or C128.
void column_dots_dev(int dtype, const void *Z, int64_t ldz, const void *Y, int64_t ldy, int64_t n,
                     int64_t q, double *d_out, hipStream_t s);
// ||X||_F^2 per column summed: device scalar.
void frob2_dev(int dtype, const void *X, int64_t ldx, int64_t n, int64_t q, double *d_out,
               hipStream_t s);

// ---------------------------------------------------------------- shared host drivers (api.cpp)

void filter_apply(afsi_matrix_t A, const double *coeffs, int degree, int dtype, const void *X,
                  void *Y, void *work, int64_t p, int64_t ld, hipStream_t s,
                  hipEvent_t *events = nullptr, int32_t *kind = nullptr);
void spmm_apply(afsi_matrix_t A, int dtype, const void *X, void *Y, int64_t p, int64_t ld,
                hipStream_t s);
void inner_dev(int dtype, const void *X, int64_t ldx, const void *Y, int64_t ldy, int64_t n,
               int64_t p, int64_t q, double *G, int64_t ldg, hipStream_t s);
void gemm_dev(int dtype, const void *X, int64_t ldx, const double *M, int64_t ldm, int64_t n,
              int64_t p, int64_t q, double alpha, double beta, void *Y, int64_t ldy, hipStream_t s,
              bool upper = false);
void project_out_dev(int dtype, const void *L, int64_t ldl, int64_t k, void *X, int64_t ldx,
                     int64_t n, int64_t p, hipStream_t s);
void orthonormalize_dev(int dtype, void *X, void *W, int64_t n, int64_t p, int64_t ld,
                        hipStream_t s, double *max_col_norm2);
void rayleigh_ritz_dev(afsi_matrix_t A, int dtype, const void *Q, void *V, void *AV, int64_t n,
                       int64_t p, int64_t ld, double *ritz, hipStream_t s);
// CholQR2 of X (work W) fused with Rayleigh-Ritz on the basis it defines, which is never
// formed; V and AV as rayleigh_ritz_dev.  V must differ from X and W; AV may be W.
void orthonormalize_rr_dev(afsi_matrix_t A, int dtype, void *X, void *W, void *V, void *AV,
                           int64_t n, int64_t p, int64_t ld, double *ritz, hipStream_t s,
                           double *max_col_norm2, double *orth_ms);
void residual_norms_host(int dtype, const void *V, int64_t ldv, const void *AV, int64_t ldav,
                         const double *lambda, int64_t n, int64_t q, double *out, hipStream_t s);
void lock_select(const double *ritz, int64_t p, const double *res, uint8_t *I, double a, double b,
                 double tau_abs, int64_t n_lock, int64_t *n_check_prev, uint8_t *lock, int *done);
void launch_scale(double *x, int64_t n, int64_t ld, int comp, double s, hipStream_t st);
void launch_fill_normal(double *x, int64_t n, int64_t p, int64_t ld, int comp, uint64_t seed,
                        hipStream_t st);
// Gather columns of src (n rows, ld) into dst columns [0, count) (ld ldd); synchronises s.
void gather_cols(int dtype, const void *src, int64_t n, int64_t ld, const int32_t *cols,
                 int64_t count, void *dst, int64_t ldd, hipStream_t s);
void batched_step(afsi_matrix_t A, int ngroups, const afsi_step_group *groups, int dtype,
                  const void *X, void *P0, void *P1, int64_t ptot, int64_t ld, hipStream_t s);
// Returns how many of the active slices the grouped kernel took (the others, with a
// width that has no exact lane mapping or unaligned blocks, ran one product each).
// kernel_launches (optional) receives the number of grouped-kernel launches.
int grouped_step(afsi_matrix_t A, int ngroups, const afsi_slice_blocks *slices, int dtype,
                 hipStream_t s, int *kernel_launches = nullptr);
void filter_batched(afsi_matrix_t A, int nslices, const afsi_slice_filter *slices, int dtype,
                    hipStream_t s);

// ---------------------------------------------------------------- host linear algebra
// host_cholesky_inverse, host_eigh: host_linalg.h (built without HIP, with OpenMP).
// host_eigh_or_throw raises AFSI_E_HIP when the tridiagonal QR does not converge.
void host_eigh_or_throw(int64_t p, bool cplx, const double *B, int64_t ldb, double *w, double *U,
                        int64_t ldu);

// ---------------------------------------------------------------- coefficients

void filter_coefficients(double lmin, double lmax, double a, double b, int kmax, int damping,
                         double m_exp, double *coeffs);
void step_params(const double *coeffs, int degree, int step, double l1, double l2,
                 afsi_step_group *g);
int select_degree(const double *ritz, int64_t p, int64_t e, const double *coeffs, int kmax,
                  double l1, double l2, double tau_a);

}  // namespace afsi
