/*
 * afsi.h -- C ABI of the MI355X (gfx950) library for adaptive Chebyshev-filtered
 * subspace iteration on sparse Hermitian matrices.
 *
 * The method is the one of "Adaptive Polynomial Filtering for Hermitian Interior
 * Eigenproblems: Convergence Analysis" (Xu, Ni, Li, Zhang): find every eigenpair
 * (lambda, v) of a Hermitian A with lambda in [a, b] (Section 1, eq. (ori_problem))
 * by subspace iteration on rho(A), where rho is a damped Chebyshev expansion of
 * the interval's step function evaluated by Clenshaw's recurrence.
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Return value: AFSI_OK (0) or a negative afsi_status.  No C++ exception
 *    crosses this boundary.  afsi_last_error() gives a message for the last
 *    failure on the calling thread.
 *  - Dense blocks (afsi_block) are caller-owned DEVICE memory, row-major: element
 *    (i, j) is at ptr + i*ld + j (in elements, complex elements count once),
 *    ld >= cols.  The library never frees or reallocates them.
 *  - Matrices (afsi_matrix_t) are library-owned device copies made from host CSR.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *    that only produce device data are asynchronous on that stream.  Calls that
 *    write host outputs synchronise that stream before returning.
 *  - Host input arrays are read before the call returns; the caller keeps
 *    ownership.
 *  - Element types: real FP64 (R64), real FP32 (R32), complex FP64 (C128, pairs
 *    of doubles re,im) and complex FP32 (C64, pairs of floats).  The filter runs
 *    in the block's type; orthonormalisation, Rayleigh-Ritz and residuals are
 *    FP64 (R64 or C128) only.
 *  - Calls that overlap on one device must use different blocks; the library
 *    keeps internal scratch per stream.
 */
#ifndef AFSI_H
#define AFSI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AFSI_OK = 0,
    AFSI_E_INVALID = -1,   /* bad argument: shape, dtype, CSR structure, a >= b ... */
    AFSI_E_NOMEM = -2,     /* device or host allocation failed */
    AFSI_E_HIP = -3,       /* a HIP runtime call failed */
    AFSI_E_NOT_HPD = -4,   /* Gram matrix not positive definite even after the shift */
    AFSI_E_BOUNDS = -5,    /* filter output grew: spectral bounds do not enclose A */
    AFSI_E_NOCONV = -6,    /* iteration limit reached (partial results returned), or the
                              host eigensolver's QR iteration did not converge */
    AFSI_E_BUSY = -7,      /* serving: request does not fit the device budget now */
    AFSI_E_NODEVICE = -8   /* no usable gfx950 device */
} afsi_status;

typedef enum { AFSI_R64 = 0, AFSI_R32 = 1, AFSI_C128 = 2, AFSI_C64 = 3 } afsi_dtype;

typedef enum {
    AFSI_DAMP_NONE = 0,     /* plain truncated Chebyshev series */
    AFSI_DAMP_JACKSON = 1,  /* Jackson factors d^J_{j,k} (Section 2.2) */
    AFSI_DAMP_LANCZOS = 2   /* exponent-m Lanczos factors, eq. (m_Lanczos_damping) */
} afsi_damping;

typedef struct afsi_matrix_s *afsi_matrix_t;

/* A dense device block, row-major, `rows` x `cols` with row stride `ld` elements. */
typedef struct {
    void *ptr;
    int64_t rows;
    int64_t cols;
    int64_t ld;
    int32_t dtype; /* afsi_dtype */
} afsi_block;

/* ------------------------------------------------------------------ utilities */

const char *afsi_last_error(void);   /* thread-local; never NULL */
const char *afsi_version(void);
/* Number of gfx950 devices visible, or a negative status. */
int afsi_device_count(void);

/* ------------------------------------------------------------------ matrices */

/*
 * Copy a square Hermitian CSR matrix from host memory to device `device`.  CSR is the
 * storage in which Section 3.3.1 keeps the sparse A of the filter's products (the
 * row-pointer / column-index / value arrays its SpMM traverses row by row); the
 * device copy is what every product of the filter, Rayleigh-Ritz and the residual
 * step reads.
 *   row_ptr[n+1] (int64, row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz),
 *   col_idx[nnz] (int32, strictly increasing within each row, in [0, n)),
 *   vals[nnz]    (val_dtype AFSI_R64: double; AFSI_C128: interleaved re,im doubles).
 * The structure is validated (AFSI_E_INVALID on violation); Hermitian symmetry is
 * the caller's promise and is not checked.  nnz must be below 2^31.
 * An FP32 copy of the values is made on first use by an FP32 / C64 filter.
 * Spectral bounds start unset (see afsi_set_spectral_bounds).
 */
int afsi_matrix_create_csr(int device, int64_t n, int64_t nnz, const int64_t *row_ptr,
                           const int32_t *col_idx, const void *vals, int32_t val_dtype,
                           afsi_matrix_t *out);
int afsi_matrix_destroy(afsi_matrix_t A);

/*
 * Column blocks of the dense operand (the first loop of Section 3.3.1's MaSpMM, over
 * column blocks of width T_k, each reused while every row of A passes over it).  With
 * `bytes` > 0 every product of a row-major block wider than `bytes` runs as one pass of
 * A per column block of that many bytes, so the gathered rows of one block stay in the
 * device's memory-side cache; results are bit-identical to whole-row passes.  0 = whole
 * rows in one pass, the default (whole rows measured as fast or faster on the
 * workloads here: blocks re-read A once per block).  `bytes` must be 0 or a width the
 * library's grouped kernel maps (64, 128, 256, 384, 512, 768, 1024, ... bytes;
 * AFSI_E_INVALID otherwise).
 */
int afsi_matrix_set_column_block(afsi_matrix_t A, int64_t bytes);
int afsi_matrix_get_column_block(afsi_matrix_t A, int64_t *bytes);
/*
 * Locality ordering of the unknowns (host-side; Section 3.3.1: the filter's cost is the
 * SpMM, and its speed is set by how often the gathered rows of the dense operand are
 * found in cache).  The eigenvalues of P A P^T are those of A and its eigenvectors are
 * P times A's, so a solve may run on a reordered matrix with blocks in the new order.
 *
 * afsi_grid_order: the pencil ordering of an nx x ny x nz grid whose natural row index is
 * (x ny + y) nz + z.  The (y, z) plane is cut into tiles of ty x tz points (the last tile
 * of a side may be smaller); tiles are taken one after another (y tiles outer), and each
 * tile runs along all of x with its (y, z) points in natural order at every x.  Then the
 * +-x neighbours of a point sit ty tz rows away, so for a 7-point stencil almost every
 * neighbour lies within a constant row distance (the tile's cross-section) instead of
 * ny nz rows; the products pick that distance up from the matrix and run each XCD on
 * rows that many positions apart, keeping the reused rows in its own L2.  fold_x != 0
 * (for a periodic x axis) takes x in the order 0, nx-1, 1, nx-2, ... along every pencil,
 * so the wrap-around neighbours are adjacent and every +-x neighbour is at most two
 * cross-sections away.  Writes perm[new] = old for all nx ny nz points (caller-allocated
 * host array).  AFSI_E_INVALID for negative sizes or tiles smaller than 1.
 */
int afsi_grid_order(int64_t nx, int64_t ny, int64_t nz, int64_t ty, int64_t tz, int32_t fold_x,
                    int64_t *perm);

/*
 * B = P A P^T in CSR on the host: B[i][j] = A[perm[i]][perm[j]], i.e. row i of B is row
 * perm[i] of A with column c renamed to the position of c in perm, entries sorted by the
 * new column.  Same array formats as afsi_matrix_create_csr (which then takes B);
 * outputs are caller-allocated: out_row_ptr[n+1], out_col_idx[nnz], out_vals[nnz].
 * perm must hold each of 0..n-1 exactly once (AFSI_E_INVALID otherwise, and for the
 * structural violations afsi_matrix_create_csr rejects).
 */
int afsi_csr_permute(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                     const void *vals, int32_t val_dtype, const int64_t *perm, int64_t *out_row_ptr,
                     int32_t *out_col_idx, void *out_vals);

/*
 * Device row permutation of a block: dst row i = src row perm[i] (inverse = 0: a block
 * in A's order to P A P^T's), or dst row perm[i] = src row i (inverse != 0: back).
 * perm: host array of src->rows entries holding each of 0..rows-1 once (validated,
 * then copied to the device on `stream`); src and dst: same shape and dtype, not
 * overlapping.  Synchronises `stream`.
 */
int afsi_permute_rows(const afsi_block *src, const int64_t *perm, int32_t inverse, afsi_block *dst,
                      void *stream);

/* n, nnz, value dtype (AFSI_R64 or AFSI_C128), device ordinal. Any output may be NULL. */
int afsi_matrix_info(afsi_matrix_t A, int64_t *n, int64_t *nnz, int32_t *dtype, int32_t *device);

/*
 * Interval [lmin, lmax] enclosing the spectrum of A; defines the affine map
 * l(x) = (2x - lmax - lmin) / (lmax - lmin) of Section 2.2.  Needs lmin < lmax.
 */
int afsi_set_spectral_bounds(afsi_matrix_t A, double lmin, double lmax);
int afsi_get_spectral_bounds(afsi_matrix_t A, double *lmin, double *lmax);

/*
 * Estimate [lmin, lmax] by `steps` Lanczos steps with full reorthogonalisation
 * from a start vector drawn from `seed` (Section 3.4 says "a few iterations").
 * The extreme Ritz values are widened by their residual bound plus 1e-3 of the
 * spread.  Stores the result in A (as afsi_set_spectral_bounds) and returns it.
 */
int afsi_estimate_spectral_bounds(afsi_matrix_t A, int steps, uint64_t seed, void *stream,
                                  double *lmin, double *lmax);

/* ------------------------------------------------------------------ filter */

/*
 * Filter coefficients a_j = c_j d_{j,kmax}, j = 0..kmax, written to coeffs[kmax+1]
 * (host).  c_j from eq. (c_j) with alpha = arccos l(a), beta = arccos l(b), l(.)
 * clipped into [-1, 1] (an interval reaching past the bounds is the extreme
 * problem of Section 1); d_{j,kmax} Jackson, exponent-m Lanczos (m_exp >= 0) or
 * none (Section 2.2).  A truncated filter of degree k^(i) <= kmax uses the first
 * k^(i)+1 entries, as in eq. (AdaPolySI).  Pure host function.
 */
int afsi_filter_coefficients(double lmin, double lmax, double a, double b, int kmax,
                             int32_t damping, double m_exp, double *coeffs);

/*
 * Y = sum_{j=0}^{degree} coeffs[j] T_j(l(A)) X  (Algorithm 2, Clenshaw's recurrence,
 * in the division-free form b_{k+1} = b_{k+2} = 0, b_j = a_j X + 2 l(A) b_{j+1}
 * - b_{j+2}, Y = a_0 X + l(A) b_1 - b_2), using exactly `degree` products with A.
 *   coeffs : host, degree+1 doubles (cast to FP32 for R32 / C64 blocks).
 *   X, Y, work : n x p blocks of one dtype; R64/R32 for a real A, C128/C64 for a
 *   complex A.  Y and work are overwritten; none of X, Y, work may overlap.
 * Needs spectral bounds on A and degree >= 1.  Asynchronous on `stream`.
 */
int afsi_filter_block(afsi_matrix_t A, const double *coeffs, int degree, const afsi_block *X,
                      afsi_block *Y, afsi_block *work, void *stream);

/*
 * afsi_filter_block with a HIP event recorded on `stream` before each product
 * and after the last (per-kernel timing without a profiler).  step_ms[degree]
 * (host) receives each product's duration; step_kind[degree] (host, may be NULL)
 * receives bit 0 = reads the previous block in place, bit 1 = adds the alpha X
 * term.  Synchronises `stream`.
 */
int afsi_filter_block_profiled(afsi_matrix_t A, const double *coeffs, int degree,
                               const afsi_block *X, afsi_block *Y, afsi_block *work, void *stream,
                               float *step_ms, int32_t *step_kind);

/*
 * Eigenvalue count of A in [a, b] by stochastic trace estimation (Section 3.4).  The
 * damped filter rho(x) = sum_{j=0}^{degree} c_j d_{j,degree} T_j(l(x)) of eq.
 * (AdaPolySI) at its full degree approximates the spectral projector onto [a, b], so
 * the count is close to tr rho(A), estimated by the mean of Re z_i^H rho(A) z_i over
 * the m columns z_i of Z (Hutchinson's estimator).  The caller draws Z (for example
 * independent +-1 entries), so the result does not depend on a generator inside the
 * library.  The paper then sizes the block as p = ceil(mu * estimate), mu = 1.8.
 *   Z         : n x m device block, R64 for a real A, C128 for a complex A; read only.
 *   Y, work   : n x m device blocks of Z's dtype, overwritten (Y = rho(A) Z).
 *   damping   : AFSI_DAMP_*; m_exp the Lanczos exponent (paper: 0.5).
 *   per_probe : host, m doubles: Re z_i^H rho(A) z_i.
 *   estimate  : host: their mean.
 * Needs spectral bounds on A, a < b, degree >= 1, m >= 1; Z, Y and work must not
 * overlap.  Errors: AFSI_E_INVALID.  Synchronises `stream`.
 */
int afsi_estimate_eigencount(afsi_matrix_t A, double a, double b, int degree, int32_t damping,
                             double m_exp, const afsi_block *Z, afsi_block *Y, afsi_block *work,
                             double *per_probe, double *estimate, void *stream);

/*
 * Block width from an eigenvalue-count estimate (Section 3.4: the subspace must hold
 * at least the e eigenvalues of [a, b], so p = ceil(mu * e~) with mu > 0; Section 4
 * uses mu = 1.8).  *p_out = ceil(mu * estimate), clipped to [1, n].  Needs mu > 0,
 * n >= 1 and a finite estimate (a negative estimate gives 1).  Pure host function.
 */
int afsi_block_size(double estimate, double mu, int64_t n, int64_t *p_out);

/* Y = A X (one sparse x dense-block product). X and Y as for afsi_filter_block. */
int afsi_spmm(afsi_matrix_t A, const afsi_block *X, afsi_block *Y, void *stream);

/*
 * One Clenshaw product for a column group of concatenated blocks:
 *   dst = sigma * A * src + tau * src - (has_v ? dst : 0) + alpha * X
 * on columns [col0, col0 + ncols) of the buffers, with src selected from
 * {X, P0, P1} and dst from {P0, P1}.  afsi_clenshaw_step_params fills
 * (src, dst, has_v, sigma, tau, alpha) for product number `step` (0..degree-1)
 * of a degree-`degree` filter so that the last product writes Y to
 * P[(degree-1) % 2].
 */
typedef struct {
    int64_t col0, ncols;
    int32_t src;    /* 0 = X, 1 = P0, 2 = P1 */
    int32_t dst;    /* 1 = P0, 2 = P1 (never equal to src) */
    int32_t has_v;  /* subtract the previous contents of dst (b_{j+2}) */
    int32_t active; /* 0: leave these columns untouched */
    double sigma, tau, alpha;
} afsi_step_group;

int afsi_clenshaw_step_params(const double *coeffs, int degree, int step, double l1, double l2,
                              afsi_step_group *g);

/*
 * Batched step for spectrum slices of one matrix (Section 1: the interval of interest
 * split into slices, each solved by its own filter; here several slices' Clenshaw
 * recurrences of Algorithm 2 advance together and A is read once per product).
 * X, P0, P1: n x ptot blocks of one dtype.  Groups must
 * not overlap; at most 64.  Columns outside every active group are untouched.
 * Per column the arithmetic is identical to afsi_filter_block's, so a slice gives
 * bit-identical results alone or batched.
 */
int afsi_clenshaw_step_batched(afsi_matrix_t A, int ngroups, const afsi_step_group *groups,
                               const afsi_block *X, afsi_block *P0, afsi_block *P1, void *stream);

/*
 * Grouped step for spectrum slices of one matrix (Section 1's slicing; one product of
 * Algorithm 2's recurrence per slice) that keep their blocks apart: one
 * product of every active slice, each on its own n x step.ncols blocks X, P0, P1
 * (row-major, leading dimension ld, device, `dtype` R64/R32 for a real A, C128/C64
 * for a complex A).  step holds the product's parameters exactly as for
 * afsi_clenshaw_step_batched (step.col0 is ignored).  The library launches one kernel
 * per distinct width (at most 32 slices each) whose gathers read whole rows of one
 * contiguous block, and gives every column the same bits as afsi_filter_block.  Rows
 * and pointers must be 16-byte aligned; a slice's three blocks must not overlap each
 * other or another slice's.  Any number of slices.  Errors: AFSI_E_INVALID.
 */
typedef struct {
    afsi_step_group step;
    const void *X;
    void *P0, *P1;
    int64_t ld;
} afsi_slice_blocks;

int afsi_clenshaw_step_grouped(afsi_matrix_t A, int ngroups, const afsi_slice_blocks *slices,
                               int32_t dtype, void *stream);

/*
 * Whole filters of several spectrum slices of one matrix (Section 1's slicing, each
 * slice filtered by Algorithm 2 with its own interval's coefficients): for every
 * slice g, Y_g = sum_{j=0}^{degree_g} coeffs_g[j] T_j(l(A)) X_g.  The library runs
 * the slices' recurrences side by side, one afsi_clenshaw_step_grouped product per
 * step for all slices that still have products left (slices start together; a
 * lower-degree slice finishes earlier), so A is read once per step for all of them.
 * Every column gets the same bits as from afsi_filter_block on that slice alone.
 *   coeffs : host, degree + 1 doubles (read before return).
 *   X, Y, work : device, n x ncols, row-major with leading dimension ld (elements),
 *   all of `dtype` (R64 / R32 for a real A, C128 / C64 for a complex A).  Y and work
 *   are overwritten; X is read only.  No block may overlap another block of any slice.
 * Needs spectral bounds on A and degree >= 1 for every slice.  Any number of slices.
 * Errors: AFSI_E_INVALID.  Asynchronous on `stream`.
 */
typedef struct {
    const double *coeffs;
    int32_t degree;
    const void *X;
    void *Y;
    void *work;
    int64_t ncols, ld;
} afsi_slice_filter;

int afsi_filter_batched(afsi_matrix_t A, int nslices, const afsi_slice_filter *slices,
                        int32_t dtype, void *stream);

/* ------------------------------------------------------------------ dense steps (FP64) */

/*
 * G = X^H Y (p x q) for n x p X and n x q Y (R64 or C128, same dtype), into the
 * device block G (p x q, same dtype).  Fixed-order reduction: deterministic.
 */
int afsi_block_inner(const afsi_block *X, const afsi_block *Y, afsi_block *G, void *stream);

/*
 * Y = X M + beta Y for n x p X, p x q M (device), n x q Y; R64 or C128; beta real.
 * Y must not overlap X or M.
 */
int afsi_block_gemm(const afsi_block *X, const afsi_block *M, double beta, afsi_block *Y,
                    void *stream);

/*
 * Orthonormalise X in place (Algorithm 4, orthogonalisation step, by Cholesky QR):
 * first X <- X - L (L^H X) twice when `locked` has columns (L orthonormal), then
 * CholQR2 (G = X^H X, R^H R = G, X <- X R^-1, repeated once).  If a Cholesky
 * factor breaks down, shifted CholQR3 is used (shift 11 (n p + p (p+1)) u ||X||_F^2).
 * `work` is an n x p scratch block of X's dtype.  R64 or C128.
 * Synchronises `stream` (the small Gram factorisations run on the host).
 */
int afsi_orthonormalize(const afsi_block *locked, afsi_block *X, afsi_block *work, void *stream);

/*
 * Rayleigh-Ritz (Algorithm 1): B = Q^H A Q, B = U diag(ritz) U^H (host, FP64),
 * V = Q U and AV = A V (a sparse product, cheaper than forming (A Q) U).  Q is
 * n x p orthonormal and left unchanged; V and AV are n x p; ritz_out[p] (host)
 * ascending.  R64 or C128.  Synchronises `stream`.
 */
int afsi_rayleigh_ritz(afsi_matrix_t A, const afsi_block *Q, afsi_block *V, afsi_block *AV,
                       double *ritz_out, void *stream);

/*
 * One iteration's orthonormalisation and Rayleigh-Ritz (Algorithm 4's orthogonalisation
 * step without locked vectors, then Algorithm 1's Rayleigh-Ritz) with the orthonormal
 * basis left implicit: CholQR2 as afsi_orthonormalize up to its last factor R, where
 * Q = Y R^-1 for the last pass's input Y; then B = R^-H (Y^H A Y) R^-1 (= Q^H A Q),
 * B = U diag(ritz) U^H, V = Y (R^-1 U) (= Q U) and AV = A V, as afsi_rayleigh_ritz.
 * This saves the n x p x p product that forms Q.  X (consumed: holds Y or a scratch
 * state on return), work, V, AV: n x p, R64 or C128, one leading dimension; V must not
 * overlap X or work; AV may be `work` (not X or V); ritz_out[p] (host) ascending.
 * Errors as afsi_orthonormalize and afsi_rayleigh_ritz.  Synchronises `stream`.
 */
int afsi_orthonormalize_rayleigh_ritz(afsi_matrix_t A, afsi_block *X, afsi_block *work,
                                      afsi_block *V, afsi_block *AV, double *ritz_out,
                                      void *stream);

/*
 * norms_out[j] = || AV[:, j] - lambda[j] V[:, j] ||_2 for j < V.cols (host output,
 * Algorithm 4 residual step).  R64 or C128.  Synchronises `stream`.
 */
int afsi_residual_norms(const afsi_block *V, const afsi_block *AV, const double *lambda,
                        double *norms_out, void *stream);

/*
 * afsi_residual_norms for callers that cannot allocate device or pinned host memory
 * (code that must not call hipMalloc, such as a tight serving loop or a caller that
 * forbids allocation).  Same arguments, results and errors as afsi_residual_norms; its
 * device work uses a fixed array of 2^17 doubles (1 MiB) that the library keeps on every
 * device it runs on until the process ends, holding the eigenvalues, the chunk partials
 * and the norms: 2 q + (row chunks) * q doubles, at most about 2 q + 65536 + 64 ceil(q/64),
 * so any n with q <= 8192 fits.  Larger shapes get AFSI_E_INVALID.  lambda and norms_out
 * are ordinary host memory, copied on `stream`; synchronises `stream`.  Calls that
 * overlap on one device share the array and race: serialise them.
 */
int afsi_residual_norms_noalloc(const afsi_block *V, const afsi_block *AV, const double *lambda,
                                double *norms_out, void *stream);

/* dst = src converted (R64 <-> R32, C128 <-> C64, or same type copy); same shape. */
int afsi_convert_block(const afsi_block *src, afsi_block *dst, void *stream);

/* dst[:, t] = src[:, cols[t]] for t < count (host index list); dst has count columns. */
int afsi_gather_columns(const afsi_block *src, const int32_t *cols, int64_t count,
                        afsi_block *dst, void *stream);

/* ------------------------------------------------------------------ host control */

/*
 * Algorithm 3: the first j in 1..kmax for which the truncated series
 * gamma = sum_{i<=j} coeffs[i] T_i(l(ritz)) satisfies |gamma|_(p) / |gamma|_(e) < tau_a
 * (p-th and e-th largest magnitudes over the p Ritz values); kmax if none.
 * Needs 1 <= e <= p.  Pure host function.
 */
int afsi_select_degree(const double *ritz, int64_t p, int64_t e, const double *coeffs, int kmax,
                       double l1, double l2, double tau_a, int *degree_out);

/*
 * Spurious-value test and locking of one iteration (Algorithm 4 with eq. (tau_s)):
 *   in_interval[j] (in, length p): 1 if ritz[j] in [a, b];
 *   res[j]: residual norms (read where in_interval[j]);
 *   tau_s = min over the interval's Ritz values of the distance to {a, b};
 *   C = {j in I : res[j] < tau_s}; n_check = |C| + n_lock; if n_check > 0 and it
 *   equals *n_check_prev, I = C; *n_check_prev = n_check;
 *   lock[j] = (j in I and res[j] < tau_abs); in_interval is overwritten with I;
 *   *done = (I minus the locked set is empty).
 * Pure host function; requires at least one in_interval entry.
 */
int afsi_lock_select(const double *ritz, int64_t p, const double *res, uint8_t *in_interval,
                     double a, double b, double tau_abs, int64_t n_lock, int64_t *n_check_prev,
                     uint8_t *lock, int *done);

/*
 * Host Hermitian eigensolver used by Rayleigh-Ritz (Algorithm 1): B (p x p,
 * row-major, ldb; R64 or C128, only its Hermitian part is used) = U diag(w) U^H,
 * w[p] ascending, U (p x p, ldu, same dtype) unitary.  Householder tridiagonal
 * reduction, then divide and conquer on the tridiagonal above 32 rows (implicit-shift
 * symmetric QR for smaller blocks and as the fallback when a secular equation does not
 * settle).  Pure host function.  AFSI_E_INVALID if B has a non-finite entry;
 * AFSI_E_NOCONV if the QR iteration does not converge (also returned by
 * afsi_rayleigh_ritz and afsi_solve; afsi_solve then reports no locked pairs).
 */
int afsi_host_eigh(int64_t p, int32_t dtype, const double *B, int64_t ldb, double *w, double *U,
                   int64_t ldu);

/*
 * Host factor used by Cholesky QR: overwrite G (p x p Hermitian positive definite,
 * row-major, R64 or C128) with R^{-1}, where R^H R = G + shift I and R is upper
 * triangular (the strictly lower part is set to zero).  AFSI_E_NOT_HPD (and G
 * unchanged) on a non-positive pivot.  Pure host function.
 */
int afsi_host_cholesky_inverse(int64_t p, int32_t dtype, double *G, int64_t ldg, double shift);

/* ------------------------------------------------------------------ full solver */

typedef struct {
    int32_t kmax;          /* maximum degree k (coefficients and damping use it) */
    int32_t k_init;        /* first degree; <= 0: kmax (fixed) or eq. (compute_k_1) (adaptive) */
    int32_t adaptive;      /* 1: Algorithm 3 after each iteration; 0: fixed degree */
    int32_t damping;       /* afsi_damping */
    double m_exp;          /* exponent m for AFSI_DAMP_LANCZOS (paper: 0.5) */
    double tau_a;          /* Algorithm 3 threshold (paper: 1e-3) */
    double tau_c;          /* lock when ||r|| < tau_c * ||A||, ||A|| = max(|lmin|,|lmax|) */
    double C;              /* eq. (compute_k_1) constant (paper: 1.4) */
    int32_t max_iter;      /* iteration limit */
    int32_t filter_dtype;  /* AFSI_R64/AFSI_C128 (plain) or AFSI_R32/AFSI_C64 (mixed form) */
} afsi_options;

/* Fill `o` with the paper's parameters (Section 4) and a fixed Jackson degree kmax. */
void afsi_options_default(afsi_options *o, int kmax);

typedef struct {
    int64_t count;         /* eigenpairs found in [a, b] */
    int32_t iterations;
    int32_t converged;     /* 1 if every Ritz pair in [a, b] was locked */
    int64_t spmv;          /* products with A times block columns (filter + Rayleigh-Ritz) */
    double avg_degree;
    double time_filter_ms, time_orth_ms, time_rr_ms, time_resid_ms, time_host_ms;
} afsi_result;

/*
 * Algorithm 4 on A with bounds already set.  X0: n x p start block (FP64 dtype of
 * A's domain, device); it is orthonormalised and then consumed (overwritten).
 * On return: eigenvalues[count] (host, ascending, capacity `capacity`),
 * residuals[count] (host), and the eigenvectors in columns 0..count-1 of
 * `evecs` (device, n x capacity, FP64 dtype).  Returns AFSI_E_NOCONV with the
 * pairs locked so far if max_iter is reached, AFSI_E_INVALID if more than
 * `capacity` pairs lock.
 */
int afsi_solve(afsi_matrix_t A, double a, double b, const afsi_options *opts, afsi_block *X0,
               afsi_block *evecs, int64_t capacity, double *eigenvalues, double *residuals,
               afsi_result *result, void *stream);

/* ------------------------------------------------------------------ filtered Lanczos */

/*
 * Filtered thick-restart block Lanczos.  Section 3.1 builds the damped filter for
 * subspace iteration and notes that it suits thick-restart Lanczos as well (Section 5
 * names filtered Lanczos as the framework to follow); the paper defines no such
 * method, so this is the library's: a block Krylov method on the operator
 * B = rho(A), the filter of eq. (AdaPolySI) at a fixed degree applied by Clenshaw's
 * recurrence (Algorithm 2), whose eigenvalues rho(lambda) are close to one inside
 * [a, b] and close to zero away from it.  Each cycle grows a basis of `basis` columns
 * in blocks of `block` (every new block B V_last projected twice against the basis and
 * the locked vectors, then Cholesky QR), does Rayleigh-Ritz on B (H = V^H B V, host
 * eigensolver, theta descending), takes lambda = u^H A u and ||A u - lambda u|| for
 * each Ritz vector u, and locks the pairs with theta >= eta = min(rho(a), rho(b)) and
 * ||A u - lambda u|| < tau_c ||A|| (||A|| = max(|lmin|, |lmax|)); locked pairs with
 * lambda in [a, b] are the results, the others are only deflated.  It stops when no
 * pair with theta >= eta is left unlocked and the largest remaining theta plus its
 * B-residual lies below eta; otherwise it restarts with the min(wanted + block,
 * basis / 2) unlocked Ritz vectors of largest theta plus the next Krylov block.  A
 * block of s columns finds eigenvalues of multiplicity up to s directly.
 */
typedef struct {
    int32_t degree;      /* filter degree k (coefficients and damping at k) */
    int32_t damping;     /* afsi_damping */
    double m_exp;        /* exponent m for AFSI_DAMP_LANCZOS */
    int32_t block;       /* s >= 1: columns per Krylov block */
    int32_t basis;       /* m: basis columns before a restart, 2 s <= m <= n */
    double tau_c;        /* lock when ||A u - lambda u|| < tau_c ||A|| */
    int32_t max_cycles;  /* restart-cycle limit */
    int32_t mixed;       /* 1: the filter runs in FP32 (complex FP32 for a complex A) on
                            converted copies of the Krylov blocks, everything else in FP64
                            (use tau_c >= 1e-6).  Rayleigh-Ritz on B can only separate
                            eigenvectors whose filter values differ by more than the FP32
                            operator's error (~1e-7): fine for windows the filter resolves,
                            but pairs deep inside a flat filter plateau then never lock.
                            0: FP64 throughout */
} afsi_lanczos_options;

/* Jackson damping, block 4, basis 128, tau_c 1e-10, 200 cycles, FP64, at degree `degree`. */
void afsi_lanczos_options_default(afsi_lanczos_options *o, int degree);

typedef struct {
    int64_t count;           /* eigenpairs found in [a, b] */
    int32_t cycles;
    int32_t converged;       /* 1 if the stopping test held */
    int64_t filter_columns;  /* columns the filter was applied to (each: `degree` products) */
    int64_t locked_outside;  /* converged pairs outside [a, b] (deflated, not returned) */
    double time_ms;
} afsi_lanczos_result;

/*
 * Run the method above on A (bounds set) for [a, b].  X0: n x block start block
 * (device, R64 for a real A, C128 for a complex A; read only).  On return:
 * eigenvalues[count] and residuals[count] (host, ascending), eigenvectors in columns
 * 0..count-1 of `evecs` (device, n x capacity, X0's dtype).  The library allocates its
 * working blocks for the call: five n x (basis + block) blocks, one n x basis block and
 * three n x block blocks (three more in FP32 for the mixed form).  Returns AFSI_E_NOCONV with the pairs found if max_cycles is reached,
 * AFSI_E_INVALID on bad arguments or if more than `capacity` pairs lock.
 * Synchronises `stream`.
 */
int afsi_filtered_lanczos(afsi_matrix_t A, double a, double b, const afsi_lanczos_options *opts,
                          const afsi_block *X0, afsi_block *evecs, int64_t capacity,
                          double *eigenvalues, double *residuals, afsi_lanczos_result *result,
                          void *stream);

/* ------------------------------------------------------------------ serving */

/*
 * Continuous-batching server for many solves on one device (spectrum slicing of
 * one matrix, Section 1, and independent matrices).  Requests are admitted when
 * their device footprint fits `hbm_budget_bytes`: a pool of three n x cols FP64
 * buffers per (matrix, filter dtype) (three more in FP32 for the mixed form), in
 * which a request owns a contiguous n x w slot of each, plus n x p for the
 * request's eigenvectors.  All filtering requests of a pool advance together, one
 * grouped Clenshaw product (afsi_clenshaw_step_grouped, one launch per width) per
 * round, on the pool's product stream and thread; the dense steps of Algorithm 4
 * (orthonormalisation, Rayleigh-Ritz, residuals, locking) of a request whose filter
 * has finished run on the pool's second stream and thread, while the other requests'
 * products go on.  Independent matrices have their own pools and overlap on the
 * device.  A request's results do not depend on what else is running.  Matrices must
 * outlive the requests that use them.
 */
typedef struct afsi_server_s *afsi_server_t;

typedef struct {
    int32_t state;       /* 0 queued, 1 running, 2 done, 3 failed */
    int32_t status;      /* afsi_status of a finished request (AFSI_E_NOCONV: iteration limit) */
    int64_t count;       /* eigenpairs found so far */
    int32_t iterations;
    int32_t converged;
    int64_t spmv;
    double avg_degree;
    double t_submit, t_admit, t_done; /* seconds on the server's clock */
} afsi_request_info;

typedef struct {
    int64_t bytes_in_use, budget;
    int64_t queued, running, done, pools;
    int64_t batched_launches, batched_groups; /* grouped rounds; slices per round = groups / launches */
    int64_t kernel_launches, kernel_slices;   /* launches of the grouped kernel and the slice
                                                 products they took (slices sharing one launch =
                                                 kernel_slices / kernel_launches); the rest of a
                                                 round's slices ran one product each */
    double now;                               /* server clock (s) */
} afsi_server_stats;

int afsi_server_create(int device, int64_t hbm_budget_bytes, afsi_server_t *out);
/* Stops the pool threads (running requests fail), frees everything. */
int afsi_server_destroy(afsi_server_t S);
/*
 * Reserve `cols` columns for A's pools (slices of one matrix share them).  A pool is
 * created with max(cols, the first request's width) columns and lives while it has
 * requests; a request wider than a live pool of its matrix and filter precision
 * waits until that pool has drained, so size the pool for the widest request.
 */
int afsi_server_set_pool_columns(afsi_server_t S, afsi_matrix_t A, int64_t cols);
/*
 * Queue a solve of [a, b] on A (bounds set) with block width p and `opts`
 * (opts->filter_dtype picks the plain or mixed form).  The start block is N(0,1)
 * from a counter-based generator keyed by `seed`.  AFSI_E_BUSY if the request
 * cannot fit the budget even alone.  Returns at once.  A request whose device
 * allocation fails at admission finishes with status AFSI_E_NOMEM.
 */
int afsi_server_submit(afsi_server_t S, afsi_matrix_t A, double a, double b, int64_t p,
                       const afsi_options *opts, uint64_t seed, int64_t *id);
int afsi_server_info(afsi_server_t S, int64_t id, afsi_request_info *info);
/* Block until request `id` finishes or `timeout_s` passes (info->state tells which). */
int afsi_server_wait(afsi_server_t S, int64_t id, double timeout_s, afsi_request_info *info);
/* Next finished request id in completion order, or -1 after `timeout_s`. */
int afsi_server_wait_any(afsi_server_t S, double timeout_s, int64_t *id);
/*
 * Copy a finished request's eigenvalues / residuals (host, `capacity` entries)
 * and eigenvectors (device block, n x count or wider; NULL to skip) and release
 * the request.  Synchronises `stream`.
 */
int afsi_server_fetch(afsi_server_t S, int64_t id, double *eigenvalues, double *residuals,
                      int64_t capacity, afsi_block *evecs, void *stream);
int afsi_server_get_stats(afsi_server_t S, afsi_server_stats *st);

#ifdef __cplusplus
}
#endif

#endif /* AFSI_H */
