// Filtered thick-restart block Lanczos for the eigenpairs of A in [a, b].
//
// The operator is B = rho(A), the damped step filter of eq. (AdaPolySI) at a fixed
// degree applied by Clenshaw's recurrence (Algorithm 2, the Clenshaw kernels): its
// eigenvalues rho(lambda) are near one for lambda in [a, b] and near zero away from
// it, so a Krylov space of B finds the interval's eigenvectors first.  The paper builds
// its filter for subspace iteration and notes that it suits thick-restart Lanczos too
// (Section 3.1; Section 5 names filtered Lanczos as the next framework) without
// defining the method; the one built here, cycle by cycle:
//   * grow the basis V (s columns per block) to m columns: the next block is B V_last
//     made orthogonal, twice, to the basis and the locked vectors, then orthonormal
//     (Cholesky QR); W = B V is kept beside V;
//   * Rayleigh-Ritz on B: H = V^H W, H = Y diag(theta) Y^H (host), theta descending,
//     U = V Y, B U = W Y (matrix cores);
//   * A-side quotients lambda = u^H A u and residuals ||A u - lambda u||; a pair is
//     wanted when theta >= eta = min(rho(a), rho(b)); wanted pairs with a residual
//     below tau_c ||A|| are locked (results when lambda is in [a, b]);
//   * stop when no wanted pair is left and the largest remaining theta plus its
//     B-residual stays below eta; else restart thick with the unlocked Ritz vectors
//     of largest theta plus the Krylov continuation block.
// The mixed form applies the filter to FP32 copies of the Krylov blocks (complex FP32
// for a complex A); everything else stays FP64.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.h"

namespace afsi {
namespace {

struct Dev {
    void *p = nullptr;
    explicit Dev(size_t bytes) { AFSI_HIP(hipMalloc(&p, std::max<size_t>(bytes, 16))); }
    ~Dev() {
        if (p) (void)hipFree(p);
    }
    Dev(const Dev &) = delete;
    Dev &operator=(const Dev &) = delete;
};

// rho(x) = sum_j c_j T_j(l(x)) in trigonometric form: cos(j arccos t) on |t| <= 1,
// (+-1)^j cosh(j arccosh |t|) outside.
double filter_value(double x, const std::vector<double> &c, double lmin, double lmax) {
    const double t = (2.0 * x - lmax - lmin) / (lmax - lmin);
    double v = 0.0;
    if (std::fabs(t) <= 1.0) {
        const double th = std::acos(t);
        for (size_t j = 0; j < c.size(); ++j) v += c[j] * std::cos((double)j * th);
    } else {
        const double ch = std::acosh(std::fabs(t));
        for (size_t j = 0; j < c.size(); ++j)
            v += c[j] * ((t < 0 && (j & 1)) ? -1.0 : 1.0) * std::cosh((double)j * ch);
    }
    return v;
}

// X <- X - L (L^H X) for n x k L (ld ldl) and n x q X (ld ldx).
void project_once(int dt, const void *L, int64_t ldl, int64_t k, void *X, int64_t ldx, int64_t n,
                  int64_t q, hipStream_t s) {
    if (k == 0 || q == 0) return;
    const int comp = is_complex(dt) ? 2 : 1;
    double *C = (double *)workspace(s).dev_reserve(SLOT_SMALL, sizeof(double) * comp * k * q);
    inner_dev(dt, L, ldl, X, ldx, n, k, q, C, q, s);
    gemm_dev(dt, L, ldl, C, q, n, k, q, -1.0, 1.0, X, ldx, s);
}

void copy_cols(const void *src, int64_t lds, void *dst, int64_t ldd, int64_t n, int64_t cols, int eb,
               hipStream_t s) {
    if (n == 0 || cols == 0) return;
    AFSI_HIP(hipMemcpy2DAsync(dst, ldd * eb, src, lds * eb, cols * eb, n, hipMemcpyDeviceToDevice, s));
}

}  // namespace
}  // namespace afsi

using namespace afsi;

extern "C" {

void afsi_lanczos_options_default(afsi_lanczos_options *o, int degree) {
    if (!o) return;
    o->degree = degree;
    o->damping = AFSI_DAMP_JACKSON;
    o->m_exp = 0.5;
    o->block = 4;
    o->basis = 128;
    o->tau_c = 1e-10;
    o->max_cycles = 200;
    o->mixed = 0;
}

int afsi_filtered_lanczos(afsi_matrix_t A, double a, double b, const afsi_lanczos_options *opts,
                          const afsi_block *X0, afsi_block *evecs, int64_t capacity,
                          double *eigenvalues, double *residuals, afsi_lanczos_result *result,
                          void *stream) {
    int converged = 0;
    int64_t n_in = 0;
    const int status = guarded([&] {
        AFSI_REQUIRE(A && opts && X0 && evecs && result, "NULL argument");
        AFSI_REQUIRE(A->has_bounds, "spectral bounds are not set on this matrix");
        AFSI_REQUIRE(b > a, "interval needs a < b");
        const int dt = X0->dtype;
        AFSI_REQUIRE(is_fp64(dt) && is_complex(dt) == (A->dtype == AFSI_C128),
                     "X0 must be R64 (real A) or C128 (complex A)");
        const int64_t n = A->n, s = opts->block, m = opts->basis;
        AFSI_REQUIRE(s >= 1 && m >= 2 * s && m <= n, "need 1 <= block, 2 block <= basis <= n");
        AFSI_REQUIRE(X0->rows == n && X0->cols == s && X0->ld >= s && X0->ptr,
                     "X0 must be n x block");
        AFSI_REQUIRE(evecs->dtype == dt && evecs->rows == n && evecs->cols >= capacity &&
                         capacity >= 0 && evecs->ld >= evecs->cols,
                     "evecs must be n x capacity of X0's dtype");
        AFSI_REQUIRE(capacity == 0 || (eigenvalues && residuals), "NULL eigenvalue/residual output");
        AFSI_REQUIRE(opts->degree >= 1 && opts->max_cycles >= 1, "degree and max_cycles must be >= 1");
        std::memset(result, 0, sizeof *result);
        DeviceGuard dg(A->device);
        hipStream_t st = reinterpret_cast<hipStream_t>(stream);
        const auto t_start = std::chrono::steady_clock::now();

        const bool cplx = is_complex(dt);
        const int comp = cplx ? 2 : 1;
        const int eb = elem_bytes(dt);
        const int k = opts->degree;
        std::vector<double> coeffs(k + 1);
        filter_coefficients(A->lmin, A->lmax, a, b, k, opts->damping, opts->m_exp, coeffs.data());
        const double eta = std::min(filter_value(a, coeffs, A->lmin, A->lmax),
                                    filter_value(b, coeffs, A->lmin, A->lmax));
        const double tau_abs = opts->tau_c * std::max(std::fabs(A->lmin), std::fabs(A->lmax));

        // basis blocks n x (up to m + s - 1) columns, even leading dimension
        const int64_t cap = m + s, ldb = (cap + 1) / 2 * 2;
        const size_t blk = (size_t)n * ldb * eb;
        Dev V(blk), W(blk), U(blk), BU(blk), AU(blk);
        Dev Lout((size_t)n * m * eb);  // locked pairs outside [a, b] (deflated, not returned)
        Dev Zb((size_t)n * s * eb), BZ((size_t)n * s * eb), Zw((size_t)n * s * eb);
        // mixed form: the filter runs on FP32 copies (complex FP32 for a complex A)
        const bool mixed = opts->mixed != 0;
        const int fdt = mixed ? (cplx ? AFSI_C64 : AFSI_R32) : dt;
        const size_t fbytes = mixed ? (size_t)n * s * elem_bytes(fdt) : 0;
        Dev F0(fbytes), F1(fbytes), F2(fbytes);
        Dev Hd(sizeof(double) * comp * cap * cap), Yd(sizeof(double) * comp * cap * cap);
        Dev dots(sizeof(double) * cap);
        std::vector<double> H((size_t)comp * cap * cap), Y((size_t)comp * cap * cap),
            Yo((size_t)comp * cap * cap);
        std::vector<double> theta(cap), tord(cap), lam(cap), rA(cap), rB(cap);
        char *Vp = (char *)V.p, *Wp = (char *)W.p;
        int64_t n_out = 0, filtered = 0;

        auto filt = [&](void *out) {  // out (n x s, ld s) = B Zb
            if (!mixed) {
                filter_apply(A, coeffs.data(), k, dt, Zb.p, out, Zw.p, s, s, st);
            } else {
                afsi_block z{Zb.p, n, s, s, dt}, z32{F0.p, n, s, s, fdt};
                launch_convert(z, z32, st);
                filter_apply(A, coeffs.data(), k, fdt, F0.p, F1.p, F2.p, s, s, st);
                afsi_block y32{F1.p, n, s, s, fdt}, y{out, n, s, s, dt};
                launch_convert(y32, y, st);
            }
            filtered += s;
        };
        // Zb <- Zb made orthogonal (twice) to V[:, :cols] and the locked vectors, orthonormal
        auto deflate_orth = [&](int64_t cols) {
            for (int pass = 0; pass < 2; ++pass) {
                project_once(dt, V.p, ldb, cols, Zb.p, s, n, s, st);
                project_once(dt, evecs->ptr, evecs->ld, n_in, Zb.p, s, n, s, st);
                project_once(dt, Lout.p, m, n_out, Zb.p, s, n, s, st);
            }
            orthonormalize_dev(dt, Zb.p, Zw.p, n, s, s, st, nullptr);
        };

        // start block: V[:, :s] = orth(X0), W[:, :s] = B V[:, :s]
        copy_cols(X0->ptr, X0->ld, Zb.p, s, n, s, eb, st);
        orthonormalize_dev(dt, Zb.p, Zw.p, n, s, s, st, nullptr);
        copy_cols(Zb.p, s, Vp, ldb, n, s, eb, st);
        filt(BZ.p);
        copy_cols(BZ.p, s, Wp, ldb, n, s, eb, st);
        int64_t cols = s;
        int cycle = 0;
        for (cycle = 1; cycle <= opts->max_cycles; ++cycle) {
            // ---- grow the block Krylov basis to m columns
            while (cols < m) {
                copy_cols(Wp + (size_t)(cols - s) * eb, ldb, Zb.p, s, n, s, eb, st);
                deflate_orth(cols);
                copy_cols(Zb.p, s, Vp + (size_t)cols * eb, ldb, n, s, eb, st);
                filt(BZ.p);
                copy_cols(BZ.p, s, Wp + (size_t)cols * eb, ldb, n, s, eb, st);
                cols += s;
            }
            // ---- Rayleigh-Ritz on B: H = V^H W (Hermitian part), eigenvalues descending
            inner_dev(dt, V.p, ldb, W.p, ldb, n, cols, cols, (double *)Hd.p, cols, st);
            AFSI_HIP(hipMemcpyAsync(H.data(), Hd.p, sizeof(double) * comp * cols * cols,
                                    hipMemcpyDeviceToHost, st));
            AFSI_HIP(hipStreamSynchronize(st));
            for (int64_t i = 0; i < cols; ++i)
                for (int64_t j = i; j < cols; ++j)
                    for (int c = 0; c < comp; ++c) {
                        const double x = H[comp * (i * cols + j) + c], y = H[comp * (j * cols + i) + c];
                        // (H + H^H) / 2: the real part symmetric, the imaginary antisymmetric
                        const double sym = c == 0 ? 0.5 * (x + y) : 0.5 * (x - y);
                        H[comp * (i * cols + j) + c] = sym;
                        H[comp * (j * cols + i) + c] = c == 0 ? sym : -sym;
                    }
            host_eigh_or_throw(cols, cplx, H.data(), cols, theta.data(), Y.data(), cols);
            std::vector<int64_t> order(cols);
            std::iota(order.begin(), order.end(), 0);
            std::stable_sort(order.begin(), order.end(),
                             [&](int64_t x, int64_t y) { return theta[x] > theta[y]; });
            for (int64_t j = 0; j < cols; ++j) {
                tord[j] = theta[order[j]];
                for (int64_t i = 0; i < cols; ++i)
                    for (int c = 0; c < comp; ++c)
                        Yo[comp * (i * cols + j) + c] = Y[comp * (i * cols + order[j]) + c];
            }
            AFSI_HIP(hipMemcpyAsync(Yd.p, Yo.data(), sizeof(double) * comp * cols * cols,
                                    hipMemcpyHostToDevice, st));
            gemm_dev(dt, V.p, ldb, (const double *)Yd.p, cols, n, cols, cols, 1.0, 0.0, U.p, ldb, st);
            gemm_dev(dt, W.p, ldb, (const double *)Yd.p, cols, n, cols, cols, 1.0, 0.0, BU.p, ldb, st);
            residual_norms_host(dt, U.p, ldb, BU.p, ldb, tord.data(), n, cols, rB.data(), st);
            // ---- A-side quotients and residuals
            spmm_apply(A, dt, U.p, AU.p, cols, ldb, st);
            column_dots_dev(dt, U.p, ldb, AU.p, ldb, n, cols, (double *)dots.p, st);
            AFSI_HIP(hipMemcpyAsync(lam.data(), dots.p, sizeof(double) * cols, hipMemcpyDeviceToHost, st));
            AFSI_HIP(hipStreamSynchronize(st));
            residual_norms_host(dt, U.p, ldb, AU.p, ldb, lam.data(), n, cols, rA.data(), st);
            // ---- locking
            std::vector<int32_t> in_idx, out_idx, free_idx;
            int64_t n_want = 0;
            for (int64_t j = 0; j < cols; ++j) {
                const bool wanted = tord[j] >= eta;
                const bool lock = wanted && rA[j] < tau_abs;
                if (lock) {
                    (lam[j] >= a && lam[j] <= b ? in_idx : out_idx).push_back((int32_t)j);
                } else {
                    free_idx.push_back((int32_t)j);
                    n_want += wanted;
                }
            }
            if (n_in + (int64_t)in_idx.size() > capacity)
                AFSI_FAIL(AFSI_E_INVALID, "more than %lld eigenpairs locked (capacity)",
                          (long long)capacity);
            AFSI_REQUIRE(n_out + (int64_t)out_idx.size() <= m,
                         "more than %lld pairs outside [a, b] locked", (long long)m);
            for (size_t t = 0; t < in_idx.size(); ++t) {
                eigenvalues[n_in + t] = lam[in_idx[t]];
                residuals[n_in + t] = rA[in_idx[t]];
            }
            if (!in_idx.empty())
                gather_cols(dt, U.p, n, ldb, in_idx.data(), (int64_t)in_idx.size(),
                            (char *)evecs->ptr + (size_t)n_in * eb, evecs->ld, st);
            if (!out_idx.empty())
                gather_cols(dt, U.p, n, ldb, out_idx.data(), (int64_t)out_idx.size(),
                            (char *)Lout.p + (size_t)n_out * eb, m, st);
            n_in += (int64_t)in_idx.size();
            n_out += (int64_t)out_idx.size();
            if (n_want == 0 && (free_idx.empty() || tord[free_idx[0]] + rB[free_idx[0]] < eta)) {
                converged = 1;
                break;
            }
            if (cycle == opts->max_cycles) break;
            // ---- thick restart: kept Ritz vectors plus the Krylov continuation block,
            // the latter computed from the old basis before it is overwritten
            const int64_t nk = std::max<int64_t>(1, std::min<int64_t>(n_want + s, m / 2));
            std::vector<int32_t> keep(free_idx.begin(), free_idx.begin() + std::min<int64_t>(nk, free_idx.size()));
            copy_cols(Wp + (size_t)(cols - s) * eb, ldb, Zb.p, s, n, s, eb, st);
            deflate_orth(cols);
            const int64_t kept = (int64_t)keep.size();
            gather_cols(dt, U.p, n, ldb, keep.data(), kept, V.p, ldb, st);
            gather_cols(dt, BU.p, n, ldb, keep.data(), kept, W.p, ldb, st);
            copy_cols(Zb.p, s, Vp + (size_t)kept * eb, ldb, n, s, eb, st);
            filt(BZ.p);
            copy_cols(BZ.p, s, Wp + (size_t)kept * eb, ldb, n, s, eb, st);
            cols = kept + s;
        }
        // ---- results ascending (eigenvector columns permuted through U)
        if (n_in > 1) {
            std::vector<int32_t> order(n_in);
            std::iota(order.begin(), order.end(), 0);
            std::stable_sort(order.begin(), order.end(),
                             [&](int32_t x, int32_t y) { return eigenvalues[x] < eigenvalues[y]; });
            std::vector<double> ev(eigenvalues, eigenvalues + n_in), rs(residuals, residuals + n_in);
            for (int64_t t = 0; t < n_in; ++t) {
                eigenvalues[t] = ev[order[t]];
                residuals[t] = rs[order[t]];
            }
            Dev tmp((size_t)n * n_in * eb);
            gather_cols(dt, evecs->ptr, n, evecs->ld, order.data(), n_in, tmp.p, n_in, st);
            copy_cols(tmp.p, n_in, evecs->ptr, evecs->ld, n, n_in, eb, st);
        }
        AFSI_HIP(hipStreamSynchronize(st));
        result->count = n_in;
        result->cycles = std::min(cycle, opts->max_cycles);
        result->converged = converged;
        result->filter_columns = filtered;
        result->locked_outside = n_out;
        result->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                                    t_start).count();
    });
    if (status == AFSI_OK && !converged) {
        set_error("cycle limit reached with %lld pairs locked", (long long)n_in);
        return AFSI_E_NOCONV;
    }
    return status;
}

}  // extern "C"
