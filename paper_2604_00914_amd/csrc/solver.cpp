// Full solver (Algorithm 4) and the Lanczos estimate of the spectral interval.
//
// Per iteration: filter the active block (Algorithm 2, degree k^(i)), make it
// orthogonal to the locked vectors and orthonormal (Cholesky QR), Rayleigh-Ritz,
// residuals of the Ritz pairs, then the spurious-value test (eq. (tau_s)) and
// locking; Algorithm 3 picks the next degree in adaptive mode.  The mixed form
// filters an FP32 copy of the active block and returns to FP64 for everything else.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.h"

namespace afsi {

namespace {

struct DevBuf {
    void *p = nullptr;
    DevBuf() = default;
    explicit DevBuf(size_t bytes) { AFSI_HIP(hipMalloc(&p, std::max<size_t>(bytes, 16))); }
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
};

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0) {
    return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

void gather(int dtype, const void *src, int64_t n, int64_t ld, const std::vector<int32_t> &cols,
            void *dst, int64_t ldd, hipStream_t s) {
    gather_cols(dtype, src, n, ld, cols.data(), (int64_t)cols.size(), dst, ldd, s);
}


}  // namespace

}  // namespace afsi

using namespace afsi;

extern "C" {

void afsi_options_default(afsi_options *o, int kmax) {
    if (!o) return;
    o->kmax = kmax;
    o->k_init = 0;
    o->adaptive = 0;
    o->damping = AFSI_DAMP_JACKSON;
    o->m_exp = 0.5;
    o->tau_a = 1e-3;
    o->tau_c = 1e-10;
    o->C = 1.4;
    o->max_iter = 200;
    o->filter_dtype = AFSI_R64;
}

int afsi_solve(afsi_matrix_t A, double a, double b, const afsi_options *opts, afsi_block *X0,
               afsi_block *evecs, int64_t capacity, double *eigenvalues, double *residuals,
               afsi_result *result, void *stream) {
    int64_t n_lock = 0;
    int converged = 0;
    int status = guarded([&] {
        AFSI_REQUIRE(A && opts && X0 && evecs && result, "NULL argument");
        AFSI_REQUIRE(A->has_bounds, "spectral bounds are not set on this matrix");
        AFSI_REQUIRE(b > a, "interval needs a < b");
        const int dt = X0->dtype;
        AFSI_REQUIRE(is_fp64(dt) && is_complex(dt) == (A->dtype == AFSI_C128),
                     "X0 must be R64 (real A) or C128 (complex A)");
        AFSI_REQUIRE(X0->rows == A->n && X0->cols >= 1 && X0->cols <= A->n && X0->ptr,
                     "X0 must be n x p with 1 <= p <= n");
        AFSI_REQUIRE(X0->ld >= X0->cols, "X0 ld < cols");
        AFSI_REQUIRE(evecs->dtype == dt && evecs->rows == A->n && evecs->cols >= capacity &&
                         capacity >= 0 && evecs->ld >= evecs->cols,
                     "evecs must be n x capacity of X0's dtype");
        AFSI_REQUIRE(capacity == 0 || (eigenvalues && residuals), "NULL eigenvalue/residual output");
        AFSI_REQUIRE(opts->kmax >= 1 && opts->max_iter >= 1, "kmax and max_iter must be >= 1");
        const int fdt = opts->filter_dtype;
        AFSI_REQUIRE(fdt >= AFSI_R64 && fdt <= AFSI_C64 && is_complex(fdt) == is_complex(dt),
                     "filter dtype must match the matrix domain");
        std::memset(result, 0, sizeof *result);
        DeviceGuard dg(A->device);
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);

        const int64_t n = A->n, p = X0->cols, ld = X0->ld;
        const int eb = elem_bytes(dt), feb = elem_bytes(fdt);
        const int kmax = opts->kmax;
        std::vector<double> coeffs(kmax + 1);
        filter_coefficients(A->lmin, A->lmax, a, b, kmax, opts->damping, opts->m_exp, coeffs.data());
        const double wdt = A->lmax - A->lmin;
        const double l1 = 2.0 / wdt, l2 = -(A->lmax + A->lmin) / wdt;
        int k_cur = kmax;
        if (opts->k_init > 0) {
            k_cur = std::min(opts->k_init, kmax);
        } else if (opts->adaptive) {
            const double ta = std::min(1.0, std::max(-1.0, (2 * a - A->lmax - A->lmin) / wdt));
            const double tb = std::min(1.0, std::max(-1.0, (2 * b - A->lmax - A->lmin) / wdt));
            const double width = std::acos(ta) - std::acos(tb);
            k_cur = (int)std::ceil(opts->C / width) - 1;  // eq. (compute_k_1)
            k_cur = std::max(1, std::min(k_cur, kmax));
        }
        const double normA = std::max(std::fabs(A->lmin), std::fabs(A->lmax));
        const double tau_abs = opts->tau_c * normA;

        // buffers: B[0] = active block (caller's X0), B[1], B[2] scratch n x p blocks
        DevBuf b1((size_t)n * ld * eb), b2((size_t)n * ld * eb);
        void *B0 = X0->ptr, *B1 = b1.p, *B2 = b2.p;
        const bool mixed = fdt != dt;
        DevBuf f0(mixed ? (size_t)n * ld * feb : 0), f1(mixed ? (size_t)n * ld * feb : 0),
            f2(mixed ? (size_t)n * ld * feb : 0);

        auto t0 = clk::now();
        orthonormalize_dev(dt, B0, B1, n, p, ld, s, nullptr);
        result->time_orth_ms += ms_since(t0);

        int64_t p_act = p;
        int64_t n_check_prev = 0;
        int64_t spmv = 0;
        std::vector<int> degrees;
        std::vector<double> ritz(p), res(p);
        std::vector<uint8_t> inI(p), lock(p);
        int it = 0;
        for (it = 1; it <= opts->max_iter; ++it) {
            // ---- filter (Algorithm 2)
            t0 = clk::now();
            if (!mixed) {
                filter_apply(A, coeffs.data(), k_cur, dt, B0, B1, B2, p_act, ld, s);
            } else {
                afsi_block src{B0, n, p_act, ld, dt}, x32{f0.p, n, p_act, ld, fdt};
                launch_convert(src, x32, s);
                filter_apply(A, coeffs.data(), k_cur, fdt, f0.p, f1.p, f2.p, p_act, ld, s);
                afsi_block y32{f1.p, n, p_act, ld, fdt}, dst{B1, n, p_act, ld, dt};
                launch_convert(y32, dst, s);
            }
            AFSI_HIP(hipStreamSynchronize(s));
            result->time_filter_ms += ms_since(t0);
            spmv += (int64_t)k_cur * p_act;
            degrees.push_back(k_cur);
            // ---- orthonormalise against the locked vectors
            t0 = clk::now();
            if (n_lock > 0) project_out_dev(dt, evecs->ptr, evecs->ld, n_lock, B1, ld, n, p_act, s);
            const double t_proj = ms_since(t0);
            // ---- Cholesky QR fused with Rayleigh-Ritz: V -> B0, AV -> B2 (the orthonormal
            // basis stays implicit)
            t0 = clk::now();
            double maxn2 = 0.0, t_orth = 0.0;
            orthonormalize_rr_dev(A, dt, B1, B2, B0, B2, n, p_act, ld, ritz.data(), s, &maxn2, &t_orth);
            result->time_orth_ms += t_proj + t_orth;
            result->time_rr_ms += ms_since(t0) - t_orth;
            // the Jackson / Lanczos filters are bounded by ~1 on [lmin, lmax]: a large
            // growth of an orthonormal input means A's spectrum leaves the bounds
            if (opts->damping != AFSI_DAMP_NONE && maxn2 > 16.0)
                AFSI_FAIL(AFSI_E_BOUNDS, "filtered block grew by %.3g: spectral bounds do not "
                          "enclose the spectrum", std::sqrt(maxn2));
            spmv += p_act;
            int64_t e = 0;
            for (int64_t j = 0; j < p_act; ++j) {
                inI[j] = ritz[j] >= a && ritz[j] <= b;
                e += inI[j];
            }
            if (e == 0) continue;
            auto th = clk::now();
            if (opts->adaptive)
                k_cur = select_degree(ritz.data(), p_act, e, coeffs.data(), kmax, l1, l2, opts->tau_a);
            result->time_host_ms += ms_since(th);
            // ---- residuals
            t0 = clk::now();
            residual_norms_host(dt, B0, ld, B2, ld, ritz.data(), n, p_act, res.data(), s);
            result->time_resid_ms += ms_since(t0);
            // ---- spurious-value test and locking
            th = clk::now();
            int done = 0;
            lock_select(ritz.data(), p_act, res.data(), inI.data(), a, b, tau_abs, n_lock,
                        &n_check_prev, lock.data(), &done);
            std::vector<int32_t> lk, keep;
            for (int64_t j = 0; j < p_act; ++j) (lock[j] ? lk : keep).push_back((int32_t)j);
            if (!lk.empty()) {
                if (n_lock + (int64_t)lk.size() > capacity)
                    AFSI_FAIL(AFSI_E_INVALID, "more than %lld eigenpairs locked (capacity)",
                              (long long)capacity);
                for (size_t t = 0; t < lk.size(); ++t) {
                    eigenvalues[n_lock + t] = ritz[lk[t]];
                    residuals[n_lock + t] = res[lk[t]];
                }
                gather(dt, B0, n, ld, lk, (char *)evecs->ptr + (size_t)n_lock * eb, evecs->ld, s);
                gather(dt, B0, n, ld, keep, B2, ld, s);
                std::swap(B0, B2);
                n_lock += (int64_t)lk.size();
                p_act -= (int64_t)lk.size();
            }
            result->time_host_ms += ms_since(th);
            if (done) {
                converged = 1;
                break;
            }
        }
        // the active block may have moved into a scratch buffer: X0 is consumed either way
        // sort the locked pairs by eigenvalue (columns permuted through B1)
        if (n_lock > 1) {
            std::vector<int32_t> order(n_lock);
            std::iota(order.begin(), order.end(), 0);
            std::stable_sort(order.begin(), order.end(),
                             [&](int32_t x, int32_t y) { return eigenvalues[x] < eigenvalues[y]; });
            std::vector<double> ev(eigenvalues, eigenvalues + n_lock), rs(residuals, residuals + n_lock);
            for (int64_t t = 0; t < n_lock; ++t) {
                eigenvalues[t] = ev[order[t]];
                residuals[t] = rs[order[t]];
            }
            // B1 holds at least p >= ... columns; use a dedicated buffer when n_lock > ld
            DevBuf tmp((size_t)n * n_lock * eb);
            gather(dt, evecs->ptr, n, evecs->ld, order, tmp.p, n_lock, s);
            AFSI_HIP(hipMemcpy2DAsync(evecs->ptr, evecs->ld * eb, tmp.p, n_lock * eb, n_lock * eb, n,
                                      hipMemcpyDeviceToDevice, s));
            AFSI_HIP(hipStreamSynchronize(s));
        }
        result->count = n_lock;
        result->iterations = std::min(it, opts->max_iter);
        result->converged = converged;
        result->spmv = spmv;
        result->avg_degree =
            degrees.empty() ? 0.0 : std::accumulate(degrees.begin(), degrees.end(), 0.0) / degrees.size();
        AFSI_HIP(hipStreamSynchronize(s));
    });
    if (status == AFSI_OK && !converged) {
        set_error("iteration limit reached with %lld pairs locked", (long long)n_lock);
        return AFSI_E_NOCONV;
    }
    return status;
}

int afsi_estimate_spectral_bounds(afsi_matrix_t A, int steps, uint64_t seed, void *stream,
                                  double *lmin, double *lmax) {
    return guarded([&] {
        AFSI_REQUIRE(A != nullptr, "matrix handle is NULL");
        AFSI_REQUIRE(steps >= 2, "need at least 2 Lanczos steps");
        AFSI_REQUIRE(A->n >= 1, "empty matrix");
        DeviceGuard dg(A->device);
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        const int dt = A->dtype;  // R64 or C128
        const int comp = dt == AFSI_C128 ? 2 : 1;
        const int64_t n = A->n;
        const int m = (int)std::min<int64_t>(steps, n);
        const int64_t ld = m + 1;
        DevBuf Q((size_t)n * ld * comp * sizeof(double));
        DevBuf h((size_t)(ld + 2) * comp * sizeof(double));
        std::vector<double> alpha, beta, hh((size_t)(ld + 2) * comp);
        double *Qd = (double *)Q.p, *hd = (double *)h.p;
        // start vector: N(0,1) entries from the device's counter-based generator keyed by
        // `seed` (written in place in the strided first column), normalised
        launch_fill_normal(Qd, n, 1, ld, comp, seed, s);
        inner_dev(dt, Qd, ld, Qd, ld, n, 1, 1, hd, 1, s);
        AFSI_HIP(hipMemcpyAsync(hh.data(), hd, comp * sizeof(double), hipMemcpyDeviceToHost, s));
        AFSI_HIP(hipStreamSynchronize(s));
        AFSI_REQUIRE(hh[0] > 0.0, "start vector of the bounds estimate is zero");
        launch_scale(Qd, n, ld, comp, 1.0 / std::sqrt(hh[0]), s);
        double last_beta = 0.0;
        for (int j = 0; j < m; ++j) {
            double *qj = Qd + (size_t)j * comp, *w = Qd + (size_t)(j + 1) * comp;
            spmm_apply(A, dt, qj, w, 1, ld, s);
            double aj = 0.0;
            for (int pass = 0; pass < 2; ++pass) {
                inner_dev(dt, Qd, ld, w, ld, n, j + 1, 1, hd, 1, s);
                AFSI_HIP(hipMemcpyAsync(hh.data(), hd, (size_t)(j + 1) * comp * sizeof(double),
                                        hipMemcpyDeviceToHost, s));
                gemm_dev(dt, Qd, ld, hd, 1, n, j + 1, 1, -1.0, 1.0, w, ld, s);
                AFSI_HIP(hipStreamSynchronize(s));
                aj += hh[(size_t)j * comp];
            }
            // ||w||
            inner_dev(dt, w, ld, w, ld, n, 1, 1, hd, 1, s);
            AFSI_HIP(hipMemcpyAsync(hh.data(), hd, comp * sizeof(double), hipMemcpyDeviceToHost, s));
            AFSI_HIP(hipStreamSynchronize(s));
            const double bj = std::sqrt(std::max(hh[0], 0.0));
            alpha.push_back(aj);
            last_beta = bj;
            if (j == m - 1 || bj == 0.0) break;
            beta.push_back(bj);
            launch_scale(w, n, ld, comp, 1.0 / bj, s);
        }
        const int k = (int)alpha.size();
        std::vector<double> T((size_t)k * k, 0.0), th(k), S((size_t)k * k);
        for (int i = 0; i < k; ++i) {
            T[(size_t)i * k + i] = alpha[i];
            if (i + 1 < k) T[(size_t)i * k + i + 1] = T[(size_t)(i + 1) * k + i] = beta[i];
        }
        host_eigh_or_throw(k, false, T.data(), k, th.data(), S.data(), k);
        const double rlo = std::fabs(last_beta * S[(size_t)(k - 1) * k + 0]);
        const double rhi = std::fabs(last_beta * S[(size_t)(k - 1) * k + (k - 1)]);
        const double spread = th[k - 1] - th[0];
        double lo = th[0] - rlo - 1e-3 * spread, hi = th[k - 1] + rhi + 1e-3 * spread;
        if (!(hi > lo)) hi = lo + 1.0;
        A->lmin = lo;
        A->lmax = hi;
        A->has_bounds = true;
        if (lmin) *lmin = lo;
        if (lmax) *lmax = hi;
    });
}

}  // extern "C"
