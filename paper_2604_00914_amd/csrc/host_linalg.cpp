// Small dense Hermitian linear algebra on the host (FP64), p up to a few thousand.
//
//  * host_cholesky_inverse: R^{-1} for the Cholesky factor R^H R = G + shift I, with
//    symmetric diagonal scaling (G -> D G D, unit diagonal) before factoring; used by
//    Cholesky QR, where only X R^{-1} is needed.
//  * host_eigh: Hermitian eigendecomposition B = U diag(w) U^H.  Householder
//    reduction to tridiagonal form (complex reflectors for Hermitian B), a diagonal
//    unitary scaling that makes the off-diagonal real and non-negative, then the
//    implicit symmetric QR iteration with Wilkinson shifts on the real tridiagonal
//    (Golub & Van Loan, Matrix Computations, ch. 8.3), accumulating rotations.
#include <algorithm>
#include <cmath>
#include <complex>
#include <limits>
#include <numeric>
#include <vector>

#include "internal.h"

namespace afsi {

using cd = std::complex<double>;

template <class T>
static inline double absq(const T &x) { return std::norm(x); }
static inline double absq(double x) { return x * x; }
static inline double conjv(double x) { return x; }
static inline cd conjv(const cd &x) { return std::conj(x); }
static inline double realv(double x) { return x; }
static inline double realv(const cd &x) { return x.real(); }

template <class T>
static bool chol_inv_impl(int64_t p, T *G, int64_t ld, double shift) {
    // H = G + shift I, scaled to unit diagonal
    std::vector<double> dscale(p);
    for (int64_t i = 0; i < p; ++i) {
        const double h = realv(G[i * ld + i]) + shift;
        if (!(h > 0.0) || !std::isfinite(h)) return false;
        dscale[i] = 1.0 / std::sqrt(h);
    }
    std::vector<T> R((size_t)p * p, T(0));
    for (int64_t i = 0; i < p; ++i)
        for (int64_t j = i; j < p; ++j) {
            T h = G[i * ld + j];
            if (i == j) h = T(realv(h) + shift);
            R[i * p + j] = h * (dscale[i] * dscale[j]);
        }
    // upper Cholesky in place: R^H R = H'
    for (int64_t j = 0; j < p; ++j) {
        double dj = realv(R[j * p + j]);
        for (int64_t k = 0; k < j; ++k) dj -= absq(R[k * p + j]);
        if (!(dj > 0.0) || !std::isfinite(dj)) return false;
        const double rjj = std::sqrt(dj);
        R[j * p + j] = T(rjj);
        for (int64_t i = j + 1; i < p; ++i) {
            T s = R[j * p + i];
            for (int64_t k = 0; k < j; ++k) s -= conjv(R[k * p + j]) * R[k * p + i];
            R[j * p + i] = s / rjj;
        }
    }
    // Z = R^{-1} (upper), column by column: R Z = I
    std::vector<T> Z((size_t)p * p, T(0));
    for (int64_t j = 0; j < p; ++j) {
        Z[j * p + j] = T(1.0) / R[j * p + j];
        for (int64_t i = j - 1; i >= 0; --i) {
            T s = T(0);
            for (int64_t k = i + 1; k <= j; ++k) s += R[i * p + k] * Z[k * p + j];
            Z[i * p + j] = -s / R[i * p + i];
        }
    }
    // (D^{-1} R')^{-1} ... : H = D^{-1} R'^H R' D^{-1}, so R = R' D^{-1}, R^{-1} = D R'^{-1}
    for (int64_t i = 0; i < p; ++i)
        for (int64_t j = 0; j < p; ++j) G[i * ld + j] = j >= i ? Z[i * p + j] * dscale[i] : T(0);
    return true;
}

bool host_cholesky_inverse(int64_t p, bool cplx, double *G, int64_t ld, double shift) {
    if (cplx) return chol_inv_impl<cd>(p, reinterpret_cast<cd *>(G), ld, shift);
    return chol_inv_impl<double>(p, G, ld, shift);
}

// Implicit symmetric tridiagonal QR with Wilkinson shift.  d[0..p), e[0..p-1).
// Zt is p x p row-major holding Z^T (row k = k-th column of Z); rotations are
// accumulated so that T_original = Z diag(d) Z^T on return.
static void tridiag_qr(int64_t p, std::vector<double> &d, std::vector<double> &e,
                       std::vector<double> &Zt) {
    const double eps = std::numeric_limits<double>::epsilon();
    int64_t iter = 0;
    const int64_t max_iter = 60 * std::max<int64_t>(p, 1);
    int64_t hi = p - 1;
    while (hi > 0) {
        // deflate negligible off-diagonals
        for (int64_t i = 0; i < hi; ++i)
            if (std::fabs(e[i]) <= eps * (std::fabs(d[i]) + std::fabs(d[i + 1]))) e[i] = 0.0;
        while (hi > 0 && e[hi - 1] == 0.0) --hi;
        if (hi == 0) break;
        int64_t lo = hi - 1;
        while (lo > 0 && e[lo - 1] != 0.0) --lo;
        if (++iter > max_iter) AFSI_FAIL(AFSI_E_HIP, "tridiagonal QR did not converge");
        // Wilkinson shift from the trailing 2x2 block
        const double delta = 0.5 * (d[hi - 1] - d[hi]);
        const double eb = e[hi - 1];
        const double den = delta + (delta >= 0 ? 1.0 : -1.0) * std::hypot(delta, eb);
        const double mu = den != 0.0 ? d[hi] - eb * eb / den : d[hi];
        double x = d[lo] - mu, z = e[lo];
        for (int64_t k = lo; k < hi; ++k) {
            const double r = std::hypot(x, z);
            double c = 1.0, s = 0.0;
            if (r != 0.0) c = x / r, s = z / r;
            if (k > lo) e[k - 1] = r;
            const double a = d[k], b = e[k], cc = d[k + 1];
            d[k] = c * c * a + 2.0 * c * s * b + s * s * cc;
            d[k + 1] = s * s * a - 2.0 * c * s * b + c * c * cc;
            e[k] = c * s * (cc - a) + (c * c - s * s) * b;
            if (k + 1 < hi) {
                z = s * e[k + 1];
                e[k + 1] = c * e[k + 1];
                x = e[k];
            }
            double *zk = &Zt[k * p], *zk1 = &Zt[(k + 1) * p];
            for (int64_t i = 0; i < p; ++i) {
                const double u = zk[i], v = zk1[i];
                zk[i] = c * u + s * v;
                zk1[i] = -s * u + c * v;
            }
        }
    }
}

template <class T>
static void eigh_impl(int64_t p, const T *B, int64_t ldb, double *w, T *U, int64_t ldu) {
    std::vector<T> A((size_t)p * p);
    for (int64_t i = 0; i < p; ++i)
        for (int64_t j = 0; j < p; ++j) A[i * p + j] = B[i * ldb + j];
    // Hermitian part (inputs are Hermitian up to rounding)
    for (int64_t i = 0; i < p; ++i) {
        A[i * p + i] = T(realv(A[i * p + i]));
        for (int64_t j = i + 1; j < p; ++j) {
            const T h = 0.5 * (A[i * p + j] + conjv(A[j * p + i]));
            A[i * p + j] = h;
            A[j * p + i] = conjv(h);
        }
    }
    std::vector<T> Q((size_t)p * p, T(0));
    for (int64_t i = 0; i < p; ++i) Q[i * p + i] = T(1);
    std::vector<T> v(p), u(p), wv(p);
    // Householder reduction: column k below the diagonal -> alpha e_1
    for (int64_t k = 0; k + 2 < p; ++k) {
        const int64_t m = p - k - 1;  // length of x = A[k+1:, k]
        double xn2 = 0.0;
        for (int64_t i = 0; i < m; ++i) xn2 += absq(A[(k + 1 + i) * p + k]);
        const double xn = std::sqrt(xn2);
        if (xn == 0.0) continue;
        const T x0 = A[(k + 1) * p + k];
        const double ax0 = std::sqrt(absq(x0));
        const T phase = ax0 > 0 ? x0 / ax0 : T(1);
        const T alpha = -phase * xn;
        for (int64_t i = 0; i < m; ++i) v[i] = A[(k + 1 + i) * p + k];
        v[0] -= alpha;
        double vn2 = 0.0;
        for (int64_t i = 0; i < m; ++i) vn2 += absq(v[i]);
        const double vn = std::sqrt(vn2);
        if (vn == 0.0) continue;
        for (int64_t i = 0; i < m; ++i) v[i] /= vn;
        // u = A_sub v, gamma = v^H u, w = 2u - 2 gamma v, A_sub -= v w^H + w v^H
        for (int64_t i = 0; i < m; ++i) {
            T s = T(0);
            const T *ar = &A[(k + 1 + i) * p + k + 1];
            for (int64_t j = 0; j < m; ++j) s += ar[j] * v[j];
            u[i] = s;
        }
        T gamma = T(0);
        for (int64_t i = 0; i < m; ++i) gamma += conjv(v[i]) * u[i];
        const double g = realv(gamma);
        for (int64_t i = 0; i < m; ++i) wv[i] = 2.0 * u[i] - 2.0 * g * v[i];
        for (int64_t i = 0; i < m; ++i) {
            T *ar = &A[(k + 1 + i) * p + k + 1];
            for (int64_t j = 0; j < m; ++j) ar[j] -= v[i] * conjv(wv[j]) + wv[i] * conjv(v[j]);
        }
        A[(k + 1) * p + k] = alpha;
        A[k * p + k + 1] = conjv(alpha);
        for (int64_t i = 1; i < m; ++i) A[(k + 1 + i) * p + k] = A[k * p + k + 1 + i] = T(0);
        // Q <- Q H on columns k+1..p-1
        for (int64_t r = 0; r < p; ++r) {
            T *qr = &Q[r * p + k + 1];
            T s = T(0);
            for (int64_t j = 0; j < m; ++j) s += qr[j] * v[j];
            s *= 2.0;
            for (int64_t j = 0; j < m; ++j) qr[j] -= s * conjv(v[j]);
        }
    }
    // real tridiagonal via phases delta_{k+1} = delta_k e_k / |e_k|
    std::vector<double> d(p), e(p > 0 ? p - 1 : 0);
    std::vector<T> delta(p, T(1));
    for (int64_t k = 0; k < p; ++k) d[k] = realv(A[k * p + k]);
    for (int64_t k = 0; k + 1 < p; ++k) {
        const T ek = A[(k + 1) * p + k];
        const double ae = std::sqrt(absq(ek));
        e[k] = ae;
        delta[k + 1] = ae > 0 ? delta[k] * (ek / ae) : delta[k];
    }
    std::vector<double> Zt((size_t)p * p, 0.0);
    for (int64_t i = 0; i < p; ++i) Zt[i * p + i] = 1.0;
    tridiag_qr(p, d, e, Zt);
    std::vector<int64_t> order(p);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return d[a] < d[b]; });
    // U = Q diag(delta) Z
    std::vector<T> QD((size_t)p * p);
    for (int64_t r = 0; r < p; ++r)
        for (int64_t k = 0; k < p; ++k) QD[r * p + k] = Q[r * p + k] * delta[k];
    for (int64_t jj = 0; jj < p; ++jj) {
        const int64_t j = order[jj];
        w[jj] = d[j];
        const double *z = &Zt[j * p];
        for (int64_t r = 0; r < p; ++r) {
            const T *qd = &QD[r * p];
            T s = T(0);
            for (int64_t k = 0; k < p; ++k) s += qd[k] * z[k];
            U[r * ldu + jj] = s;
        }
    }
}

void host_eigh(int64_t p, bool cplx, const double *B, int64_t ldb, double *w, double *U,
               int64_t ldu) {
    if (cplx)
        eigh_impl<cd>(p, reinterpret_cast<const cd *>(B), ldb, w, reinterpret_cast<cd *>(U), ldu);
    else
        eigh_impl<double>(p, B, ldb, w, U, ldu);
}

}  // namespace afsi
