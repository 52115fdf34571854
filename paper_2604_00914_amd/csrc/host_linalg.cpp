// Small dense Hermitian linear algebra on the host (FP64), p up to a few thousand.
// Built with the host compiler and OpenMP (no HIP).
//
//  * host_cholesky_inverse: R^{-1} for the Cholesky factor R^H R = G + shift I, with
//    symmetric diagonal scaling (G -> D G D, unit diagonal) before factoring; used by
//    Cholesky QR, where only X R^{-1} is needed.  Right-looking factorisation in
//    panels and a row-block inverse, both with register-tiled updates.
//  * host_eigh: Hermitian eigendecomposition B = U diag(w) U^H (Golub & Van Loan,
//    Matrix Computations, ch. 8.3): Householder reduction to tridiagonal form
//    (complex reflectors for Hermitian B), a diagonal unitary scaling that makes the
//    off-diagonal real, the tridiagonal's eigenpairs by divide and conquer (Golub & Van
//    Loan ch. 8.4; Gu & Eisenstat's eigenvectors) with the implicit symmetric QR
//    iteration with Wilkinson shifts for blocks of at most 32 (and as the fallback), then
//    U = H_0 ... H_{p-3} diag(delta) Z.  Reflectors (and the QR path's rotations) are
//    applied to column chunks of the eigenvector matrix in parallel.
//
// Compiled twice (AFSI_ISA_NS = generic, and avx2 with -mavx2 -mfma); the entry
// points in host_linalg_dispatch.cpp pick one at run time.
#include "host_linalg.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <omp.h>
#include <type_traits>
#include <cstdlib>
#include <new>
#include <limits>
#include <numeric>
#include <vector>

#ifndef AFSI_ISA_NS
#define AFSI_ISA_NS generic
#endif

namespace afsi {
namespace AFSI_ISA_NS {

using cd = std::complex<double>;

static inline double absq(double x) { return x * x; }
static inline double absq(const cd &x) { return std::norm(x); }
static inline double conjv(double x) { return x; }
static inline cd conjv(const cd &x) { return std::conj(x); }
static inline double realv(double x) { return x; }
static inline double realv(const cd &x) { return x.real(); }

static const int64_t kParallelMin = 160;  // below this size threads cost more than they save
// the Householder reduction synchronises its threads several times per column, which
// only pays for larger matrices (size in real units: a complex p counts 2p)
static const int64_t kHouseholderParallelMin = 320;
static const int64_t kChunk = 32;         // columns per task when applying rotations / reflectors

// Row-major scratch matrix whose rows start on 64-byte cache lines, so that column
// chunks owned by different threads never share a line (a shared line would move
// between cores on every rotation).
template <class T>
struct LineMatrix {
    int64_t ld = 0;
    T *data = nullptr;
    LineMatrix(int64_t rows, int64_t cols) {
        const int64_t per_line = 64 / (int64_t)sizeof(T);
        ld = (cols + per_line - 1) / per_line * per_line;
        const size_t bytes = (size_t)std::max<int64_t>(rows * ld, 1) * sizeof(T);
        data = static_cast<T *>(std::aligned_alloc(64, (bytes + 63) / 64 * 64));
        if (!data) throw std::bad_alloc();
        std::fill(data, data + rows * ld, T(0));
    }
    ~LineMatrix() { std::free(data); }
    LineMatrix(const LineMatrix &) = delete;
    LineMatrix &operator=(const LineMatrix &) = delete;
    T *row(int64_t r) { return data + r * ld; }
};

// sqrt(x^2 + z^2) without the cost of std::hypot when no scaling is needed
static inline double fast_hypot(double x, double z) {
    const double s = x * x + z * z;
    if (s > 1e-290 && s < 1e290) return std::sqrt(s);
    return std::hypot(x, z);
}

// sum_j a[j] * b[j] with kDotLanes independent partial sums, added in a fixed order
// at the end: the lanes map onto packed registers, so the loop vectorises without
// reassociation
static const int kDotLanes = 16;
template <class T>
static inline T dot_lanes(const T *a, const T *b, int64_t m) {
    T acc[kDotLanes];
    for (int t = 0; t < kDotLanes; ++t) acc[t] = T(0);
    int64_t j = 0;
    for (; j + kDotLanes <= m; j += kDotLanes)
        for (int t = 0; t < kDotLanes; ++t) acc[t] += a[j + t] * b[j + t];
    for (int t = 0; j < m; ++j, ++t) acc[t] += a[j] * b[j];
    for (int w = kDotLanes / 2; w > 0; w /= 2)
        for (int t = 0; t < w; ++t) acc[t] += acc[t + w];
    return acc[0];
}

// C[r][c] -= sum_{k<kb} op(A)[r][k] * B[k][c] on an RB x CB register tile:
// op(A)[r][k] = conj(A[k * lda + r]) (TRANS_A, the panel of the Cholesky update) or
// A[r * lda + k].  Full tiles only; the caller masks what it stores.
constexpr int kRB = 4, kCB = 8;
template <class T, bool TRANS_A>
static inline void tile_product(int64_t kb, const T *A, int64_t lda, const T *B, int64_t ldb,
                                T (&acc)[kRB][kCB]) {
    for (int r = 0; r < kRB; ++r)
        for (int c = 0; c < kCB; ++c) acc[r][c] = T(0);
    for (int64_t k = 0; k < kb; ++k) {
        T f[kRB], v[kCB];
        for (int r = 0; r < kRB; ++r) f[r] = TRANS_A ? conjv(A[k * lda + r]) : A[r * lda + k];
        const T *bk = B + k * ldb;
        for (int c = 0; c < kCB; ++c) v[c] = bk[c];
        for (int r = 0; r < kRB; ++r)
            for (int c = 0; c < kCB; ++c) acc[r][c] += f[r] * v[c];
    }
}

// Upper part of H (m x m, ldh) -= P^H P for the kb x m panel P (ldp): H[i][l] for l >= i.
// Rows and columns are processed in register tiles; P is padded by the caller to a whole
// number of tiles in both directions (zero columns), so tiles never read past it.
template <class T>
static void update_upper(int64_t m, int64_t kb, const T *P, int64_t ldp, T *H, int64_t ldh) {
    for (int64_t i0 = 0; i0 < m; i0 += kRB)
        for (int64_t l0 = i0 / kCB * kCB; l0 < m; l0 += kCB) {
            T acc[kRB][kCB];
            tile_product<T, true>(kb, P + i0, ldp, P + l0, ldp, acc);
            for (int r = 0; r < kRB && i0 + r < m; ++r) {
                T *hr = H + (i0 + r) * ldh;
                for (int c = 0; c < kCB && l0 + c < m; ++c)
                    if (l0 + c >= i0 + r) hr[l0 + c] -= acc[r][c];
            }
        }
}

// Cholesky QR's host factor: R^{-1} with R^H R = G + shift I (upper R), computed on the
// unit-diagonal scaling H' = D (G + shift I) D, D = diag(1/sqrt(G_ii + shift)).
// Factorisation: right-looking in panels of kPanel rows, each panel finished row by row
// and then subtracted from the trailing rows as one register-tiled update (the trailing
// matrix is read once per panel instead of once per row).  Inverse: Z = R'^{-1} by row
// blocks from the bottom, each block's contribution of the rows below as one tiled
// product.  R = R' D^{-1}, so R^{-1} = D R'^{-1}.  Single-threaded: on the 16-core host
// of the GPU machine p = 360 takes 0.56 ms on one thread and 0.68 ms on sixteen (the
// row-by-row version took 1.62 ms).
static const int64_t kPanel = 32;
template <class T>
static bool chol_inv_impl(int64_t p, T *G, int64_t ld, double shift) {
    std::vector<double> dscale(p);
    for (int64_t i = 0; i < p; ++i) {
        const double h = realv(G[i * ld + i]) + shift;
        if (!(h > 0.0) || !std::isfinite(h)) return false;
        dscale[i] = 1.0 / std::sqrt(h);
    }
    // work matrices padded to whole register tiles (pad columns and rows stay zero)
    const int64_t pp = (p + kCB - 1) / kCB * kCB + kCB;
    const int64_t pr = pp + kRB;
    // H' = D (G + shift I) D, upper triangle, row-major p x p (ld pp)
    std::vector<T> R((size_t)pr * pp, T(0));
    for (int64_t i = 0; i < p; ++i)
        for (int64_t j = i; j < p; ++j) {
            T h = G[i * ld + j];
            if (i == j) h = T(realv(h) + shift);
            R[i * pp + j] = h * (dscale[i] * dscale[j]);
        }
    for (int64_t k0 = 0; k0 < p; k0 += kPanel) {
        const int64_t k1 = std::min(p, k0 + kPanel);
        // finish rows k0..k1-1: scale row j, subtract it from the later rows of the panel
        for (int64_t j = k0; j < k1; ++j) {
            T *rj = &R[j * pp];
            const double d = realv(rj[j]);
            if (!(d > 0.0) || !std::isfinite(d)) return false;
            const double rjj = std::sqrt(d);
            rj[j] = T(rjj);
            const double inv = 1.0 / rjj;
            for (int64_t l = j + 1; l < p; ++l) rj[l] *= inv;
            for (int64_t i = j + 1; i < k1; ++i) {
                const T f = conjv(rj[i]);
                T *ri = &R[i * pp];
                for (int64_t l = i; l < p; ++l) ri[l] -= f * rj[l];
            }
        }
        // trailing rows k1..p-1 minus the panel's contribution
        if (k1 < p) update_upper<T>(p - k1, k1 - k0, &R[k0 * pp + k1], pp, &R[k1 * pp + k1], pp);
    }
    // Z = R'^{-1} (upper), by row blocks from the bottom:
    //   Z[i, :] = (e_i - sum_{k > i} R'[i, k] Z[k, :]) / R'_ii
    std::vector<T> Z((size_t)pr * pp, T(0));
    for (int64_t i1 = p; i1 > 0;) {
        const int64_t i0 = std::max<int64_t>(0, i1 - kPanel);
        // rows below the block: Z[i, j] -= sum_{k >= i1} R'[i, k] Z[k, j] for j >= i1, as
        // tiles of kRB rows (rows past the block compute into a scratch tile and are dropped)
        if (i1 < p) {
            const int64_t jt0 = i1 / kCB * kCB;
            for (int64_t r0 = i0; r0 < i1; r0 += kRB)
                for (int64_t j0 = jt0; j0 < p; j0 += kCB) {
                    T acc[kRB][kCB];
                    // k runs over i1 .. min(p, j0 + kCB): Z[k][j] = 0 for j < k
                    const int64_t kend = std::min(p, j0 + kCB);
                    tile_product<T, false>(kend - i1, &R[r0 * pp + i1], pp, &Z[i1 * pp + j0], pp, acc);
                    for (int r = 0; r < kRB && r0 + r < i1; ++r)
                        for (int c = 0; c < kCB && j0 + c < p; ++c)
                            if (j0 + c >= i1) Z[(r0 + r) * pp + j0 + c] -= acc[r][c];
                }
        }
        // inside the block, bottom row first
        for (int64_t i = i1 - 1; i >= i0; --i) {
            T *zi = &Z[i * pp];
            const T *ri = &R[i * pp];
            for (int64_t k = i + 1; k < i1; ++k) {
                const T f = ri[k];
                const T *zk = &Z[k * pp];
                for (int64_t j = k; j < p; ++j) zi[j] -= f * zk[j];
            }
            const T inv = T(1.0) / ri[i];
            for (int64_t j = i + 1; j < p; ++j) zi[j] *= inv;
            zi[i] = inv;
        }
        i1 = i0;
    }
    for (int64_t i = 0; i < p; ++i)
        for (int64_t j = 0; j < p; ++j) G[i * ld + j] = j >= i ? Z[i * pp + j] * dscale[i] : T(0);
    return true;
}

bool host_cholesky_inverse(int64_t p, bool cplx, double *G, int64_t ld, double shift) {
    if (cplx) return chol_inv_impl<cd>(p, reinterpret_cast<cd *>(G), ld, shift);
    return chol_inv_impl<double>(p, G, ld, shift);
}

struct Rot {
    int64_t k;
    double c, s;
};

// Implicit symmetric tridiagonal QR with Wilkinson shifts on d[0..p), e[0..p-1).
// Each plane rotation J (T <- J T J^T on rows/columns k, k+1, J = [[c, s], [-s, c]])
// is appended to `rots` in application order; T_original = Z diag(d) Z^T with
// Z = J_1^T J_2^T ... .
static bool tridiag_qr(int64_t p, std::vector<double> &d, std::vector<double> &e,
                       std::vector<Rot> &rots) {
    const double eps = std::numeric_limits<double>::epsilon();
    int64_t iter = 0;
    const int64_t max_iter = 60 * std::max<int64_t>(p, 1);
    int64_t hi = p - 1;
    while (hi > 0) {
        for (int64_t i = 0; i < hi; ++i)
            if (std::fabs(e[i]) <= eps * (std::fabs(d[i]) + std::fabs(d[i + 1]))) e[i] = 0.0;
        while (hi > 0 && e[hi - 1] == 0.0) --hi;
        if (hi == 0) break;
        int64_t lo = hi - 1;
        while (lo > 0 && e[lo - 1] != 0.0) --lo;
        if (++iter > max_iter) return false;
        const double delta = 0.5 * (d[hi - 1] - d[hi]);
        const double eb = e[hi - 1];
        const double den = delta + (delta >= 0 ? 1.0 : -1.0) * fast_hypot(delta, eb);
        const double mu = den != 0.0 ? d[hi] - eb * eb / den : d[hi];
        double x = d[lo] - mu, z = e[lo];
        for (int64_t k = lo; k < hi; ++k) {
            const double r = fast_hypot(x, z);
            double c = 1.0, s = 0.0;
            if (r != 0.0) {
                const double rinv = 1.0 / r;
                c = x * rinv;
                s = z * rinv;
            }
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
            rots.push_back({k, c, s});
        }
    }
    return true;
}

// Applies the recorded rotations, in order, to columns [i0, i0 + width) of Zt (W > 0:
// width == W, known at compile time).  The rotations of one QR sweep act on rows
// (k, k+1), (k+1, k+2), ...: the row they share stays in `carry`, so each rotation
// reads one row and writes one instead of two and two.
template <int W>
static void rotate_columns(LineMatrix<double> &Zt, const std::vector<Rot> &rots, int64_t i0,
                           int64_t width) {
    constexpr int kMax = W > 0 ? W : kChunk;
    const int64_t nw = W > 0 ? W : width;
    double carry[kMax];
    int64_t held = -1;  // row whose current values are in carry (memory copy is stale)
    for (const Rot &r : rots) {
        if (r.k != held) {
            if (held >= 0) {
                double *zh = Zt.row(held) + i0;
                for (int64_t i = 0; i < nw; ++i) zh[i] = carry[i];
            }
            const double *zk = Zt.row(r.k) + i0;
            for (int64_t i = 0; i < nw; ++i) carry[i] = zk[i];
        }
        double *__restrict__ zk = Zt.row(r.k) + i0;
        const double *__restrict__ zn = Zt.row(r.k + 1) + i0;
        const double c = r.c, s = r.s;
        for (int64_t i = 0; i < nw; ++i) {
            const double a = carry[i], b = zn[i];
            zk[i] = c * a + s * b;
            carry[i] = -s * a + c * b;
        }
        held = r.k + 1;
    }
    if (held >= 0) {
        double *zh = Zt.row(held) + i0;
        for (int64_t i = 0; i < nw; ++i) zh[i] = carry[i];
    }
}

// ---------------------------------------------------------------- divide and conquer
//
// Eigenpairs of a real symmetric tridiagonal matrix (d, e) by Cuppen's divide and
// conquer with Gu and Eisenstat's eigenvector formula (SIAM J. Matrix Anal. Appl. 16,
// 1995), as in Golub & Van Loan ch. 8.4.  The matrix is torn at its middle,
//   T = diag(T1', T2') + rho v v^T,  rho = |beta|, v = e_{m-1} + sign(beta) e_m,
// where beta = e[m-1] and T1', T2' have |beta| taken off their touching diagonal
// entries; the halves are solved recursively (T_i' = Q_i D_i Q_i^T) and the rank-one
// update D + rho z z^T, z = diag(Q1, Q2)^T v, is solved by its secular equation
//   f(lambda) = 1 + rho sum_i z_i^2 / (d_i - lambda) = 0,
// one root in each gap of the poles.  Entries with a negligible z_i, and one of two
// poles closer than the tolerance (after a plane rotation that zeroes its z entry),
// are deflated: they keep their pole as eigenvalue and their column of diag(Q1, Q2) as
// eigenvector.  Each root is found as an offset tau from its nearer pole, so every
// difference d_i - lambda_j = (d_i - d_origin) - tau is accurate; z is then recomputed
// from the roots by Loewner's formula, which makes the eigenvectors
// u_j = (zhat_i / (d_i - lambda_j))_i numerically orthogonal.  The new eigenvectors are
// diag(Q1, Q2) [deflated columns | Q_k U] with one dense product.  Small blocks use the
// QR iteration.

static const int64_t kDcLeaf = 32;

// Eigenpairs of a tridiagonal of order n <= kDcLeaf by the QR iteration: Z (n x n,
// row-major, ldz) column j the eigenvector of d[j], d ascending.
static bool dc_leaf(int64_t n, double *d, const double *e, double *Z, int64_t ldz) {
    std::vector<double> dd(d, d + n), ee(n > 1 ? n - 1 : 0);
    for (int64_t i = 0; i + 1 < n; ++i) ee[i] = e[i];
    std::vector<Rot> rots;
    if (!tridiag_qr(n, dd, ee, rots)) return false;
    std::vector<double> Zt((size_t)n * n, 0.0);  // row k = column k of Z
    for (int64_t i = 0; i < n; ++i) Zt[(size_t)i * n + i] = 1.0;
    for (const Rot &r : rots) {
        double *zk = &Zt[(size_t)r.k * n], *zn = &Zt[(size_t)(r.k + 1) * n];
        for (int64_t i = 0; i < n; ++i) {
            const double a = zk[i], b = zn[i];
            zk[i] = r.c * a + r.s * b;
            zn[i] = -r.s * a + r.c * b;
        }
    }
    std::vector<int64_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return dd[a] < dd[b]; });
    for (int64_t j = 0; j < n; ++j) {
        d[j] = dd[order[j]];
        for (int64_t i = 0; i < n; ++i) Z[i * ldz + j] = Zt[(size_t)order[j] * n + i];
    }
    return true;
}

// Root j of the secular equation with poles p[0] < ... < p[k-1], weights w = rho z^2
// (all > 0): the root is found as origin + tau, origin its nearer pole; returns false
// if the iteration does not settle.  Steps: the two-pole rational model of Li's
// "middle way" (the poles left of the root summed as psi, those right as phi; each
// replaced by a constant plus one pole term matching its value and slope at tau, and
// the model's root taken), Newton where that model has no root between the poles, and
// bisection of the bracket where a step leaves it.
static bool secular_root(int64_t k, const double *p, const double *w, double rho, int64_t j,
                         double &origin, double &tau) {
    const double eps = std::numeric_limits<double>::epsilon();
    const double lo = p[j], hi = j + 1 < k ? p[j + 1] : p[k - 1] + rho;
    int64_t o = j;
    if (j + 1 < k) {  // which half of the gap holds the root: f at the midpoint
        const double mid = 0.5 * (lo + hi);
        double f = 1.0;
        for (int64_t i = 0; i < k; ++i) f += w[i] / (p[i] - mid);
        if (f < 0.0) o = j + 1;
    }
    origin = p[o];
    double a, b;  // bracket of tau: g(a) < 0 < g(b)
    if (o == j) {
        a = 0.0;
        b = j + 1 < k ? 0.5 * (hi - lo) : rho;
    } else {
        a = -0.5 * (hi - lo);
        b = 0.0;
    }
    std::vector<double> off(k);
    for (int64_t i = 0; i < k; ++i) off[i] = p[i] - origin;
    double t = 0.5 * (a + b);
    for (int it = 0; it < 400; ++it) {
        double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0;
        for (int64_t i = 0; i <= j; ++i) {
            const double q = 1.0 / (off[i] - t);
            psi += w[i] * q;
            dpsi += w[i] * q * q;
        }
        for (int64_t i = j + 1; i < k; ++i) {
            const double q = 1.0 / (off[i] - t);
            phi += w[i] * q;
            dphi += w[i] * q * q;
        }
        const double g = 1.0 + psi + phi, gp = dpsi + dphi;
        if (g == 0.0) break;
        if (g < 0.0) a = t; else b = t;
        if (b - a <= 2.0 * eps * std::max(std::fabs(a), std::fabs(b))) break;
        // two-pole model in the correction eta: c + B1 / (dl - eta) + B2 / (dr - eta) = 0
        double tn = t - g / gp;
        const double dl = off[j] - t;
        const double B1 = dpsi * dl * dl;
        double c = 1.0 + (psi - dpsi * dl), eta = 0.0;
        bool ok = false;
        if (j + 1 < k) {
            const double dr = off[j + 1] - t;
            const double B2 = dphi * dr * dr;
            c += phi - dphi * dr;
            // c eta^2 - (c (dl + dr) + B1 + B2) eta + (c dl dr + B1 dr + B2 dl) = 0,
            // the root with dl < eta < dr
            const double qa = c, qb = -(c * (dl + dr) + B1 + B2), qc = c * dl * dr + B1 * dr + B2 * dl;
            if (qa == 0.0) {
                if (qb != 0.0) { eta = -qc / qb; ok = true; }
            } else {
                const double disc = qb * qb - 4.0 * qa * qc;
                if (disc >= 0.0) {
                    const double qq = -0.5 * (qb + std::copysign(std::sqrt(disc), qb));
                    const double r1 = qq / qa, r2 = qq != 0.0 ? qc / qq : r1;
                    if (r1 > dl && r1 < dr) { eta = r1; ok = true; }
                    else if (r2 > dl && r2 < dr) { eta = r2; ok = true; }
                }
            }
        } else if (c != 0.0) {  // last root: no pole to the right, c (dl - eta) + B1 = 0
            eta = dl + B1 / c;
            ok = eta > dl;
        }
        if (ok) tn = t + eta;
        if (!(tn > a && tn < b)) tn = 0.5 * (a + b);
        if (tn == t) break;
        t = tn;
        if (it == 399) return false;
    }
    tau = t;
    return true;
}

// C (n x k, ldc) = A (n x k, lda) B (k x k, ldb), rows in parallel, four at a time, each
// four-row group in register tiles of eight columns; terms whose four A entries are all
// zero (the block structure of diag(Q1, Q2)) are skipped.  Every C entry sums its terms
// over l in order, as a plain loop would.
static void dense_product(int64_t n, int64_t k, const double *A, int64_t lda, const double *B,
                          int64_t ldb, double *C, int64_t ldc) {
#pragma omp parallel for schedule(static) if (n * k * k >= 4000000)
    for (int64_t i0 = 0; i0 < n; i0 += 4) {
        const int64_t rows = std::min<int64_t>(4, n - i0);
        if (rows < 4) {
            for (int64_t r = 0; r < rows; ++r) std::fill(C + (i0 + r) * ldc, C + (i0 + r) * ldc + k, 0.0);
            for (int64_t l = 0; l < k; ++l) {
                const double *b = B + l * ldb;
                for (int64_t r = 0; r < rows; ++r) {
                    const double a = A[(i0 + r) * lda + l];
                    if (a == 0.0) continue;
                    double *c = C + (i0 + r) * ldc;
                    for (int64_t j = 0; j < k; ++j) c[j] += a * b[j];
                }
            }
            continue;
        }
        const double *a0 = A + i0 * lda;
        int64_t jb = 0;
        for (; jb + 8 <= k; jb += 8) {
            double acc[4][8] = {};
            for (int64_t l = 0; l < k; ++l) {
                const double x0 = a0[l], x1 = a0[lda + l], x2 = a0[2 * lda + l], x3 = a0[3 * lda + l];
                if (x0 == 0.0 && x1 == 0.0 && x2 == 0.0 && x3 == 0.0) continue;
                const double *b = B + l * ldb + jb;
                for (int j = 0; j < 8; ++j) {
                    acc[0][j] += x0 * b[j];
                    acc[1][j] += x1 * b[j];
                    acc[2][j] += x2 * b[j];
                    acc[3][j] += x3 * b[j];
                }
            }
            for (int r = 0; r < 4; ++r)
                for (int j = 0; j < 8; ++j) C[(i0 + r) * ldc + jb + j] = acc[r][j];
        }
        for (; jb < k; ++jb) {
            for (int r = 0; r < 4; ++r) {
                double acc = 0.0;
                for (int64_t l = 0; l < k; ++l) {
                    const double a = a0[r * lda + l];
                    if (a != 0.0) acc += a * B[l * ldb + jb];
                }
                C[(i0 + r) * ldc + jb] = acc;
            }
        }
    }
}

// Eigenpairs of the tridiagonal (d, e) of order n: eigenvalues ascending in d, the
// eigenvectors in the columns of Z (n x n block of a row-major matrix with ldz).
static bool dc_eig(int64_t n, double *d, double *e, double *Z, int64_t ldz) {
    if (n <= kDcLeaf) return dc_leaf(n, d, e, Z, ldz);
    const double eps = std::numeric_limits<double>::epsilon();
    const int64_t m = n / 2;
    const double beta = e[m - 1], rb = std::fabs(beta), sg = beta < 0 ? -1.0 : 1.0;
    d[m - 1] -= rb;
    d[m] -= rb;
    for (int64_t i = 0; i < m; ++i) std::fill(Z + i * ldz + m, Z + i * ldz + n, 0.0);
    for (int64_t i = m; i < n; ++i) std::fill(Z + i * ldz, Z + i * ldz + m, 0.0);
    if (!dc_eig(m, d, e, Z, ldz)) return false;
    if (!dc_eig(n - m, d + m, e + m, Z + m * ldz + m, ldz)) return false;
    // z = diag(Q1, Q2)^T v: last row of Q1, sign(beta) times the first row of Q2
    std::vector<double> z(n);
    for (int64_t j = 0; j < m; ++j) z[j] = Z[(m - 1) * ldz + j];
    for (int64_t j = m; j < n; ++j) z[j] = sg * Z[m * ldz + j];
    double zn = 0.0;
    for (double x : z) zn += x * x;
    zn = std::sqrt(zn);
    for (double &x : z) x /= zn;
    const double rho = rb * zn * zn;
    // poles in ascending order (columns of Z follow through `perm`)
    std::vector<int64_t> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) { return d[a] < d[b]; });
    std::vector<double> ds(n), zs(n);
    for (int64_t i = 0; i < n; ++i) ds[i] = d[perm[i]], zs[i] = z[perm[i]];
    double dmax = 0.0;
    for (double x : ds) dmax = std::max(dmax, std::fabs(x));
    const double tol = 8.0 * eps * std::max(dmax, rho);
    // columns of diag(Q1, Q2) in pole order; deflating rotations act on them
    std::vector<double> Q((size_t)n * n);
#pragma omp parallel for schedule(static) if (n >= 128)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) Q[(size_t)i * n + j] = Z[i * ldz + perm[j]];
    std::vector<char> defl(n, 0);
    for (int64_t i = 0; i < n; ++i)
        if (rho * std::fabs(zs[i]) <= tol) defl[i] = 1;
    int64_t prev = -1;
    for (int64_t i = 0; i < n; ++i) {
        if (defl[i]) continue;
        if (prev >= 0 && ds[i] - ds[prev] <= tol) {
            // rotate (prev, i) so that z[prev] = 0: prev deflates
            const double r = std::hypot(zs[prev], zs[i]);
            const double c = zs[i] / r, s = -zs[prev] / r;
            zs[i] = r;
            zs[prev] = 0.0;
            const double dp = ds[prev], di = ds[i];
            ds[prev] = c * c * dp + s * s * di;
            ds[i] = s * s * dp + c * c * di;
            for (int64_t row = 0; row < n; ++row) {
                double *q = &Q[(size_t)row * n];
                const double a = q[prev], b = q[i];
                q[prev] = c * a + s * b;
                q[i] = -s * a + c * b;
            }
            defl[prev] = 1;
        }
        prev = i;
    }
    std::vector<int64_t> keep;
    for (int64_t i = 0; i < n; ++i)
        if (!defl[i]) keep.push_back(i);
    const int64_t k = (int64_t)keep.size();
    std::vector<double> pk(k), wk(k), zk(k), lam(k), org(k), tau(k);
    for (int64_t t = 0; t < k; ++t) {
        pk[t] = ds[keep[t]];
        zk[t] = zs[keep[t]];
        wk[t] = rho * zk[t] * zk[t];
    }
    for (int64_t t = 0; t + 1 < k; ++t)
        if (!(pk[t + 1] > pk[t])) return false;  // deflation keeps the poles apart
    bool ok = true;
#pragma omp parallel for schedule(dynamic, 8) if (k >= 128)
    for (int64_t j = 0; j < k; ++j) {
        if (!secular_root(k, pk.data(), wk.data(), rho, j, org[j], tau[j])) ok = false;
        lam[j] = org[j] + tau[j];
    }
    if (!ok) return false;
    // Loewner: zhat from the roots, pairing factors so that each ratio is at most one
    std::vector<double> zh(k);
#pragma omp parallel for schedule(static) if (k >= 128)
    for (int64_t i = 0; i < k; ++i) {
        auto diff = [&](int64_t j) { return (pk[i] - org[j]) - tau[j]; };  // d_i - lambda_j
        double v = -diff(k - 1) / rho;
        for (int64_t j = 0; j < i; ++j) v *= diff(j) / (pk[i] - pk[j]);
        for (int64_t j = i; j + 1 < k; ++j) v *= diff(j) / (pk[i] - pk[j + 1]);
        zh[i] = std::copysign(std::sqrt(std::fabs(v)), zk[i]);
    }
    // U (k x k): column j = (zhat_i / (d_i - lambda_j))_i, normalised
    std::vector<double> U((size_t)k * k);
#pragma omp parallel for schedule(static) if (k >= 128)
    for (int64_t j = 0; j < k; ++j) {
        double nrm = 0.0;
        for (int64_t i = 0; i < k; ++i) {
            const double u = zh[i] / ((pk[i] - org[j]) - tau[j]);
            U[(size_t)i * k + j] = u;
            nrm += u * u;
        }
        nrm = 1.0 / std::sqrt(nrm);
        for (int64_t i = 0; i < k; ++i) U[(size_t)i * k + j] *= nrm;
    }
    // new eigenvectors: Q_k U for the roots, the deflated columns as they are
    std::vector<double> Qk((size_t)n * k), QU((size_t)n * k);
#pragma omp parallel for schedule(static) if (n >= 128)
    for (int64_t row = 0; row < n; ++row)
        for (int64_t t = 0; t < k; ++t) Qk[(size_t)row * k + t] = Q[(size_t)row * n + keep[t]];
    dense_product(n, k, Qk.data(), k, U.data(), k, QU.data(), k);
    // all eigenvalues with their source: root t (>= 0) or deflated column -(i + 1)
    std::vector<std::pair<double, int64_t>> all;
    all.reserve(n);
    for (int64_t t = 0; t < k; ++t) all.push_back({lam[t], t});
    for (int64_t i = 0; i < n; ++i)
        if (defl[i]) all.push_back({ds[i], -(i + 1)});
    std::stable_sort(all.begin(), all.end(),
                     [](const std::pair<double, int64_t> &x, const std::pair<double, int64_t> &y) {
                         return x.first < y.first;
                     });
    // row by row (Z is row-major): column j of Z is root all[j].second's column of QU, or
    // a deflated column of Q
    for (int64_t j = 0; j < n; ++j) d[j] = all[j].first;
#pragma omp parallel for schedule(static) if (n >= 128)
    for (int64_t row = 0; row < n; ++row) {
        const double *qu = &QU[(size_t)row * k], *q = &Q[(size_t)row * n];
        double *z = Z + row * ldz;
        for (int64_t j = 0; j < n; ++j) {
            const int64_t src = all[j].second;
            z[j] = src >= 0 ? qu[src] : q[-src - 1];
        }
    }
    return true;
}

// Consecutive Householder reflectors H_k = I - 2 v_k v_k^H (v_k unit, acting on
// indices k+1..p-1; an empty v_k is the identity) grouped as
//   H_k0 H_k0+1 ... H_k0+cnt-1 = I - Vb T Vb^H
// (Schreiber & Van Loan's compact WY form): Vb holds v_k0+l in column l over rows
// k0+1..p-1 (row-major, zero above each vector's first row), T is cnt x cnt upper
// triangular with T_ll = tau_l and T[0:l, l] = -tau_l T[0:l, 0:l] (Vb[:, 0:l]^H v_l).
static const int64_t kReflBlock = 16;

template <class T>
struct ReflBlock {
    int64_t k0 = 0, cnt = 0;
    std::vector<T> V, Tm;  // Vb (rows x cnt, row-major), T (cnt x cnt, row-major)
};

template <class T>
static std::vector<ReflBlock<T>> reflector_blocks(int64_t p, const std::vector<std::vector<T>> &Vs) {
    std::vector<ReflBlock<T>> out;
    const int64_t nref = std::max<int64_t>(p - 2, 0);
    for (int64_t k0 = 0; k0 < nref; k0 += kReflBlock) {
        ReflBlock<T> rb;
        rb.k0 = k0;
        rb.cnt = std::min(kReflBlock, nref - k0);
        const int64_t cnt = rb.cnt, rows = p - k0 - 1;
        rb.V.assign((size_t)rows * cnt, T(0));
        std::vector<double> tau(cnt);
        for (int64_t l = 0; l < cnt; ++l) {
            const std::vector<T> &v = Vs[k0 + l];
            tau[l] = v.empty() ? 0.0 : 2.0;
            for (size_t i = 0; i < v.size(); ++i) rb.V[(size_t)(l + i) * cnt + l] = v[i];
        }
        rb.Tm.assign((size_t)cnt * cnt, T(0));
        std::vector<T> sv(cnt);
        for (int64_t l = 0; l < cnt; ++l) {
            for (int64_t m = 0; m < l; ++m) {
                T acc = T(0);
                for (int64_t r = l; r < rows; ++r)
                    acc += conjv(rb.V[(size_t)r * cnt + m]) * rb.V[(size_t)r * cnt + l];
                sv[m] = acc;
            }
            for (int64_t m = 0; m < l; ++m) {
                T acc = T(0);
                for (int64_t q = m; q < l; ++q) acc += rb.Tm[(size_t)m * cnt + q] * sv[q];
                rb.Tm[(size_t)m * cnt + l] = -tau[l] * acc;
            }
            rb.Tm[(size_t)l * cnt + l] = T(tau[l]);
        }
        out.push_back(std::move(rb));
    }
    return out;
}

// Register-tiled forms of the two block-reflector products of the back-transformation
// for real data, a chunk of kChunk columns and a block of a multiple of 4 reflectors.
// Each output element accumulates its terms in the same order as the plain loops (over
// rows r for W, over reflectors l for C), so the results are the same bits.
//   W (cnt x kChunk) = V^T C, V: rows x cnt (row-major), C: rows x kChunk (ld ldc)
static void refl_w_tiled(int64_t rows, int64_t cnt, const double *V, const double *C0, int64_t ldc,
                         double *W) {
    for (int64_t lb = 0; lb < cnt; lb += 4)
        for (int64_t jb = 0; jb < kChunk; jb += 8) {
            double acc[4][8] = {};
            for (int64_t r = 0; r < rows; ++r) {
                const double *cr = C0 + r * ldc + jb;
                const double *vr = V + r * cnt + lb;
                for (int a = 0; a < 4; ++a) {
                    const double f = vr[a];
                    for (int j = 0; j < 8; ++j) acc[a][j] += f * cr[j];
                }
            }
            for (int a = 0; a < 4; ++a)
                for (int j = 0; j < 8; ++j) W[(lb + a) * kChunk + jb + j] = acc[a][j];
        }
}
//   C -= V W2, W2: cnt x kChunk
static void refl_update_tiled(int64_t rows, int64_t cnt, const double *V, const double *W2,
                              double *C0, int64_t ldc) {
    int64_t r = 0;
    for (; r + 4 <= rows; r += 4)
        for (int64_t jb = 0; jb < kChunk; jb += 8) {
            double acc[4][8];
            for (int a = 0; a < 4; ++a)
                for (int j = 0; j < 8; ++j) acc[a][j] = C0[(r + a) * ldc + jb + j];
            for (int64_t l = 0; l < cnt; ++l) {
                const double *w2 = W2 + l * kChunk + jb;
                for (int a = 0; a < 4; ++a) {
                    const double f = V[(r + a) * cnt + l];
                    for (int j = 0; j < 8; ++j) acc[a][j] -= f * w2[j];
                }
            }
            for (int a = 0; a < 4; ++a)
                for (int j = 0; j < 8; ++j) C0[(r + a) * ldc + jb + j] = acc[a][j];
        }
    for (; r < rows; ++r) {
        double *cr = C0 + r * ldc;
        for (int64_t l = 0; l < cnt; ++l) {
            const double f = V[r * cnt + l];
            const double *w2 = W2 + l * kChunk;
            for (int64_t j = 0; j < kChunk; ++j) cr[j] -= f * w2[j];
        }
    }
}

template <class T>
static bool eigh_impl(int64_t p, const T *B, int64_t ldb, double *w, T *U, int64_t ldu) {
    if (p == 0) return true;
    std::vector<T> A((size_t)p * p);
    for (int64_t i = 0; i < p; ++i)
        for (int64_t j = 0; j < p; ++j) A[i * p + j] = B[i * ldb + j];
    for (int64_t i = 0; i < p; ++i) {  // Hermitian part
        A[i * p + i] = T(realv(A[i * p + i]));
        for (int64_t j = i + 1; j < p; ++j) {
            const T h = 0.5 * (A[i * p + j] + conjv(A[j * p + i]));
            A[i * p + j] = h;
            A[j * p + i] = conjv(h);
        }
    }
    // Householder reduction with look-ahead.  Reflector k (unit v_k on indices
    // k+1..p-1, H_k = I - 2 v_k v_k^H) maps column k to (.., alpha_k, 0, ..).  With
    // u_k = A_k v_k (A_k the trailing matrix from k+1), gamma = v_k^H u_k and
    // w_k = 2 u_k - 2 gamma v_k, H_k A_k H_k = A_k - v_k w_k^H - w_k v_k^H.  Per column,
    // every thread forms w_k, applies update k to column k+1 and forms reflector k+1
    // from it, each in its own copy (O(p) work, the same arithmetic everywhere); then
    // the threads sweep the rows once, each row receiving update k and giving its entry
    // of u_{k+1} = A_{k+1} v_{k+1}: one barrier per column and one pass over the trailing
    // matrix.  Only the diagonal of column k+1 is written back (the rest of that column
    // is used by reflector k+1 alone); row k+1 is never read again and is left stale.
    std::vector<std::vector<T>> V(p);
    std::vector<T> vb0(p);
    std::vector<T> ub[2] = {std::vector<T>(p), std::vector<T>(p)};
    // reflector from x[0..m) (the part of a column below the diagonal); false if x = 0
    auto make_reflector = [](int64_t m, const T *x, std::vector<T> &v, T &alpha) -> bool {
        double xn2 = 0.0;
        for (int64_t i = 0; i < m; ++i) xn2 += absq(x[i]);
        const double xn = std::sqrt(xn2);
        const T x0 = x[0];
        alpha = x0;
        if (xn == 0.0) return false;
        const double ax0 = std::sqrt(absq(x0));
        const T phase = ax0 > 0 ? x0 / ax0 : T(1);
        alpha = -phase * xn;
        for (int64_t i = 0; i < m; ++i) v[i] = x[i];
        v[0] -= alpha;
        double vn2 = 0.0;
        for (int64_t i = 0; i < m; ++i) vn2 += absq(v[i]);
        const double inv = 1.0 / std::sqrt(vn2);
        for (int64_t i = 0; i < m; ++i) v[i] *= inv;
        return true;
    };
    std::vector<T> alphas(p, T(0));
    const bool householder_threads =
        p * (int64_t)(sizeof(T) / sizeof(double)) >= kHouseholderParallelMin;
    if (p > 2) {
        std::vector<T> col0(p - 1);
        for (int64_t i = 0; i + 1 < p; ++i) col0[i] = A[(1 + i) * p];
        const bool have0 = make_reflector(p - 1, col0.data(), vb0, alphas[0]);
#pragma omp parallel if (householder_threads)
        {
            const bool lead = omp_get_thread_num() == 0;
            std::vector<T> vp[2] = {vb0, std::vector<T>(p)};  // v_k, v_{k+1} (this thread's)
            std::vector<T> wk(p), wkc(p), col(p);           // w_k, its conjugate, column k+1
            bool have[2] = {have0, false};
            if (have[0]) {
#pragma omp for schedule(static)
                for (int64_t i = 0; i < p - 1; ++i)
                    ub[0][i] = dot_lanes(&A[(1 + i) * p + 1], vp[0].data(), p - 1);
            }
            for (int64_t k = 0; k + 2 < p; ++k) {
                const int cur = (int)(k & 1), nxt = cur ^ 1;
                const std::vector<T> &v = vp[cur];
                const int64_t m = p - k - 1;
                // column k+1 from row k+1 down, with update k applied (index i = row - (k+1))
                for (int64_t i = 0; i < m; ++i) col[i] = A[(k + 1 + i) * p + k + 1];
                if (have[cur]) {
                    const std::vector<T> &u = ub[cur];
                    T gamma = T(0);
                    for (int64_t i = 0; i < m; ++i) gamma += conjv(v[i]) * u[i];
                    const double g = realv(gamma);
                    for (int64_t i = 0; i < m; ++i) {
                        wk[i] = 2.0 * u[i] - 2.0 * g * v[i];
                        wkc[i] = conjv(wk[i]);
                    }
                    const T w0c = wkc[0], v0c = conjv(v[0]);
                    for (int64_t i = 0; i < m; ++i) col[i] -= v[i] * w0c + wk[i] * v0c;
                }
                T alpha_next = T(0);
                have[nxt] = k + 3 < p && make_reflector(m - 1, col.data() + 1, vp[nxt], alpha_next);
                if (lead) {
                    A[(k + 1) * p + k + 1] = col[0];
                    if (have[cur]) V[k].assign(v.begin(), v.begin() + m);
                    A[(k + 1) * p + k] = alphas[k];
                    // alpha_{k+1}: the subdiagonal entry of column k+1 once reflected, written
                    // at the next column; the last column has no reflector and keeps its
                    // updated subdiagonal entry
                    if (k + 3 < p)
                        alphas[k + 1] = alpha_next;
                    else
                        A[(k + 2) * p + k + 1] = col[1];
                }
                // rows k+2..: update k on columns k+2.., then u_{k+1} entries
                const bool upd = have[cur], nx = have[nxt];
                const int64_t m1 = p - k - 2;  // length of v_{k+1}
#pragma omp for schedule(static)
                for (int64_t r = k + 2; r < p; ++r) {
                    T *ar = &A[r * p + k + 2];
                    if (upd) {
                        const T vi = v[r - k - 1], wi = wk[r - k - 1];
                        const T *wcj = &wkc[1];
                        const T *vj = &v[1];
                        for (int64_t j = 0; j < m1; ++j) ar[j] -= vi * wcj[j] + wi * conjv(vj[j]);
                    }
                    if (nx) ub[nxt][r - k - 2] = dot_lanes(ar, vp[nxt].data(), m1);
                }
            }
        }
    }
    // real tridiagonal via phases delta_{k+1} = delta_k e_k / |e_k|
    std::vector<double> d(p), e(p - 1);
    std::vector<T> delta(p, T(1));
    for (int64_t k = 0; k < p; ++k) d[k] = realv(A[k * p + k]);
    for (int64_t k = 0; k + 1 < p; ++k) {
        const T ek = A[(k + 1) * p + k];
        const double ae = std::sqrt(absq(ek));
        e[k] = ae;
        delta[k + 1] = ae > 0 ? delta[k] * (ek / ae) : delta[k];
    }
    // eigenpairs of the tridiagonal: divide and conquer (Zd, eigenvalues ascending), or
    // the QR iteration's recorded rotations where the blocks are small or the secular
    // solver reports trouble
    std::vector<double> Zd;
    bool dc_ok = false;
    if (p > kDcLeaf) {
        std::vector<double> dd(d), ee(e);
        Zd.assign((size_t)p * p, 0.0);
        dc_ok = dc_eig(p, dd.data(), ee.data(), Zd.data(), p);
        if (dc_ok) d = dd;
    }
    std::vector<Rot> rots;
    std::vector<int64_t> order(p);
    std::iota(order.begin(), order.end(), 0);
    if (!dc_ok) {
        rots.reserve((size_t)2 * p * p);
        if (!tridiag_qr(p, d, e, rots)) return false;
        std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return d[a] < d[b]; });
    }
    // C = diag(delta) Z as a row-major p x p matrix.  Z = I J_1^T J_2^T ...: rotation
    // (k, c, s) replaces columns (z_k, z_{k+1}) by (c z_k + s z_{k+1}, -s z_k + c z_{k+1});
    // kept transposed (Zt row k = column k of Z) so each rotation is two row axpys,
    // applied to independent column chunks in parallel.  Then the reflectors
    // H_{p-3}, ..., H_0 act on rows k+1.. of C, again chunk by chunk, kReflBlock at a
    // time in the compact form I - Vb T Vb^H.
    LineMatrix<double> Zt(p, p);
    LineMatrix<T> C(p, p);
    const int64_t nchunks = (p + kChunk - 1) / kChunk;
    const std::vector<ReflBlock<T>> blocks = reflector_blocks(p, V);
#pragma omp parallel if (p >= kParallelMin / 2)
    {
        if (!dc_ok) {
#pragma omp for schedule(dynamic)
            for (int64_t ch = 0; ch < nchunks; ++ch) {
                const int64_t i0 = ch * kChunk, i1 = std::min(p, i0 + kChunk);
                for (int64_t i = i0; i < i1; ++i) Zt.row(i)[i] = 1.0;
                if (i1 - i0 == kChunk)
                    rotate_columns<kChunk>(Zt, rots, i0, kChunk);
                else
                    rotate_columns<0>(Zt, rots, i0, i1 - i0);
            }
            // C[r][jj] = delta[r] * Z[r][order[jj]] = delta[r] * Zt[order[jj]][r]
#pragma omp for schedule(static)
            for (int64_t r = 0; r < p; ++r)
                for (int64_t jj = 0; jj < p; ++jj) C.row(r)[jj] = delta[r] * Zt.row(order[jj])[r];
        } else {
#pragma omp for schedule(static)
            for (int64_t r = 0; r < p; ++r)
                for (int64_t jj = 0; jj < p; ++jj) C.row(r)[jj] = delta[r] * Zd[(size_t)r * p + jj];
        }
#pragma omp for schedule(dynamic)
        for (int64_t ch = 0; ch < nchunks; ++ch) {
            const int64_t j0 = ch * kChunk, j1 = std::min(p, j0 + kChunk), nc = j1 - j0;
            std::vector<T> W((size_t)kReflBlock * kChunk), W2((size_t)kReflBlock * kChunk);
            for (int64_t b = (int64_t)blocks.size() - 1; b >= 0; --b) {
                const ReflBlock<T> &rb = blocks[b];
                const int64_t cnt = rb.cnt, r0 = rb.k0 + 1;
                const bool tiled = std::is_same<T, double>::value && nc == kChunk && cnt % 4 == 0;
                // W = Vb^H C[r0.., chunk]
                if constexpr (std::is_same<T, double>::value) {
                    if (tiled) refl_w_tiled(p - r0, cnt, rb.V.data(), C.row(r0) + j0, C.ld, W.data());
                }
                if (!tiled) std::fill(W.begin(), W.begin() + cnt * nc, T(0));
                for (int64_t r = tiled ? p : r0; r < p; ++r) {
                    const T *cr = C.row(r) + j0;
                    const T *vr = &rb.V[(size_t)(r - r0) * cnt];
                    for (int64_t l = 0; l < cnt; ++l) {
                        const T f = conjv(vr[l]);
                        T *wl = &W[(size_t)l * nc];
                        for (int64_t j = 0; j < nc; ++j) wl[j] += f * cr[j];
                    }
                }
                // W2 = T W (T upper triangular)
                for (int64_t l = 0; l < cnt; ++l) {
                    T *w2 = &W2[(size_t)l * nc];
                    std::fill(w2, w2 + nc, T(0));
                    for (int64_t m = l; m < cnt; ++m) {
                        const T t = rb.Tm[(size_t)l * cnt + m];
                        const T *wm = &W[(size_t)m * nc];
                        for (int64_t j = 0; j < nc; ++j) w2[j] += t * wm[j];
                    }
                }
                // C -= Vb W2
                if constexpr (std::is_same<T, double>::value) {
                    if (tiled) refl_update_tiled(p - r0, cnt, rb.V.data(), W2.data(), C.row(r0) + j0, C.ld);
                }
                for (int64_t r = tiled ? p : r0; r < p; ++r) {
                    T *cr = C.row(r) + j0;
                    const T *vr = &rb.V[(size_t)(r - r0) * cnt];
                    for (int64_t l = 0; l < cnt; ++l) {
                        const T f = vr[l];
                        const T *w2 = &W2[(size_t)l * nc];
                        for (int64_t j = 0; j < nc; ++j) cr[j] -= f * w2[j];
                    }
                }
            }
        }
    }
    for (int64_t r = 0; r < p; ++r)
        for (int64_t jj = 0; jj < p; ++jj) U[r * ldu + jj] = C.row(r)[jj];
    for (int64_t jj = 0; jj < p; ++jj) w[jj] = d[order[jj]];
    return true;
}

bool host_eigh(int64_t p, bool cplx, const double *B, int64_t ldb, double *w, double *U,
               int64_t ldu) {
    if (cplx)
        return eigh_impl<cd>(p, reinterpret_cast<const cd *>(B), ldb, w, reinterpret_cast<cd *>(U), ldu);
    return eigh_impl<double>(p, B, ldb, w, U, ldu);
}

}  // namespace AFSI_ISA_NS
}  // namespace afsi
