// C ABI of the library: argument checking, resource management and the host side
// of each call.  The arithmetic of the hot path runs in the HIP kernels
// (clenshaw_*.hip, dense.hip, util.hip); small p x p factorisations run on the host
// (host_linalg.cpp).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <utility>
#include <vector>

#include "internal.h"

namespace afsi {

// ---------------------------------------------------------------- errors

static thread_local std::string g_error = "no error";

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
}

// ---------------------------------------------------------------- device / scratch

DeviceGuard::DeviceGuard(int dev) {
    AFSI_HIP(hipGetDevice(&prev));
    if (prev != dev) AFSI_HIP(hipSetDevice(dev));
    else prev = -1;
}
DeviceGuard::~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
}

void *Workspace::dev_reserve(int slot, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (bytes > dev_bytes[slot]) {
        // grow by at least half, so that slowly increasing requests reallocate rarely
        const size_t want = std::max(bytes, dev_bytes[slot] + dev_bytes[slot] / 2);
        if (dev[slot]) {
            AFSI_HIP(hipStreamSynchronize(stream));
            AFSI_HIP(hipFree(dev[slot]));
            dev[slot] = nullptr;
            dev_bytes[slot] = 0;
        }
        AFSI_HIP(hipMalloc(&dev[slot], want));
        dev_bytes[slot] = want;
    }
    return dev[slot];
}

void *Workspace::host_reserve(int slot, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (bytes > host_bytes[slot]) {
        if (host[slot]) {
            AFSI_HIP(hipStreamSynchronize(stream));
            AFSI_HIP(hipHostFree(host[slot]));
            host[slot] = nullptr;
            host_bytes[slot] = 0;
        }
        AFSI_HIP(hipHostMalloc(&host[slot], bytes, hipHostMallocDefault));
        host_bytes[slot] = bytes;
    }
    return host[slot];
}

static std::mutex g_ws_mu;
static std::map<std::pair<int, hipStream_t>, std::unique_ptr<Workspace>> g_ws;

Workspace &workspace(hipStream_t stream) {
    int dev = 0;
    AFSI_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto &slot = g_ws[{dev, stream}];
    if (!slot) {
        slot.reset(new Workspace());
        slot->stream = stream;
    }
    return *slot;
}

// ---------------------------------------------------------------- matrix access

MatView matrix_view(afsi_matrix_t A, int block_dtype, hipStream_t stream) {
    const bool want_complex = is_complex(block_dtype);
    AFSI_REQUIRE(want_complex == (A->dtype == AFSI_C128),
                 "block dtype %d does not match the matrix (%s)", block_dtype,
                 A->dtype == AFSI_C128 ? "complex" : "real");
    MatView v{A->n, A->d_rp, A->d_ci, A->d_val64};
    v.stage_near = 2 * A->near_nnz >= A->n;
    v.seg_bytes = A->seg_bytes;
    v.band = A->band;
    if (!is_fp64(block_dtype)) {
        std::lock_guard<std::mutex> lk(A->mu);
        if (!A->d_val32) {
            const int64_t count = A->nnz * (want_complex ? 2 : 1);
            AFSI_HIP(hipMalloc(&A->d_val32, std::max<int64_t>(count, 1) * sizeof(float)));
            launch_to_f32((const double *)A->d_val64, (float *)A->d_val32, count, stream);
            AFSI_HIP(hipStreamSynchronize(stream));
        }
        v.val = A->d_val32;
    }
    return v;
}

// ---------------------------------------------------------------- block checks

static hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

static void check_block(const afsi_block *b, const char *name) {
    AFSI_REQUIRE(b != nullptr, "%s is NULL", name);
    AFSI_REQUIRE(b->dtype >= AFSI_R64 && b->dtype <= AFSI_C64, "%s has unknown dtype %d", name,
                 b->dtype);
    AFSI_REQUIRE(b->rows >= 0 && b->cols >= 0, "%s has negative shape", name);
    AFSI_REQUIRE(b->ld >= b->cols && b->ld >= 1, "%s: ld (%lld) < cols (%lld)", name,
                 (long long)b->ld, (long long)b->cols);
    AFSI_REQUIRE(b->ptr != nullptr || b->rows * b->cols == 0, "%s has a NULL pointer", name);
}

static void check_fp64(const afsi_block *b, const char *name) {
    AFSI_REQUIRE(is_fp64(b->dtype), "%s must be R64 or C128 (got dtype %d)", name, b->dtype);
}

static std::pair<uintptr_t, uintptr_t> span(const afsi_block *b) {
    const uintptr_t p = (uintptr_t)b->ptr;
    if (b->rows * b->cols == 0) return {p, p};
    return {p, p + (uintptr_t)(((b->rows - 1) * b->ld + b->cols) * elem_bytes(b->dtype))};
}

static bool overlap(const afsi_block *a, const afsi_block *b) {
    auto x = span(a), y = span(b);
    return x.first < y.second && y.first < x.second;
}

static void check_same_shape(const afsi_block *a, const afsi_block *b, const char *na,
                             const char *nb) {
    AFSI_REQUIRE(a->rows == b->rows && a->cols == b->cols && a->ld == b->ld && a->dtype == b->dtype,
                 "%s and %s must have the same shape, leading dimension and dtype", na, nb);
}

// ---------------------------------------------------------------- Clenshaw step launch

static bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// One product over column blocks of seg bytes (Section 3.3.1's MaSpMM loop over column
// blocks of the dense operand): the blocks are the "slices" of one grouped launch (up
// to kGroupedMax per launch), so the whole matrix passes over block 0's columns, then
// block 1's, ..., and a block's gathered source rows can stay cached while every row
// reuses them.  Per column the arithmetic is the single kernel's.  Returns false
// (nothing launched) when blocking does not apply.  Off unless the caller sets a width:
// on the n = 2e6 matrix with uniform random columns (p = 640 FP32) 64/128/256/512-byte
// blocks took 32.5/16.7/15.3/15.9 ms per product against 16.4 ms unblocked (FP64
// 63.6/38.7/36.8/35.7 against 32.8 ms), and the 100^3 stencil 2.19 against 1.61 ms at
// 256 bytes: A is re-read per block and 64-byte random gathers use the memory system
// poorly.
static bool column_blocked_step(const MatView &mv, int dtype, const void *src, const void *X,
                                void *dst, int64_t p, int64_t ld, bool hv, bool hx, double sg,
                                double ta, double al, hipStream_t s) {
    const int eb = elem_bytes(dtype);
    const int64_t seg = mv.seg_bytes;
    if (seg <= 0 || seg % 16 || p * eb <= seg || (p * eb) % seg || (ld * eb) % 16 ||
        !aligned16(src) || !aligned16(dst) || (hx && !aligned16(X)))
        return false;
    const int p16 = (int)(seg / 16);
    if (grouped_width_at_least(p16) != p16) return false;
    const int64_t nseg = p * eb / seg, segel = seg / eb;
    for (int64_t g0 = 0; g0 < nseg; g0 += kGroupedMax) {
        GroupArgs args;
        std::memset(&args, 0, sizeof args);
        const int cnt = (int)std::min<int64_t>(kGroupedMax, nseg - g0);
        for (int k = 0; k < cnt; ++k) {
            const int64_t c0 = (g0 + k) * segel * eb;
            args.P0[k] = (char *)const_cast<void *>(src) + c0;
            args.P1[k] = (char *)dst + c0;
            args.X[k] = hx ? (const char *)X + c0 : args.P0[k];
            args.ldv[k] = ld * eb / 16;
            args.src[k] = 1;
            args.dst[k] = 2;
            args.has_v[k] = hv;
            args.sigma[k] = sg;
            args.tau[k] = ta;
            args.alpha[k] = hx ? al : 0.0;
        }
        args.ngroups = cnt;
        bool done = false;
        switch (dtype) {
        case AFSI_R64: done = clenshaw_r64_grouped(mv, p16, args, s); break;
        case AFSI_R32: done = clenshaw_r32_grouped(mv, p16, args, s); break;
        case AFSI_C128: done = clenshaw_c128_grouped(mv, p16, args, s); break;
        case AFSI_C64: done = clenshaw_c64_grouped(mv, p16, args, s); break;
        }
        AFSI_REQUIRE(done, "column-blocked step: no lane mapping for %d vectors", p16);
    }
    return true;
}

static void run_step(const MatView &mv, int dtype, const void *src, const void *X, void *dst,
                     int64_t p, int64_t ld, bool hv, bool hx, double sg, double ta, double al,
                     hipStream_t s) {
    if (mv.n == 0 || p == 0) return;
    AFSI_REQUIRE(p < (1LL << 31) && ld < (1LL << 40), "block too wide");
    if (column_blocked_step(mv, dtype, src, X, dst, p, ld, hv, hx, sg, ta, al, s)) {
        AFSI_HIP(hipGetLastError());
        return;
    }
    const int eb = elem_bytes(dtype);
    // narrow rows (fewer than 16 vectors, no exact lane mapping): one lane per row
    const bool narrow = p <= kNarrowMax && p * eb < 16 * 16;
    const bool vec = !narrow && (p * eb) % 16 == 0 && (ld * eb) % 16 == 0 && aligned16(src) &&
                     aligned16(dst) && (!hx || aligned16(X));
    if (vec) {
        const int p16 = (int)(p * eb / 16);
        const int64_t ldv = ld * eb / 16;
        switch (dtype) {
        case AFSI_R64: clenshaw_r64_step(mv, src, X, dst, p16, ldv, hv, hx, sg, ta, al, s); break;
        case AFSI_R32: clenshaw_r32_step(mv, src, X, dst, p16, ldv, hv, hx, sg, ta, al, s); break;
        case AFSI_C128: clenshaw_c128_step(mv, src, X, dst, p16, ldv, hv, hx, sg, ta, al, s); break;
        case AFSI_C64: clenshaw_c64_step(mv, src, X, dst, p16, ldv, hv, hx, sg, ta, al, s); break;
        }
    } else {
        const int pi = (int)p;
        switch (dtype) {
        case AFSI_R64: clenshaw_r64_scalar(mv, src, X, dst, pi, ld, hv, hx, sg, ta, al, s); break;
        case AFSI_R32: clenshaw_r32_scalar(mv, src, X, dst, pi, ld, hv, hx, sg, ta, al, s); break;
        case AFSI_C128: clenshaw_c128_scalar(mv, src, X, dst, pi, ld, hv, hx, sg, ta, al, s); break;
        case AFSI_C64: clenshaw_c64_scalar(mv, src, X, dst, pi, ld, hv, hx, sg, ta, al, s); break;
        }
    }
    AFSI_HIP(hipGetLastError());
}

static void map_coeffs(const afsi_matrix_s *A, double &l1, double &l2) {
    AFSI_REQUIRE(A->has_bounds, "spectral bounds are not set on this matrix");
    const double w = A->lmax - A->lmin;
    l1 = 2.0 / w;
    l2 = -(A->lmax + A->lmin) / w;
}

static void check_matrix(afsi_matrix_t A) { AFSI_REQUIRE(A != nullptr, "matrix handle is NULL"); }

// Filter on raw pointers (shared by afsi_filter_block and the solver).  When
// `events` is given (degree + 1 events), one is recorded before every product
// and one after the last; `kind[s]` gets has_v | has_x << 1 of product s.
void filter_apply(afsi_matrix_t A, const double *coeffs, int degree, int dtype, const void *X,
                  void *Y, void *work, int64_t p, int64_t ld, hipStream_t s, hipEvent_t *events,
                  int32_t *kind) {
    double l1, l2;
    map_coeffs(A, l1, l2);
    AFSI_REQUIRE(degree >= 1, "degree must be >= 1 (got %d)", degree);
    const MatView mv = matrix_view(A, dtype, s);
    void *P[3] = {const_cast<void *>(X), nullptr, nullptr};
    P[1 + (degree - 1) % 2] = Y;
    P[1 + degree % 2] = work;
    for (int st = 0; st < degree; ++st) {
        afsi_step_group g;
        step_params(coeffs, degree, st, l1, l2, &g);
        if (events) AFSI_HIP(hipEventRecord(events[st], s));
        if (kind) kind[st] = (g.has_v ? 1 : 0) | (g.alpha != 0.0 ? 2 : 0);
        run_step(mv, dtype, P[g.src], X, P[g.dst], p, ld, g.has_v != 0, g.alpha != 0.0, g.sigma,
                 g.tau, g.alpha, s);
    }
    if (events) AFSI_HIP(hipEventRecord(events[degree], s));
}

void spmm_apply(afsi_matrix_t A, int dtype, const void *X, void *Y, int64_t p, int64_t ld,
                hipStream_t s) {
    const MatView mv = matrix_view(A, dtype, s);
    run_step(mv, dtype, X, nullptr, Y, p, ld, false, false, 1.0, 0.0, 0.0, s);
}

// ---------------------------------------------------------------- dense helpers

void inner_dev(int dtype, const void *X, int64_t ldx, const void *Y, int64_t ldy, int64_t n,
               int64_t p, int64_t q, double *G, int64_t ldg, hipStream_t s) {
    if (dtype == AFSI_C128)
        gram_c128((const double *)X, ldx, (const double *)Y, ldy, n, p, q, G, ldg, s);
    else
        gram_f64((const double *)X, ldx, (const double *)Y, ldy, n, p, q, G, ldg, s);
}

void gemm_dev(int dtype, const void *X, int64_t ldx, const double *M, int64_t ldm, int64_t n,
              int64_t p, int64_t q, double alpha, double beta, void *Y, int64_t ldy,
              hipStream_t s, bool upper) {
    if (dtype == AFSI_C128)
        gemm_c128((const double *)X, ldx, M, ldm, n, p, q, alpha, beta, (double *)Y, ldy, s, upper);
    else
        gemm_f64((const double *)X, ldx, M, ldm, n, p, q, alpha, beta, (double *)Y, ldy, s, upper);
}

// X <- X - L (L^H X), twice.  L: n x k (ld ldl), X: n x p (ld ldx).
void project_out_dev(int dtype, const void *L, int64_t ldl, int64_t k, void *X, int64_t ldx,
                     int64_t n, int64_t p, hipStream_t s) {
    if (k == 0 || p == 0) return;
    const int comp = dtype == AFSI_C128 ? 2 : 1;
    double *C = (double *)workspace(s).dev_reserve(SLOT_SMALL, sizeof(double) * comp * k * p);
    for (int pass = 0; pass < 2; ++pass) {
        inner_dev(dtype, L, ldl, X, ldx, n, k, p, C, p, s);
        gemm_dev(dtype, L, ldl, C, p, n, k, p, -1.0, 1.0, X, ldx, s);
    }
}

// CholQR2 with shifted CholQR3 fallback.  X and W: n x p, same ld.
// max_col_norm2 (optional): largest squared column norm of X on entry.
// Without rinv the result is in X (returned).  With rinv (host, comp p^2 doubles) the
// last pass's product is not formed: Q = Y R^{-1} with Y the returned block (X or W)
// and R^{-1} (upper triangular, row-major) in rinv.
static void *cholqr_passes(int dtype, void *X, void *W, int64_t n, int64_t p, int64_t ld,
                           hipStream_t s, double *max_col_norm2, double *rinv) {
    const bool cplx = dtype == AFSI_C128;
    const int comp = cplx ? 2 : 1;
    const size_t gbytes = sizeof(double) * comp * p * p;
    Workspace &ws = workspace(s);
    double *G = (double *)ws.dev_reserve(SLOT_SMALL, gbytes);
    double *Gh = (double *)ws.host_reserve(0, gbytes);
    void *cur = X, *oth = W;
    const double u = std::numeric_limits<double>::epsilon() / 2;
    int plain_passes = 0, shifted = 0;
    while (plain_passes < 2) {
        inner_dev(dtype, cur, ld, cur, ld, n, p, p, G, p, s);
        AFSI_HIP(hipMemcpyAsync(Gh, G, gbytes, hipMemcpyDeviceToHost, s));
        AFSI_HIP(hipStreamSynchronize(s));
        if (max_col_norm2 && cur == X && plain_passes == 0 && shifted == 0) {
            double mx = 0.0;
            for (int64_t i = 0; i < p; ++i) mx = std::max(mx, Gh[comp * (i * p + i)]);
            *max_col_norm2 = mx;
        }
        // host_cholesky_inverse leaves Gh untouched when it reports a breakdown
        if (host_cholesky_inverse(p, cplx, Gh, p, 0.0)) {
            if (++plain_passes == 2 && rinv) {
                std::memcpy(rinv, Gh, gbytes);
                return cur;
            }
        } else {
            // shifted Cholesky QR (Fukaya et al. 2020): s = 11 (n p + p (p+1)) u ||X||_F^2,
            // followed by two plain passes
            if (shifted >= 2) AFSI_FAIL(AFSI_E_NOT_HPD, "Cholesky QR broke down even with a shift");
            double fro2 = 0.0;
            for (int64_t i = 0; i < p; ++i) fro2 += Gh[comp * (i * p + i)];
            const double shift = 11.0 * ((double)n * p + (double)p * (p + 1)) * u * fro2;
            if (!host_cholesky_inverse(p, cplx, Gh, p, shift))
                AFSI_FAIL(AFSI_E_NOT_HPD, "Cholesky QR broke down even with a shift");
            ++shifted;
            plain_passes = 0;
        }
        AFSI_HIP(hipMemcpyAsync(G, Gh, gbytes, hipMemcpyHostToDevice, s));
        gemm_dev(dtype, cur, ld, G, p, n, p, p, 1.0, 0.0, oth, ld, s, true);  // X R^{-1}
        std::swap(cur, oth);
    }
    if (cur != X) {
        const int eb = elem_bytes(dtype);
        AFSI_HIP(hipMemcpy2DAsync(X, ld * eb, cur, ld * eb, p * eb, n, hipMemcpyDeviceToDevice, s));
    }
    AFSI_HIP(hipStreamSynchronize(s));
    return X;
}

void orthonormalize_dev(int dtype, void *X, void *W, int64_t n, int64_t p, int64_t ld,
                        hipStream_t s, double *max_col_norm2) {
    if (p == 0) return;
    cholqr_passes(dtype, X, W, n, p, ld, s, max_col_norm2, nullptr);
}

// CholQR2 of X fused with Rayleigh-Ritz on its basis Q, which is never formed: with the
// last pass's input Y and factor R, Q = Y R^{-1}, so Q^H A Q = R^{-H} (Y^H A Y) R^{-1} and
// V = Q U = Y (R^{-1} U): one n x p x p block product fewer than orthonormalising first.
// The p x p products run on the device: T = (Y^H A Y) R^{-1}, then T^H R^{-1} (equal to
// R^{-H} (Y^H A Y) R^{-1} since Y^H A Y is Hermitian), and R^{-1} U.  V must differ from
// X and W; AV may be W.  orth_ms (optional): host time until the Cholesky-QR part is done.
void orthonormalize_rr_dev(afsi_matrix_t A, int dtype, void *X, void *W, void *V, void *AV,
                           int64_t n, int64_t p, int64_t ld, double *ritz, hipStream_t s,
                           double *max_col_norm2, double *orth_ms) {
    if (p == 0) return;
    const auto t0 = std::chrono::steady_clock::now();
    const bool cplx = dtype == AFSI_C128;
    const int comp = cplx ? 2 : 1;
    const size_t mel = (size_t)comp * p * p, mbytes = sizeof(double) * mel;
    std::vector<double> rinv(mel), U(mel);
    void *Y = cholqr_passes(dtype, X, W, n, p, ld, s, max_col_norm2, rinv.data());
    if (orth_ms)
        *orth_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    Workspace &ws = workspace(s);
    double *Bd = (double *)ws.dev_reserve(SLOT_SMALL, 3 * mbytes);
    double *Rd = Bd + mel, *Td = Rd + mel;
    double *Hh = (double *)ws.host_reserve(0, mbytes);
    AFSI_HIP(hipMemcpyAsync(Rd, rinv.data(), mbytes, hipMemcpyHostToDevice, s));
    spmm_apply(A, dtype, Y, V, p, ld, s);                               // V <- A Y
    inner_dev(dtype, Y, ld, V, ld, n, p, p, Bd, p, s);                  // Y^H A Y
    gemm_dev(dtype, Bd, p, Rd, p, p, p, p, 1.0, 0.0, Td, p, s, true);   // T = (Y^H A Y) R^{-1}
    inner_dev(dtype, Td, p, Rd, p, p, p, p, Bd, p, s);                  // Q^H A Q = T^H R^{-1}
    AFSI_HIP(hipMemcpyAsync(Hh, Bd, mbytes, hipMemcpyDeviceToHost, s));
    AFSI_HIP(hipStreamSynchronize(s));
    host_eigh_or_throw(p, cplx, Hh, p, ritz, U.data(), p);
    AFSI_HIP(hipMemcpyAsync(Td, U.data(), mbytes, hipMemcpyHostToDevice, s));
    gemm_dev(dtype, Rd, p, Td, p, p, p, p, 1.0, 0.0, Bd, p, s);         // R^{-1} U
    gemm_dev(dtype, Y, ld, Bd, p, n, p, p, 1.0, 0.0, V, ld, s);         // V  <- Q U
    spmm_apply(A, dtype, V, AV, p, ld, s);                              // AV <- A V
    AFSI_HIP(hipStreamSynchronize(s));
}

// Rayleigh-Ritz on raw pointers.  Q, V, AV: n x p with leading dimension ld.
void rayleigh_ritz_dev(afsi_matrix_t A, int dtype, const void *Q, void *V, void *AV, int64_t n,
                       int64_t p, int64_t ld, double *ritz, hipStream_t s) {
    if (p == 0) return;
    const bool cplx = dtype == AFSI_C128;
    const int comp = cplx ? 2 : 1;
    const size_t mbytes = sizeof(double) * comp * p * p;
    Workspace &ws = workspace(s);
    double *B = (double *)ws.dev_reserve(SLOT_SMALL, mbytes);
    double *Bh = (double *)ws.host_reserve(0, 2 * mbytes);
    double *Uh = Bh + comp * p * p;
    spmm_apply(A, dtype, Q, V, p, ld, s);                  // V <- A Q
    inner_dev(dtype, Q, ld, V, ld, n, p, p, B, p, s);      // B <- Q^H A Q
    AFSI_HIP(hipMemcpyAsync(Bh, B, mbytes, hipMemcpyDeviceToHost, s));
    AFSI_HIP(hipStreamSynchronize(s));
    host_eigh_or_throw(p, cplx, Bh, p, ritz, Uh, p);
    AFSI_HIP(hipMemcpyAsync(B, Uh, mbytes, hipMemcpyHostToDevice, s));
    gemm_dev(dtype, Q, ld, B, p, n, p, p, 1.0, 0.0, V, ld, s);   // V  <- Q U
    spmm_apply(A, dtype, V, AV, p, ld, s);                        // AV <- A V
    AFSI_HIP(hipStreamSynchronize(s));
}

void residual_norms_host(int dtype, const void *V, int64_t ldv, const void *AV, int64_t ldav,
                         const double *lambda, int64_t n, int64_t q, double *out, hipStream_t s) {
    if (q == 0) return;
    Workspace &ws = workspace(s);
    double *d = (double *)ws.dev_reserve(SLOT_VEC, sizeof(double) * 2 * q);
    double *h = (double *)ws.host_reserve(1, sizeof(double) * q);
    std::memcpy(h, lambda, sizeof(double) * q);
    AFSI_HIP(hipMemcpyAsync(d, h, sizeof(double) * q, hipMemcpyHostToDevice, s));
    residual_norms_dev(dtype, V, ldv, AV, ldav, d, n, q, d + q, s);
    AFSI_HIP(hipMemcpyAsync(h, d + q, sizeof(double) * q, hipMemcpyDeviceToHost, s));
    AFSI_HIP(hipStreamSynchronize(s));
    std::memcpy(out, h, sizeof(double) * q);
}

// Spurious-value and locking test (shared by afsi_lock_select and the solver).
void lock_select(const double *ritz, int64_t p, const double *res, uint8_t *I, double a, double b,
                 double tau_abs, int64_t n_lock, int64_t *n_check_prev, uint8_t *lock, int *done) {
    double tau_s = INFINITY;
    int64_t e = 0;
    for (int64_t j = 0; j < p; ++j)
        if (I[j]) {
            tau_s = std::min(tau_s, std::min(std::fabs(ritz[j] - a), std::fabs(ritz[j] - b)));
            ++e;
        }
    AFSI_REQUIRE(e > 0, "no Ritz value inside the interval");
    int64_t nc = 0;
    for (int64_t j = 0; j < p; ++j)
        if (I[j] && res[j] < tau_s) ++nc;
    const int64_t n_check = nc + n_lock;
    if (n_check > 0 && n_check == *n_check_prev)
        for (int64_t j = 0; j < p; ++j) I[j] = (I[j] && res[j] < tau_s) ? 1 : 0;
    *n_check_prev = n_check;
    int left = 0;
    for (int64_t j = 0; j < p; ++j) {
        lock[j] = (I[j] && res[j] < tau_abs) ? 1 : 0;
        if (I[j] && !lock[j]) left = 1;
    }
    *done = left ? 0 : 1;
}

}  // namespace afsi

using namespace afsi;

// ====================================================================== C ABI

extern "C" {

const char *afsi_last_error(void) { return g_error.c_str(); }

const char *afsi_version(void) { return "afsi 0.1 (gfx950)"; }

int afsi_device_count(void) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) {
        set_error("hipGetDeviceCount failed");
        return AFSI_E_NODEVICE;
    }
    int count = 0;
    for (int d = 0; d < n; ++d) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, d) == hipSuccess &&
            std::strncmp(prop.gcnArchName, "gfx950", 6) == 0)
            ++count;
    }
    return count;
}

int afsi_matrix_create_csr(int device, int64_t n, int64_t nnz, const int64_t *row_ptr,
                           const int32_t *col_idx, const void *vals, int32_t val_dtype,
                           afsi_matrix_t *out) {
    return guarded([&] {
        AFSI_REQUIRE(out != nullptr, "out is NULL");
        *out = nullptr;
        AFSI_REQUIRE(n >= 0 && nnz >= 0, "negative size");
        AFSI_REQUIRE(n < (1LL << 31) && nnz < (1LL << 31), "n and nnz must be below 2^31");
        AFSI_REQUIRE(val_dtype == AFSI_R64 || val_dtype == AFSI_C128,
                     "values must be R64 or C128 (got %d)", val_dtype);
        AFSI_REQUIRE(row_ptr != nullptr, "row_ptr is NULL");
        AFSI_REQUIRE(nnz == 0 || (col_idx && vals), "col_idx / vals are NULL");
        AFSI_REQUIRE(row_ptr[0] == 0 && row_ptr[n] == nnz, "row_ptr must start at 0 and end at nnz");
        std::vector<int> rp32(n + 1);
        std::vector<int64_t> reach(n);
        int64_t near_nnz = 0;
        for (int64_t i = 0; i < n; ++i) {
            AFSI_REQUIRE(row_ptr[i + 1] >= row_ptr[i], "row_ptr decreases at row %lld", (long long)i);
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                AFSI_REQUIRE(col_idx[e] >= 0 && col_idx[e] < n, "column %d out of range in row %lld",
                             col_idx[e], (long long)i);
                AFSI_REQUIRE(e == row_ptr[i] || col_idx[e] > col_idx[e - 1],
                             "columns not strictly increasing in row %lld", (long long)i);
                near_nnz += col_idx[e] >= i - 1 && col_idx[e] <= i + 1;
            }
            reach[i] = row_ptr[i + 1] > row_ptr[i]
                           ? std::max<int64_t>(i - col_idx[row_ptr[i]], col_idx[row_ptr[i + 1] - 1] - i)
                           : 0;
            rp32[i] = (int)row_ptr[i];
        }
        rp32[n] = (int)nnz;
        DeviceGuard dg(device);
        std::unique_ptr<afsi_matrix_s> A(new afsi_matrix_s());
        A->device = device;
        A->n = n;
        A->nnz = nnz;
        A->near_nnz = near_nnz;
        if (n > 0) {
            std::nth_element(reach.begin(), reach.begin() + n / 2, reach.end());
            A->band = std::max<int64_t>(0, reach[n / 2]);
        }
        A->dtype = val_dtype;
        const size_t vbytes = (size_t)nnz * elem_bytes(val_dtype);
        try {
            AFSI_HIP(hipMalloc(&A->d_rp, sizeof(int) * (n + 1)));
            AFSI_HIP(hipMalloc(&A->d_ci, sizeof(int) * std::max<int64_t>(nnz, 1)));
            AFSI_HIP(hipMalloc(&A->d_val64, std::max<size_t>(vbytes, 16)));
            AFSI_HIP(hipMemcpy(A->d_rp, rp32.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice));
            if (nnz) {
                AFSI_HIP(hipMemcpy(A->d_ci, col_idx, sizeof(int) * nnz, hipMemcpyHostToDevice));
                AFSI_HIP(hipMemcpy(A->d_val64, vals, vbytes, hipMemcpyHostToDevice));
            }
        } catch (...) {
            (void)hipFree(A->d_rp);
            (void)hipFree(A->d_ci);
            (void)hipFree(A->d_val64);
            throw;
        }
        *out = A.release();
    });
}

int afsi_matrix_set_column_block(afsi_matrix_t A, int64_t bytes) {
    return guarded([&] {
        check_matrix(A);
        AFSI_REQUIRE(bytes >= 0 && bytes % 16 == 0, "column block must be a multiple of 16 bytes");
        AFSI_REQUIRE(bytes == 0 || grouped_width_at_least(bytes / 16) == bytes / 16,
                     "no lane mapping for %lld-byte column blocks", (long long)bytes);
        A->seg_bytes = bytes;
    });
}

int afsi_matrix_get_column_block(afsi_matrix_t A, int64_t *bytes) {
    return guarded([&] {
        check_matrix(A);
        AFSI_REQUIRE(bytes != nullptr, "bytes is NULL");
        *bytes = A->seg_bytes;
    });
}

int afsi_matrix_destroy(afsi_matrix_t A) {
    return guarded([&] {
        if (!A) return;
        DeviceGuard dg(A->device);
        AFSI_HIP(hipDeviceSynchronize());
        (void)hipFree(A->d_rp);
        (void)hipFree(A->d_ci);
        (void)hipFree(A->d_val64);
        if (A->d_val32) (void)hipFree(A->d_val32);
        delete A;
    });
}

int afsi_matrix_info(afsi_matrix_t A, int64_t *n, int64_t *nnz, int32_t *dtype, int32_t *device) {
    return guarded([&] {
        check_matrix(A);
        if (n) *n = A->n;
        if (nnz) *nnz = A->nnz;
        if (dtype) *dtype = A->dtype;
        if (device) *device = A->device;
    });
}

int afsi_set_spectral_bounds(afsi_matrix_t A, double lmin, double lmax) {
    return guarded([&] {
        check_matrix(A);
        AFSI_REQUIRE(std::isfinite(lmin) && std::isfinite(lmax) && lmin < lmax,
                     "bounds need finite lmin < lmax (got %g, %g)", lmin, lmax);
        A->lmin = lmin;
        A->lmax = lmax;
        A->has_bounds = true;
    });
}

int afsi_get_spectral_bounds(afsi_matrix_t A, double *lmin, double *lmax) {
    return guarded([&] {
        check_matrix(A);
        AFSI_REQUIRE(A->has_bounds, "spectral bounds are not set");
        if (lmin) *lmin = A->lmin;
        if (lmax) *lmax = A->lmax;
    });
}

int afsi_filter_coefficients(double lmin, double lmax, double a, double b, int kmax,
                             int32_t damping, double m_exp, double *coeffs) {
    return guarded([&] {
        AFSI_REQUIRE(coeffs != nullptr, "coeffs is NULL");
        filter_coefficients(lmin, lmax, a, b, kmax, damping, m_exp, coeffs);
    });
}

int afsi_filter_block(afsi_matrix_t A, const double *coeffs, int degree, const afsi_block *X,
                      afsi_block *Y, afsi_block *work, void *stream) {
    return guarded([&] {
        check_matrix(A);
        AFSI_REQUIRE(coeffs != nullptr, "coeffs is NULL");
        check_block(X, "X");
        check_block(Y, "Y");
        check_block(work, "work");
        check_same_shape(X, Y, "X", "Y");
        check_same_shape(X, work, "X", "work");
        AFSI_REQUIRE(X->rows == A->n, "X has %lld rows, A has %lld", (long long)X->rows,
                     (long long)A->n);
        AFSI_REQUIRE(!overlap(X, Y) && !overlap(X, work) && !overlap(Y, work),
                     "X, Y and work must not overlap");
        DeviceGuard dg(A->device);
        filter_apply(A, coeffs, degree, X->dtype, X->ptr, Y->ptr, work->ptr, X->cols, X->ld,
                     as_stream(stream));
    });
}

int afsi_filter_block_profiled(afsi_matrix_t A, const double *coeffs, int degree,
                               const afsi_block *X, afsi_block *Y, afsi_block *work, void *stream,
                               float *step_ms, int32_t *step_kind) {
    std::vector<hipEvent_t> ev;
    const int status = guarded([&] {
        check_matrix(A);
        AFSI_REQUIRE(coeffs != nullptr && step_ms != nullptr, "NULL argument");
        check_block(X, "X");
        check_block(Y, "Y");
        check_block(work, "work");
        check_same_shape(X, Y, "X", "Y");
        check_same_shape(X, work, "X", "work");
        AFSI_REQUIRE(X->rows == A->n, "X rows != n");
        AFSI_REQUIRE(!overlap(X, Y) && !overlap(X, work) && !overlap(Y, work),
                     "X, Y and work must not overlap");
        AFSI_REQUIRE(degree >= 1, "degree must be >= 1");
        DeviceGuard dg(A->device);
        hipStream_t s = as_stream(stream);
        ev.resize(degree + 1, nullptr);
        for (auto &e : ev) AFSI_HIP(hipEventCreate(&e));
        std::vector<int32_t> kind(degree);
        filter_apply(A, coeffs, degree, X->dtype, X->ptr, Y->ptr, work->ptr, X->cols, X->ld, s,
                     ev.data(), kind.data());
        AFSI_HIP(hipEventSynchronize(ev[degree]));
        for (int i = 0; i < degree; ++i) {
            AFSI_HIP(hipEventElapsedTime(&step_ms[i], ev[i], ev[i + 1]));
            if (step_kind) step_kind[i] = kind[i];
        }
    });
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    return status;
}

int afsi_spmm(afsi_matrix_t A, const afsi_block *X, afsi_block *Y, void *stream) {
    return guarded([&] {
        check_matrix(A);
        check_block(X, "X");
        check_block(Y, "Y");
        check_same_shape(X, Y, "X", "Y");
        AFSI_REQUIRE(X->rows == A->n, "X rows != n");
        AFSI_REQUIRE(!overlap(X, Y), "X and Y must not overlap");
        DeviceGuard dg(A->device);
        spmm_apply(A, X->dtype, X->ptr, Y->ptr, X->cols, X->ld, as_stream(stream));
    });
}

int afsi_estimate_eigencount(afsi_matrix_t A, double a, double b, int degree, int32_t damping,
                             double m_exp, const afsi_block *Z, afsi_block *Y, afsi_block *work,
                             double *per_probe, double *estimate, void *stream) {
    return guarded([&] {
        check_matrix(A);
        AFSI_REQUIRE(per_probe != nullptr && estimate != nullptr, "NULL per_probe / estimate");
        AFSI_REQUIRE(A->has_bounds, "spectral bounds of A are not set");
        check_block(Z, "Z");
        check_block(Y, "Y");
        check_block(work, "work");
        check_fp64(Z, "Z");
        check_same_shape(Z, Y, "Z", "Y");
        check_same_shape(Z, work, "Z", "work");
        AFSI_REQUIRE(Z->rows == A->n, "Z has %lld rows, A has %lld", (long long)Z->rows,
                     (long long)A->n);
        AFSI_REQUIRE(Z->cols >= 1, "Z needs at least one probe column");
        AFSI_REQUIRE(!overlap(Z, Y) && !overlap(Z, work) && !overlap(Y, work),
                     "Z, Y and work must not overlap");
        AFSI_REQUIRE(degree >= 1, "degree must be >= 1 (got %d)", degree);
        // the damped filter of eq. (AdaPolySI) at its full degree, as the paper's projector
        std::vector<double> c(degree + 1);
        filter_coefficients(A->lmin, A->lmax, a, b, degree, damping, m_exp, c.data());
        DeviceGuard dg(A->device);
        hipStream_t s = as_stream(stream);
        filter_apply(A, c.data(), degree, Z->dtype, Z->ptr, Y->ptr, work->ptr, Z->cols, Z->ld, s);
        const int64_t m = Z->cols;
        Workspace &ws = workspace(s);
        double *d = (double *)ws.dev_reserve(SLOT_VEC, sizeof(double) * m);
        column_dots_dev(Z->dtype, Z->ptr, Z->ld, Y->ptr, Y->ld, Z->rows, m, d, s);
        double *h = (double *)ws.host_reserve(1, sizeof(double) * m);
        AFSI_HIP(hipMemcpyAsync(h, d, sizeof(double) * m, hipMemcpyDeviceToHost, s));
        AFSI_HIP(hipStreamSynchronize(s));
        double sum = 0.0;
        for (int64_t i = 0; i < m; ++i) {
            per_probe[i] = h[i];
            sum += h[i];
        }
        *estimate = sum / (double)m;
    });
}

int afsi_clenshaw_step_params(const double *coeffs, int degree, int step, double l1, double l2,
                              afsi_step_group *g) {
    return guarded([&] {
        AFSI_REQUIRE(coeffs && g, "NULL argument");
        const int64_t c0 = g->col0, nc = g->ncols;
        step_params(coeffs, degree, step, l1, l2, g);
        g->col0 = c0;
        g->ncols = nc;
    });
}

int afsi_clenshaw_step_grouped(afsi_matrix_t A, int ngroups, const afsi_slice_blocks *slices,
                               int32_t dtype, void *stream) {
    return guarded([&] {
        check_matrix(A);
        DeviceGuard dg(A->device);
        grouped_step(A, ngroups, slices, dtype, as_stream(stream));
    });
}

int afsi_filter_batched(afsi_matrix_t A, int nslices, const afsi_slice_filter *slices,
                        int32_t dtype, void *stream) {
    return guarded([&] {
        check_matrix(A);
        DeviceGuard dg(A->device);
        filter_batched(A, nslices, slices, dtype, as_stream(stream));
    });
}

int afsi_block_size(double estimate, double mu, int64_t n, int64_t *p_out) {
    return guarded([&] {
        AFSI_REQUIRE(p_out != nullptr, "p_out is NULL");
        AFSI_REQUIRE(mu > 0.0 && std::isfinite(mu), "mu must be positive (got %g)", mu);
        AFSI_REQUIRE(n >= 1, "n must be >= 1");
        AFSI_REQUIRE(std::isfinite(estimate), "estimate is not finite");
        const double want = std::ceil(mu * estimate);
        *p_out = want < 1.0 ? 1 : (want >= (double)n ? n : (int64_t)want);
    });
}

int afsi_clenshaw_step_batched(afsi_matrix_t A, int ngroups, const afsi_step_group *groups,
                               const afsi_block *X, afsi_block *P0, afsi_block *P1, void *stream) {
    return guarded([&] {
        check_matrix(A);
        check_block(X, "X");
        check_block(P0, "P0");
        check_block(P1, "P1");
        check_same_shape(X, P0, "X", "P0");
        check_same_shape(X, P1, "X", "P1");
        AFSI_REQUIRE(X->rows == A->n, "X rows != n");
        AFSI_REQUIRE(!overlap(X, P0) && !overlap(X, P1) && !overlap(P0, P1),
                     "X, P0 and P1 must not overlap");
        DeviceGuard dg(A->device);
        batched_step(A, ngroups, groups, X->dtype, X->ptr, P0->ptr, P1->ptr, X->cols, X->ld,
                     as_stream(stream));
    });
}

}  // extern "C"

namespace afsi {

void batched_step(afsi_matrix_t A, int ngroups, const afsi_step_group *groups, int dtype,
                  const void *Xp, void *P0p, void *P1p, int64_t ptot, int64_t ld, hipStream_t s) {
    {
        AFSI_REQUIRE(ngroups >= 0 && ngroups <= 64, "ngroups must be in 0..64");
        AFSI_REQUIRE(ngroups == 0 || groups, "groups is NULL");
        const int eb = elem_bytes(dtype);
        const int E = 16 / eb;
        AFSI_REQUIRE((ld * eb) % 16 == 0 && aligned16(Xp) && aligned16(P0p) && aligned16(P1p),
                     "batched step needs 16-byte aligned rows");
        BatchArgs args;
        std::memset(&args, 0, sizeof args);
        std::vector<std::pair<int64_t, int64_t>> ranges;
        for (int g = 0; g < ngroups; ++g) {
            const afsi_step_group &G = groups[g];
            if (!G.active || G.ncols == 0) continue;
            AFSI_REQUIRE(G.col0 >= 0 && G.ncols > 0 && G.col0 + G.ncols <= ptot,
                         "group %d columns out of range", g);
            AFSI_REQUIRE(G.col0 % E == 0 && G.ncols % E == 0,
                         "group %d: col0 and ncols must be multiples of %d", g, E);
            AFSI_REQUIRE(G.src >= 0 && G.src <= 2 && (G.dst == 1 || G.dst == 2) && G.src != G.dst,
                         "group %d: bad src/dst", g);
            for (auto &r : ranges)
                AFSI_REQUIRE(G.col0 + G.ncols <= r.first || r.first + r.second <= G.col0,
                             "groups overlap");
            ranges.push_back({G.col0, G.ncols});
            const int k = args.ngroups++;
            args.vec0[k] = (int)(G.col0 / E);
            args.vec1[k] = (int)((G.col0 + G.ncols) / E);
            args.src[k] = G.src;
            args.dst[k] = G.dst;
            args.has_v[k] = G.has_v;
            args.sigma[k] = G.sigma;
            args.tau[k] = G.tau;
            args.alpha[k] = G.alpha;
        }
        if (args.ngroups == 0 || A->n == 0) return;
        const MatView mv = matrix_view(A, dtype, s);
        const int p16 = (int)((ptot * eb + 15) / 16);
        const int64_t ldv = ld * eb / 16;
        switch (dtype) {
        case AFSI_R64: clenshaw_r64_batched(mv, Xp, P0p, P1p, p16, ldv, args, s); break;
        case AFSI_R32: clenshaw_r32_batched(mv, Xp, P0p, P1p, p16, ldv, args, s); break;
        case AFSI_C128: clenshaw_c128_batched(mv, Xp, P0p, P1p, p16, ldv, args, s); break;
        case AFSI_C64: clenshaw_c64_batched(mv, Xp, P0p, P1p, p16, ldv, args, s); break;
        }
        AFSI_HIP(hipGetLastError());
    }
}

int grouped_step(afsi_matrix_t A, int ngroups, const afsi_slice_blocks *slices, int dtype,
                 hipStream_t s, int *kernel_launches) {
    if (kernel_launches) *kernel_launches = 0;
    AFSI_REQUIRE(ngroups >= 0 && (ngroups == 0 || slices != nullptr), "bad slice list");
    AFSI_REQUIRE(dtype >= AFSI_R64 && dtype <= AFSI_C64, "unknown dtype %d", dtype);
    const int eb = elem_bytes(dtype);
    const int64_t n = A->n;
    std::vector<int> act;
    std::vector<std::pair<uintptr_t, uintptr_t>> spans;
    for (int g = 0; g < ngroups; ++g) {
        const afsi_slice_blocks &S = slices[g];
        if (!S.step.active || S.step.ncols == 0) continue;
        const afsi_step_group &G = S.step;
        AFSI_REQUIRE(G.ncols > 0 && S.ld >= G.ncols, "slice %d: bad ncols / ld", g);
        AFSI_REQUIRE(S.X && S.P0 && S.P1, "slice %d: NULL block", g);
        AFSI_REQUIRE(G.src >= 0 && G.src <= 2 && (G.dst == 1 || G.dst == 2) && G.src != G.dst,
                     "slice %d: bad src/dst", g);
        const uintptr_t len = n == 0 ? 0 : (uintptr_t)(((n - 1) * S.ld + G.ncols) * eb);
        for (const void *ptr : {S.X, (const void *)S.P0, (const void *)S.P1}) {
            const uintptr_t a = (uintptr_t)ptr, b = a + len;
            for (auto &o : spans)
                AFSI_REQUIRE(b <= o.first || o.second <= a, "slice %d overlaps another block", g);
            spans.push_back({a, b});
        }
        act.push_back(g);
    }
    if (act.empty() || n == 0) return 0;
    const MatView mv = matrix_view(A, dtype, s);
    int taken = 0;
    // slices whose rows are whole 16-byte vectors go to the grouped kernel, by width
    std::map<int, std::vector<int>> by_width;
    std::vector<int> rest;
    for (int g : act) {
        const afsi_slice_blocks &S = slices[g];
        const bool vec = (S.step.ncols * eb) % 16 == 0 && (S.ld * eb) % 16 == 0 &&
                         aligned16(S.X) && aligned16(S.P0) && aligned16(S.P1);
        if (vec && S.step.ncols * eb / 16 < (1 << 30)) by_width[(int)(S.step.ncols * eb / 16)].push_back(g);
        else rest.push_back(g);
    }
    for (auto &kv : by_width) {
        const int p16 = kv.first;
        const std::vector<int> &gs = kv.second;
        for (size_t g0 = 0; g0 < gs.size(); g0 += kGroupedMax) {
            GroupArgs args;
            std::memset(&args, 0, sizeof args);
            const size_t cnt = std::min<size_t>(kGroupedMax, gs.size() - g0);
            for (size_t k = 0; k < cnt; ++k) {
                const afsi_slice_blocks &S = slices[gs[g0 + k]];
                args.X[k] = S.X;
                args.P0[k] = S.P0;
                args.P1[k] = S.P1;
                args.ldv[k] = S.ld * eb / 16;
                args.src[k] = S.step.src;
                args.dst[k] = S.step.dst;
                args.has_v[k] = S.step.has_v;
                args.sigma[k] = S.step.sigma;
                args.tau[k] = S.step.tau;
                args.alpha[k] = S.step.alpha;
            }
            args.ngroups = (int)cnt;
            bool done = false;
            switch (dtype) {
            case AFSI_R64: done = clenshaw_r64_grouped(mv, p16, args, s); break;
            case AFSI_R32: done = clenshaw_r32_grouped(mv, p16, args, s); break;
            case AFSI_C128: done = clenshaw_c128_grouped(mv, p16, args, s); break;
            case AFSI_C64: done = clenshaw_c64_grouped(mv, p16, args, s); break;
            }
            if (!done)
                for (size_t k = 0; k < cnt; ++k) rest.push_back(gs[g0 + k]);
            else {
                taken += (int)cnt;
                if (kernel_launches) ++*kernel_launches;
            }
        }
    }
    // widths without an exact lane mapping, and unaligned blocks: one product each
    for (int g : rest) {
        const afsi_slice_blocks &S = slices[g];
        const void *src = S.step.src == 0 ? S.X : (S.step.src == 1 ? (const void *)S.P0 : S.P1);
        void *dst = S.step.dst == 1 ? S.P0 : S.P1;
        run_step(mv, dtype, src, S.X, dst, S.step.ncols, S.ld, S.step.has_v != 0,
                 S.step.alpha != 0.0, S.step.sigma, S.step.tau, S.step.alpha, s);
    }
    AFSI_HIP(hipGetLastError());
    return taken;
}

void filter_batched(afsi_matrix_t A, int nslices, const afsi_slice_filter *slices, int dtype,
                    hipStream_t s) {
    AFSI_REQUIRE(nslices >= 0 && (nslices == 0 || slices != nullptr), "bad slice list");
    double l1, l2;
    map_coeffs(A, l1, l2);
    int kmax = 0;
    for (int g = 0; g < nslices; ++g) {
        const afsi_slice_filter &F = slices[g];
        AFSI_REQUIRE(F.coeffs != nullptr, "slice %d: coeffs is NULL", g);
        AFSI_REQUIRE(F.degree >= 1, "slice %d: degree must be >= 1 (got %d)", g, F.degree);
        AFSI_REQUIRE(F.ncols >= 0 && F.ld >= F.ncols && F.ld >= 1, "slice %d: bad ncols / ld", g);
        AFSI_REQUIRE(F.ncols == 0 || (F.X && F.Y && F.work), "slice %d: NULL block", g);
        kmax = std::max(kmax, (int)F.degree);
    }
    // per slice: P[0] = X, the last product lands in Y = P[1 + (k-1) % 2] (as filter_apply)
    std::vector<afsi_slice_blocks> sb(nslices);
    for (int g = 0; g < nslices; ++g) {
        const afsi_slice_filter &F = slices[g];
        void *P[2];
        P[(F.degree - 1) % 2] = F.Y;
        P[F.degree % 2] = F.work;
        sb[g].X = F.X;
        sb[g].P0 = P[0];
        sb[g].P1 = P[1];
        sb[g].ld = F.ld;
    }
    for (int st = 0; st < kmax; ++st) {
        for (int g = 0; g < nslices; ++g) {
            const afsi_slice_filter &F = slices[g];
            afsi_step_group &G = sb[g].step;
            std::memset(&G, 0, sizeof G);
            if (st < F.degree && F.ncols > 0) {
                step_params(F.coeffs, F.degree, st, l1, l2, &G);
                G.col0 = 0;
                G.ncols = F.ncols;
                G.active = 1;
            }
        }
        grouped_step(A, nslices, sb.data(), dtype, s);
    }
}

void gather_cols(int dtype, const void *src, int64_t n, int64_t ld, const int32_t *cols,
                 int64_t count, void *dst, int64_t ldd, hipStream_t s) {
    if (count == 0 || n == 0) return;
    afsi_block sb{const_cast<void *>(src), n, ld, ld, dtype};
    afsi_block db{dst, n, count, ldd, dtype};
    Workspace &ws = workspace(s);
    int32_t *d = (int32_t *)ws.dev_reserve(SLOT_GATHER, sizeof(int32_t) * count);
    int32_t *h = (int32_t *)ws.host_reserve(1, sizeof(int32_t) * count);
    std::memcpy(h, cols, sizeof(int32_t) * count);
    AFSI_HIP(hipMemcpyAsync(d, h, sizeof(int32_t) * count, hipMemcpyHostToDevice, s));
    launch_gather_columns(sb, d, count, db, s);
    AFSI_HIP(hipStreamSynchronize(s));  // the index list lives in reusable scratch
}

}  // namespace afsi

extern "C" {

int afsi_block_inner(const afsi_block *X, const afsi_block *Y, afsi_block *G, void *stream) {
    return guarded([&] {
        check_block(X, "X");
        check_block(Y, "Y");
        check_block(G, "G");
        check_fp64(X, "X");
        AFSI_REQUIRE(X->dtype == Y->dtype && X->dtype == G->dtype, "dtypes differ");
        AFSI_REQUIRE(X->rows == Y->rows && G->rows == X->cols && G->cols == Y->cols,
                     "shapes do not match G = X^H Y");
        AFSI_REQUIRE(!overlap(G, X) && !overlap(G, Y), "G overlaps an input");
        inner_dev(X->dtype, X->ptr, X->ld, Y->ptr, Y->ld, X->rows, X->cols, Y->cols,
                  (double *)G->ptr, G->ld, as_stream(stream));
    });
}

int afsi_block_gemm(const afsi_block *X, const afsi_block *M, double beta, afsi_block *Y,
                    void *stream) {
    return guarded([&] {
        check_block(X, "X");
        check_block(M, "M");
        check_block(Y, "Y");
        check_fp64(X, "X");
        AFSI_REQUIRE(X->dtype == M->dtype && X->dtype == Y->dtype, "dtypes differ");
        AFSI_REQUIRE(M->rows == X->cols && Y->rows == X->rows && Y->cols == M->cols,
                     "shapes do not match Y = X M");
        AFSI_REQUIRE(!overlap(Y, X) && !overlap(Y, M), "Y overlaps an input");
        gemm_dev(X->dtype, X->ptr, X->ld, (const double *)M->ptr, M->ld, X->rows, X->cols, M->cols,
                 1.0, beta, Y->ptr, Y->ld, as_stream(stream));
    });
}

int afsi_orthonormalize(const afsi_block *locked, afsi_block *X, afsi_block *work, void *stream) {
    return guarded([&] {
        check_block(X, "X");
        check_block(work, "work");
        check_fp64(X, "X");
        check_same_shape(X, work, "X", "work");
        AFSI_REQUIRE(!overlap(X, work), "X and work overlap");
        AFSI_REQUIRE(X->cols <= X->rows, "more columns than rows");
        hipStream_t s = as_stream(stream);
        if (locked && locked->cols > 0) {
            check_block(locked, "locked");
            AFSI_REQUIRE(locked->dtype == X->dtype && locked->rows == X->rows, "locked shape/dtype");
            AFSI_REQUIRE(!overlap(locked, X) && !overlap(locked, work), "locked overlaps X/work");
            AFSI_REQUIRE(locked->cols + X->cols <= X->rows, "too many columns");
            project_out_dev(X->dtype, locked->ptr, locked->ld, locked->cols, X->ptr, X->ld, X->rows,
                            X->cols, s);
        }
        orthonormalize_dev(X->dtype, X->ptr, work->ptr, X->rows, X->cols, X->ld, s, nullptr);
    });
}

int afsi_rayleigh_ritz(afsi_matrix_t A, const afsi_block *Q, afsi_block *V, afsi_block *AV,
                       double *ritz_out, void *stream) {
    return guarded([&] {
        check_matrix(A);
        check_block(Q, "Q");
        check_block(V, "V");
        check_block(AV, "AV");
        check_fp64(Q, "Q");
        check_same_shape(Q, V, "Q", "V");
        check_same_shape(Q, AV, "Q", "AV");
        AFSI_REQUIRE(Q->rows == A->n, "Q rows != n");
        AFSI_REQUIRE(!overlap(Q, V) && !overlap(Q, AV) && !overlap(V, AV), "blocks overlap");
        AFSI_REQUIRE(ritz_out != nullptr || Q->cols == 0, "ritz_out is NULL");
        DeviceGuard dg(A->device);
        rayleigh_ritz_dev(A, Q->dtype, Q->ptr, V->ptr, AV->ptr, Q->rows, Q->cols, Q->ld, ritz_out,
                          as_stream(stream));
    });
}

int afsi_orthonormalize_rayleigh_ritz(afsi_matrix_t A, afsi_block *X, afsi_block *work,
                                      afsi_block *V, afsi_block *AV, double *ritz_out,
                                      void *stream) {
    return guarded([&] {
        check_matrix(A);
        check_block(X, "X");
        check_block(work, "work");
        check_block(V, "V");
        check_block(AV, "AV");
        check_fp64(X, "X");
        check_same_shape(X, work, "X", "work");
        check_same_shape(X, V, "X", "V");
        check_same_shape(X, AV, "X", "AV");
        AFSI_REQUIRE(X->rows == A->n, "X rows != n");
        AFSI_REQUIRE(X->ld == work->ld && X->ld == V->ld && X->ld == AV->ld,
                     "X, work, V and AV must share one leading dimension");
        AFSI_REQUIRE(!overlap(X, work) && !overlap(X, V) && !overlap(work, V) && !overlap(X, AV) &&
                         !overlap(V, AV),
                     "blocks overlap (only AV and work may share memory)");
        AFSI_REQUIRE(ritz_out != nullptr || X->cols == 0, "ritz_out is NULL");
        DeviceGuard dg(A->device);
        orthonormalize_rr_dev(A, X->dtype, X->ptr, work->ptr, V->ptr, AV->ptr, X->rows, X->cols,
                              X->ld, ritz_out, as_stream(stream), nullptr, nullptr);
    });
}

int afsi_residual_norms(const afsi_block *V, const afsi_block *AV, const double *lambda,
                        double *norms_out, void *stream) {
    return guarded([&] {
        check_block(V, "V");
        check_block(AV, "AV");
        check_fp64(V, "V");
        AFSI_REQUIRE(V->rows == AV->rows && V->cols == AV->cols && V->dtype == AV->dtype,
                     "V and AV shapes differ");
        AFSI_REQUIRE(V->cols == 0 || (lambda && norms_out), "NULL lambda / norms_out");
        residual_norms_host(V->dtype, V->ptr, V->ld, AV->ptr, AV->ld, lambda, V->rows, V->cols,
                            norms_out, as_stream(stream));
    });
}

int afsi_residual_norms_noalloc(const afsi_block *V, const afsi_block *AV, const double *lambda,
                                double *norms_out, void *stream) {
    return guarded([&] {
        check_block(V, "V");
        check_block(AV, "AV");
        check_fp64(V, "V");
        AFSI_REQUIRE(V->rows == AV->rows && V->cols == AV->cols && V->dtype == AV->dtype,
                     "V and AV shapes differ");
        AFSI_REQUIRE(V->cols == 0 || (lambda && norms_out), "NULL lambda / norms_out");
        residual_norms_noalloc(V->dtype, V->ptr, V->ld, AV->ptr, AV->ld, lambda, V->rows, V->cols,
                               norms_out, as_stream(stream));
    });
}

int afsi_convert_block(const afsi_block *src, afsi_block *dst, void *stream) {
    return guarded([&] {
        check_block(src, "src");
        check_block(dst, "dst");
        AFSI_REQUIRE(src->rows == dst->rows && src->cols == dst->cols, "shapes differ");
        AFSI_REQUIRE(is_complex(src->dtype) == is_complex(dst->dtype), "real/complex mismatch");
        AFSI_REQUIRE(!overlap(src, dst), "src and dst overlap");
        launch_convert(*src, *dst, as_stream(stream));
    });
}

int afsi_gather_columns(const afsi_block *src, const int32_t *cols, int64_t count, afsi_block *dst,
                        void *stream) {
    return guarded([&] {
        check_block(src, "src");
        check_block(dst, "dst");
        AFSI_REQUIRE(count >= 0 && dst->cols == count && dst->rows == src->rows &&
                         dst->dtype == src->dtype,
                     "dst must be rows x count of src's dtype");
        AFSI_REQUIRE(count == 0 || cols, "cols is NULL");
        for (int64_t t = 0; t < count; ++t)
            AFSI_REQUIRE(cols[t] >= 0 && cols[t] < src->cols, "column index %d out of range", cols[t]);
        AFSI_REQUIRE(!overlap(src, dst), "src and dst overlap");
        if (count == 0 || src->rows == 0) return;
        hipStream_t s = as_stream(stream);
        Workspace &ws = workspace(s);
        int32_t *d = (int32_t *)ws.dev_reserve(SLOT_GATHER, sizeof(int32_t) * count);
        AFSI_HIP(hipMemcpyAsync(d, cols, sizeof(int32_t) * count, hipMemcpyHostToDevice, s));
        launch_gather_columns(*src, d, count, *dst, s);
        AFSI_HIP(hipStreamSynchronize(s));
    });
}

// perm must hold each of 0..n-1 once
static void check_permutation(const int64_t *perm, int64_t n) {
    AFSI_REQUIRE(n == 0 || perm != nullptr, "perm is NULL");
    std::vector<char> seen(n, 0);
    for (int64_t i = 0; i < n; ++i) {
        AFSI_REQUIRE(perm[i] >= 0 && perm[i] < n, "perm[%lld] = %lld out of range", (long long)i,
                     (long long)perm[i]);
        AFSI_REQUIRE(!seen[perm[i]], "perm repeats %lld", (long long)perm[i]);
        seen[perm[i]] = 1;
    }
}

int afsi_permute_rows(const afsi_block *src, const int64_t *perm, int32_t inverse, afsi_block *dst,
                      void *stream) {
    return guarded([&] {
        check_block(src, "src");
        check_block(dst, "dst");
        AFSI_REQUIRE(src->rows == dst->rows && src->cols == dst->cols && src->dtype == dst->dtype,
                     "dst must have src's shape and dtype");
        AFSI_REQUIRE(!overlap(src, dst), "src and dst overlap");
        check_permutation(perm, src->rows);
        if (src->rows == 0 || src->cols == 0) return;
        hipStream_t s = as_stream(stream);
        Workspace &ws = workspace(s);
        int64_t *d = (int64_t *)ws.dev_reserve(SLOT_GATHER, sizeof(int64_t) * src->rows);
        AFSI_HIP(hipMemcpyAsync(d, perm, sizeof(int64_t) * src->rows, hipMemcpyHostToDevice, s));
        launch_permute_rows(*src, d, inverse != 0, *dst, s);
        AFSI_HIP(hipStreamSynchronize(s));
    });
}

int afsi_grid_order(int64_t nx, int64_t ny, int64_t nz, int64_t ty, int64_t tz, int32_t fold_x,
                    int64_t *perm) {
    return guarded([&] {
        AFSI_REQUIRE(nx >= 0 && ny >= 0 && nz >= 0, "negative grid size");
        AFSI_REQUIRE(ty >= 1 && tz >= 1, "tile sides must be at least 1");
        const int64_t n = nx * ny * nz;
        AFSI_REQUIRE(n == 0 || perm != nullptr, "perm is NULL");
        // x positions along a pencil: natural, or folded (0, nx-1, 1, nx-2, ...) so that on a
        // periodic x axis every neighbour, the wrap-around pair included, is at most two
        // positions away
        std::vector<int64_t> xs(nx);
        for (int64_t i = 0; i < nx; ++i) xs[i] = !fold_x ? i : (i % 2 == 0 ? i / 2 : nx - 1 - i / 2);
        // pencils: ty x tz tiles of the (y, z) plane, one after another (y tile outer), each
        // running along x with its (y, z) points in natural order at every x
        int64_t k = 0;
        for (int64_t y0 = 0; y0 < ny; y0 += ty)
            for (int64_t z0 = 0; z0 < nz; z0 += tz)
                for (int64_t xi = 0; xi < nx; ++xi)
                    for (int64_t y = y0; y < std::min(ny, y0 + ty); ++y)
                        for (int64_t z = z0; z < std::min(nz, z0 + tz); ++z)
                            perm[k++] = (xs[xi] * ny + y) * nz + z;
    });
}

int afsi_csr_permute(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                     const void *vals, int32_t val_dtype, const int64_t *perm, int64_t *out_row_ptr,
                     int32_t *out_col_idx, void *out_vals) {
    return guarded([&] {
        AFSI_REQUIRE(n >= 0 && nnz >= 0, "negative size");
        AFSI_REQUIRE(n < (1LL << 31), "n must be below 2^31");
        AFSI_REQUIRE(val_dtype == AFSI_R64 || val_dtype == AFSI_C128,
                     "values must be R64 or C128 (got %d)", val_dtype);
        AFSI_REQUIRE(row_ptr && out_row_ptr, "row_ptr / out_row_ptr is NULL");
        AFSI_REQUIRE(nnz == 0 || (col_idx && vals && out_col_idx && out_vals), "NULL array");
        AFSI_REQUIRE(row_ptr[0] == 0 && row_ptr[n] == nnz, "row_ptr must start at 0 and end at nnz");
        check_permutation(perm, n);
        std::vector<int32_t> inv(n);
        for (int64_t i = 0; i < n; ++i) inv[perm[i]] = (int32_t)i;
        out_row_ptr[0] = 0;
        for (int64_t i = 0; i < n; ++i) {
            const int64_t r = perm[i];
            AFSI_REQUIRE(row_ptr[r + 1] >= row_ptr[r], "row_ptr decreases at row %lld", (long long)r);
            out_row_ptr[i + 1] = out_row_ptr[i] + (row_ptr[r + 1] - row_ptr[r]);
        }
        const size_t eb = (size_t)elem_bytes(val_dtype);
        const char *v = (const char *)vals;
        char *ov = (char *)out_vals;
        std::vector<std::pair<int32_t, int64_t>> row;
        for (int64_t i = 0; i < n; ++i) {
            // row i of P A P^T is row perm[i] of A, columns renamed by the inverse
            // permutation and sorted
            const int64_t r = perm[i], e0 = row_ptr[r], len = row_ptr[r + 1] - e0, o = out_row_ptr[i];
            row.resize(len);
            for (int64_t t = 0; t < len; ++t) {
                const int32_t c = col_idx[e0 + t];
                AFSI_REQUIRE(c >= 0 && c < n, "column %d out of range in row %lld", c, (long long)r);
                row[t] = {inv[c], e0 + t};
            }
            std::sort(row.begin(), row.end());
            for (int64_t t = 0; t < len; ++t) {
                out_col_idx[o + t] = row[t].first;
                std::memcpy(ov + (size_t)(o + t) * eb, v + (size_t)row[t].second * eb, eb);
            }
        }
    });
}

int afsi_select_degree(const double *ritz, int64_t p, int64_t e, const double *coeffs, int kmax,
                       double l1, double l2, double tau_a, int *degree_out) {
    return guarded([&] {
        AFSI_REQUIRE(ritz && coeffs && degree_out, "NULL argument");
        AFSI_REQUIRE(kmax >= 1, "kmax must be >= 1");
        *degree_out = select_degree(ritz, p, e, coeffs, kmax, l1, l2, tau_a);
    });
}

int afsi_host_eigh(int64_t p, int32_t dtype, const double *B, int64_t ldb, double *w, double *U,
                   int64_t ldu) {
    return guarded([&] {
        AFSI_REQUIRE(dtype == AFSI_R64 || dtype == AFSI_C128, "dtype must be R64 or C128");
        AFSI_REQUIRE(p >= 0 && ldb >= p && ldu >= p, "bad shape");
        AFSI_REQUIRE(p == 0 || (B && w && U), "NULL argument");
        host_eigh_or_throw(p, dtype == AFSI_C128, B, ldb, w, U, ldu);
    });
}

}  // extern "C"

namespace afsi {
void host_eigh_or_throw(int64_t p, bool cplx, const double *B, int64_t ldb, double *w, double *U,
                        int64_t ldu) {
    const int comp = cplx ? 2 : 1;
    for (int64_t i = 0; i < p; ++i)
        for (int64_t j = 0; j < comp * p; ++j)
            AFSI_REQUIRE(std::isfinite(B[i * comp * ldb + j]),
                         "Hermitian eigensolver input has a non-finite entry at row %lld",
                         (long long)i);
    if (!host_eigh(p, cplx, B, ldb, w, U, ldu))
        AFSI_FAIL(AFSI_E_NOCONV, "Hermitian eigensolver (tridiagonal QR) did not converge");
}
}  // namespace afsi

extern "C" {

int afsi_host_cholesky_inverse(int64_t p, int32_t dtype, double *G, int64_t ldg, double shift) {
    return guarded([&] {
        AFSI_REQUIRE(dtype == AFSI_R64 || dtype == AFSI_C128, "dtype must be R64 or C128");
        AFSI_REQUIRE(p >= 0 && ldg >= p && (p == 0 || G), "bad argument");
        if (!host_cholesky_inverse(p, dtype == AFSI_C128, G, ldg, shift))
            AFSI_FAIL(AFSI_E_NOT_HPD, "matrix is not positive definite");
    });
}

int afsi_lock_select(const double *ritz, int64_t p, const double *res, uint8_t *in_interval,
                     double a, double b, double tau_abs, int64_t n_lock, int64_t *n_check_prev,
                     uint8_t *lock, int *done) {
    return guarded([&] {
        AFSI_REQUIRE(ritz && res && in_interval && n_check_prev && lock && done, "NULL argument");
        lock_select(ritz, p, res, in_interval, a, b, tau_abs, n_lock, n_check_prev, lock, done);
    });
}

}  // extern "C"
