// Host-side pieces of the method: filter coefficients (Section 2.2), the
// Clenshaw product schedule (Algorithm 2), degree selection (Algorithm 3) and the
// spurious-value / locking test of Algorithm 4 (eq. (tau_s)).
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace afsi {

static const double kPi = 3.14159265358979323846;

void filter_coefficients(double lmin, double lmax, double a, double b, int kmax, int damping,
                         double m_exp, double *coeffs) {
    AFSI_REQUIRE(lmax > lmin, "spectral bounds need lmin < lmax (got %g, %g)", lmin, lmax);
    AFSI_REQUIRE(b > a, "interval needs a < b (got %g, %g)", a, b);
    AFSI_REQUIRE(kmax >= 0, "kmax must be >= 0");
    AFSI_REQUIRE(damping >= AFSI_DAMP_NONE && damping <= AFSI_DAMP_LANCZOS, "unknown damping %d",
                 damping);
    AFSI_REQUIRE(damping != AFSI_DAMP_LANCZOS || m_exp >= 0.0, "Lanczos exponent must be >= 0");
    // l(x) = (2x - lmax - lmin) / (lmax - lmin), clipped to [-1, 1] (extreme problems)
    const double width = lmax - lmin;
    const double ta = std::min(1.0, std::max(-1.0, (2.0 * a - lmax - lmin) / width));
    const double tb = std::min(1.0, std::max(-1.0, (2.0 * b - lmax - lmin) / width));
    const double alpha = std::acos(ta), beta = std::acos(tb);
    // c_j of the step function (eq. (c_j)) times the damping factor at degree kmax
    const double q = kPi / (kmax + 2);
    for (int j = 0; j <= kmax; ++j) {
        double c = j == 0 ? (alpha - beta) / kPi
                          : 2.0 / kPi * (std::sin(j * alpha) - std::sin(j * beta)) / j;
        double d = 1.0;
        if (damping == AFSI_DAMP_JACKSON) {
            d = ((kmax + 2 - j) * std::sin(q) * std::cos(j * q) + std::cos(q) * std::sin(j * q)) /
                ((kmax + 2) * std::sin(q));
        } else if (damping == AFSI_DAMP_LANCZOS && j > 0) {
            const double t = j * kPi / (kmax + 1);
            d = std::pow(std::sin(t) / t, m_exp);
        }
        coeffs[j] = c * d;
    }
}

// Product s (0-based) of a degree-k filter computes b_j with j = k-1-s (b_0 = Y):
//   s = 0 : b_{k-1} = (sig a_k) A X + (tau a_k + a_{k-1}) X            (b_k = a_k X folded in)
//   s = 1 : b_{k-2} = sig A b_{k-1} + tau b_{k-1} + (a_{k-2} - a_k) X  (b_k = a_k X subtracted)
//   s >= 2: b_j     = sig A b_{j+1} + tau b_{j+1} - b_{j+2} + a_j X
// with (sig, tau) = (2 l1, 2 l2) for j >= 1 and (l1, l2) for the final j = 0.
// b_j is written to P[s % 2], so Y lands in P[(k-1) % 2].
void step_params(const double *a, int k, int s, double l1, double l2, afsi_step_group *g) {
    AFSI_REQUIRE(k >= 1 && s >= 0 && s < k, "step %d outside 0..%d", s, k - 1);
    const int j = k - 1 - s;
    const double sig = j == 0 ? l1 : 2.0 * l1;
    const double tau = j == 0 ? l2 : 2.0 * l2;
    g->dst = 1 + (s % 2);
    g->active = 1;
    if (s == 0) {
        g->src = 0;
        g->has_v = 0;
        g->sigma = sig * a[k];
        g->tau = tau * a[k] + a[k - 1];
        g->alpha = 0.0;
    } else if (s == 1) {
        g->src = 1;
        g->has_v = 0;
        g->sigma = sig;
        g->tau = tau;
        g->alpha = a[j] - a[k];
    } else {
        g->src = 1 + ((s - 1) % 2);
        g->has_v = 1;
        g->sigma = sig;
        g->tau = tau;
        g->alpha = a[j];
    }
}

int select_degree(const double *ritz, int64_t p, int64_t e, const double *a, int kmax, double l1,
                  double l2, double tau_a) {
    AFSI_REQUIRE(p >= 1 && e >= 1 && e <= p, "need 1 <= e <= p (e=%lld, p=%lld)", (long long)e,
                 (long long)p);
    std::vector<double> t(p), h0(p, 1.0), h1(p), gam(p), mag(p);
    for (int64_t i = 0; i < p; ++i) {
        t[i] = l1 * ritz[i] + l2;
        h1[i] = t[i];
        gam[i] = a[0];
    }
    for (int j = 1; j <= kmax; ++j) {
        for (int64_t i = 0; i < p; ++i) {
            gam[i] += a[j] * h1[i];
            mag[i] = std::fabs(gam[i]);
        }
        std::sort(mag.begin(), mag.end(), [](double x, double y) { return x > y; });
        const double gp = mag[p - 1], ge = mag[e - 1];
        if (ge != 0.0 && gp / ge < tau_a) return j;
        for (int64_t i = 0; i < p; ++i) {
            const double nx = 2.0 * t[i] * h1[i] - h0[i];
            h0[i] = h1[i];
            h1[i] = nx;
        }
    }
    return kmax;
}

}  // namespace afsi
