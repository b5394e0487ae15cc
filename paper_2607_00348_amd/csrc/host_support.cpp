// Host-side helpers of the search: the period grid (Sect. 2.2.1), the
// duration grid over the period-duration envelope (Sect. 2.2.2) and the
// unit-depth limb-darkened transit template.  None of these run per window;
// tls_search takes their outputs as plain arrays.
#include <cmath>
#include <vector>

#include "gtls.h"

namespace {

constexpr double kG = 6.674e-11;      // SI; the paper does not state its constants
constexpr double kMsun = 1.989e30;
constexpr double kRsun = 6.957e8;
constexpr double kDay = 86400.0;
constexpr double kPi = 3.14159265358979323846;

// Gauss-Legendre nodes/weights on [-1, 1] (Newton on P_n).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int k = 1; k <= n; ++k) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
            }
            dp = n * (z * p0 - p1) / (z * z - 1.0);
            double dz = p0 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

struct Quadrature {
    std::vector<std::vector<double>> xs, ws;
    Quadrature() {
        for (int n = 8; n <= 512; n *= 2) {
            std::vector<double> x, w;
            gauss_legendre(n, x, w);
            xs.push_back(x);
            ws.push_back(w);
        }
    }
};

double intensity(double r, double u1, double u2) {
    double mu = std::sqrt(std::fmax(0.0, 1.0 - r * r));
    double a = 1.0 - mu;
    return 1.0 - u1 * a - u2 * a * a;
}

// Half-angle of the stellar annulus of radius r inside a planet disk of
// radius p at separation z.
double half_angle(double r, double z, double p) {
    if (r <= p - z) return kPi;
    if (r <= z - p || r >= z + p) return 0.0;
    double c = (r * r + z * z - p * p) / (2.0 * r * z);
    return std::acos(std::fmin(1.0, std::fmax(-1.0, c)));
}

// Integral of I(r) 2 r kappa(r) over [a, b] with r = a + (b-a)(1 - cos th)/2,
// which turns the square-root edges of kappa and mu into smooth ends.
double panel(const Quadrature& q, double a, double b, double z, double p, double u1, double u2) {
    double prev = 0.0;
    for (size_t lvl = 0; lvl < q.xs.size(); ++lvl) {
        const auto& x = q.xs[lvl];
        const auto& w = q.ws[lvl];
        double acc = 0.0;
        for (size_t k = 0; k < x.size(); ++k) {
            double th = 0.5 * kPi * (x[k] + 1.0);
            double r = a + 0.5 * (b - a) * (1.0 - std::cos(th));
            double jac = 0.5 * (b - a) * std::sin(th) * 0.5 * kPi;
            acc += w[k] * jac * intensity(r, u1, u2) * 2.0 * r * half_angle(r, z, p);
        }
        if (lvl > 0 && std::fabs(acc - prev) <= 1e-15 * std::fmax(1e-300, std::fabs(acc))) return acc;
        prev = acc;
    }
    return prev;
}

double occulted(const Quadrature& q, double z, double p, double u1, double u2) {
    if (z >= 1.0 + p) return 0.0;
    double lo = std::fmax(0.0, z - p), hi = std::fmin(1.0, z + p);
    if (hi <= lo) return 0.0;
    double cuts[4];
    int nc = 0;
    cuts[nc++] = lo;
    double k1 = std::fabs(z - p), k2 = z + p;
    if (k1 > lo && k1 < hi) cuts[nc++] = k1;
    if (k2 > lo && k2 < hi && k2 != k1) cuts[nc++] = k2;
    cuts[nc++] = hi;
    double total = 0.0;
    for (int i = 0; i + 1 < nc; ++i) total += panel(q, cuts[i], cuts[i + 1], z, p, u1, u2);
    return total / (kPi * (1.0 - u1 / 3.0 - u2 / 6.0));
}

}  // namespace

extern "C" gtls_status gtls_period_grid_ofir(double baseline_days, double os, double m_sun,
                                             double r_sun, double pmin_days, double pmax_days,
                                             double* out, int32_t cap, int32_t* n_out) {
    if (!(baseline_days > 0.0) || !(os > 0.0) || !(m_sun > 0.0) || !(r_sun > 0.0) ||
        pmin_days < 0.0 || pmax_days < 0.0 || !n_out || (cap > 0 && !out))
        return GTLS_EINVAL;
    double s = baseline_days * kDay;
    double gm = kG * (m_sun * kMsun);
    double r = r_sun * kRsun;
    double a3 = 3.0 * r;
    double roche = (1.0 / (2.0 * kPi)) * std::sqrt(gm / (a3 * a3 * a3));
    double fmin = (pmax_days <= 0.0) ? (2.0 / s) : 1.0 / (pmax_days * kDay);
    double fmax = (pmin_days <= 0.0) ? roche : 1.0 / (pmin_days * kDay);
    if (!(fmax > fmin)) return GTLS_EINVAL;
    double A = std::pow(2.0 * kPi, 2.0 / 3.0) / kPi * r / std::pow(gm, 1.0 / 3.0) / (s * os);
    double C = std::pow(fmin, 1.0 / 3.0) - A / 3.0;
    double N = (std::pow(fmax, 1.0 / 3.0) - std::pow(fmin, 1.0 / 3.0) + A / 3.0) * 3.0 / A;
    if (!(N < 2.0e9)) return GTLS_EINVAL;
    int64_t count = (int64_t)std::ceil(N);
    double pmin = 1.0 / fmax / kDay, pmax = 1.0 / fmin / kDay;
    int64_t k = 0;
    for (int64_t i = count; i >= 1; --i) {
        double x = A / 3.0 * (double)i + C;
        double f = x * x * x;
        double p = 1.0 / f / kDay;
        if (p >= pmin && p <= pmax) {
            if (cap > 0 && k < cap) out[k] = p;
            ++k;
        }
    }
    *n_out = (int32_t)k;
    if (cap > 0 && k > cap) return GTLS_EINVAL;
    return GTLS_OK;
}

extern "C" gtls_status gtls_duration_grid(double pmin_days, double pmax_days, int32_t n,
                                          double k_min, double k_max, double q_cap, double* out) {
    if (!(pmin_days > 0.0) || !(pmax_days >= pmin_days) || n < 1 || !out || !(k_min > 0.0) ||
        !(k_max > k_min) || !(q_cap > 0.0))
        return GTLS_EINVAL;
    double lo_q = k_min * std::pow(pmin_days * kDay, -2.0 / 3.0);
    double hi_q = std::fmin(k_max * std::pow(pmax_days * kDay, -2.0 / 3.0), q_cap);
    double t_lo = lo_q * pmin_days;
    double t_hi = hi_q * pmax_days;
    if (!(t_hi >= t_lo)) return GTLS_EINVAL;
    if (n == 1) {
        out[0] = t_lo;
        return GTLS_OK;
    }
    double ratio = t_hi / t_lo;
    for (int32_t j = 0; j < n; ++j) out[j] = t_lo * std::pow(ratio, (double)j / (double)(n - 1));
    return GTLS_OK;
}

extern "C" gtls_status gtls_template_quadratic(double u1, double u2, double p, double b,
                                               int32_t m, double* out) {
    if (m < 2 || !out || !(p > 0.0) || !(p < 1.0) || b < 0.0 || !(b < 1.0 + p) ||
        !std::isfinite(u1) || !std::isfinite(u2) || !(1.0 - u1 / 3.0 - u2 / 6.0 > 0.0))
        return GTLS_EINVAL;
    static const Quadrature q;
    double half = std::sqrt((1.0 + p) * (1.0 + p) - b * b);
    double mx = 0.0;
    for (int32_t k = 0; k < m; ++k) {
        double x = ((double)k + 0.5) / (double)m;
        double xx = (2.0 * x - 1.0) * half;
        double z = std::sqrt(b * b + xx * xx);
        out[k] = occulted(q, z, p, u1, u2);
        if (out[k] > mx) mx = out[k];
    }
    if (!(mx > 0.0)) return GTLS_EINVAL;
    for (int32_t k = 0; k < m; ++k) out[k] = out[k] / mx;
    return GTLS_OK;
}
