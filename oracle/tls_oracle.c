/*
 * tls_oracle.c -- plain, slow, obviously-correct FP64 reference of the
 * Transit Least Squares search as GTLS describes it (Hu, Ge, Jin, Willis,
 * "GTLS: A GPU-accelerated method for periodic transit detection").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load the library built from this file.
 * It shares no code, header, table or helper with the HIP library: every
 * function below is written from the paper's text.
 *
 * Build (done by the package build step):
 *   gcc -O2 -mfma -ffp-contract=off -fopenmp -shared -fPIC tls_oracle.c -lm
 * -ffp-contract=off keeps every a*b+c as two rounded operations; the only
 * fused operations are the explicit fma() calls of the correlation sums.
 *
 * Pins: every function here is checked against something other than itself
 * (brute force, closed forms, library routines, invariants) by the tests
 * under tests/ that are marked "not gpu".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SECONDS_PER_DAY 86400.0
#define TWO_POW_53 9007199254740992.0

/* ------------------------------------------------------------------------ */
/* Null chi-square: the flat model m = 1 everywhere (Sect. 2.3.4 takes the
 * out-of-transit model to be unity).  chi2_0 = sum_i w_i (y_i - 1)^2 with
 * w_i = 1/dy_i^2, summed in input order with Neumaier compensation.        */
double oracle_chi2_null(const double *y, const double *dy, int64_t n)
{
    double sum = 0.0, comp = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double w = 1.0 / (dy[i] * dy[i]);
        double d = y[i] - 1.0;
        double x = w * (d * d);
        double t = sum + x;
        if (fabs(sum) >= fabs(x))
            comp += (sum - t) + x;
        else
            comp += (x - t) + sum;
        sum = t;
    }
    return sum + comp;
}

/* ------------------------------------------------------------------------ */
/* Phase fold (Sect. 2.3.1): p_i = t_i/P - floor(t_i/P), on the raw times.   */
double oracle_phase(double t, double period)
{
    double x = t / period;
    return x - floor(x);
}

typedef struct { double phi; int32_t idx; } phase_key;

static int cmp_phase_key(const void *a, const void *b)
{
    const phase_key *pa = (const phase_key *)a, *pb = (const phase_key *)b;
    if (pa->phi < pb->phi) return -1;
    if (pa->phi > pb->phi) return 1;
    return (pa->idx > pb->idx) - (pa->idx < pb->idx);
}

/* The folded light curve ordered by phase (Sect. 2.3.1, "then sorted").
 * Ties in phase keep input order, so the (phase, index) key is a total order
 * and any correct sort of it gives the stable argsort.                    */
void oracle_fold_sort(const double *t, int64_t n, double period, int32_t *perm)
{
    phase_key *k = (phase_key *)malloc(sizeof(phase_key) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        k[i].phi = oracle_phase(t[i], period);
        k[i].idx = (int32_t)i;
    }
    qsort(k, (size_t)n, sizeof(phase_key), cmp_phase_key);
    for (int64_t i = 0; i < n; ++i) perm[i] = k[i].idx;
    free(k);
}

/* ------------------------------------------------------------------------ */
/* Duration envelope (Sect. 2.2.2): k_min P^(-2/3) <= T14/P <= k_max P^(-2/3)
 * with P in seconds, and T14/P <= q_cap.  Both sides of the k-inequalities
 * are positive, so they are evaluated cubed, q^3 P^2 against k^3, which needs
 * no transcendental function.                                               */
int oracle_duration_valid(double period_days, double dur_days, int envelope,
                          double k_min, double k_max, double q_cap)
{
    double q = dur_days / period_days;
    if (q > q_cap) return 0;
    if (envelope) {
        double ps = period_days * SECONDS_PER_DAY;
        double lhs = (q * q * q) * (ps * ps);
        if (lhs < k_min * k_min * k_min) return 0;
        if (lhs > k_max * k_max * k_max) return 0;
    }
    return 1;
}

/* D = number of points inside one transit duration (Sect. 2.2.2): the
 * folded curve covers one period with n points, so D = round(n T14 / P),
 * rounded half up and clamped to [1, n].                                    */
int64_t oracle_points_in_duration(int64_t n, double period_days, double dur_days)
{
    double q = dur_days / period_days;
    double d = floor((double)n * q + 0.5);
    if (d < 1.0) return 1;
    if (d > (double)n) return n;
    return (int64_t)d;
}

/* T0 stride (Sect. 2.5): N_skip = n_IT * dt0, taken as floor, at least 1;
 * dt0 = 0 means every offset.                                               */
int64_t oracle_t0_stride(int64_t d, double dt0)
{
    if (!(dt0 > 0.0)) return 1;
    double s = floor(dt0 * (double)d);
    return s < 1.0 ? 1 : (int64_t)s;
}

/* The ideal transit of D points: linear interpolation of the m-sample unit-
 * depth template at the point centres x_k = (k + 1/2)/D.                    */
void oracle_resample(const double *tmpl, int32_t m, int64_t d, double *s)
{
    for (int64_t k = 0; k < d; ++k) {
        double u = ((double)k + 0.5) * (double)m / (double)d - 0.5;
        double fl = floor(u);
        int64_t m0 = (int64_t)fl;
        if (m0 < 0) m0 = 0;
        if (m0 > m - 2) m0 = m - 2;
        double f = u - (double)m0;
        if (f < 0.0) f = 0.0;
        if (f > 1.0) f = 1.0;
        double a = tmpl[m0] * (1.0 - f);
        double b = tmpl[m0 + 1] * f;
        s[k] = a + b;
    }
}

/* ------------------------------------------------------------------------ */
/* Literal chi-square of one trial (P, duration, start i, depth) over ALL n
 * points (Sect. 2.3.4, chi2 = out-of-transit part + in-transit part): the
 * model is 1 - depth * s_k on the D points at sorted positions (i+k) mod n,
 * and 1 everywhere else.  perm is the phase order of that period.          */
double oracle_chi2_literal(const double *y, const double *dy, int64_t n,
                           const int32_t *perm, int64_t i, int64_t d,
                           const double *s, double depth)
{
    double *model = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t a = 0; a < n; ++a) model[a] = 1.0;
    for (int64_t k = 0; k < d; ++k) {
        int64_t pos = (i + k) % n;
        model[perm[pos]] = 1.0 - depth * s[k];
    }
    double chi2 = 0.0;
    for (int64_t a = 0; a < n; ++a) {
        double r = (y[a] - model[a]) / dy[a];
        chi2 += r * r;
    }
    free(model);
    return chi2;
}

/* ------------------------------------------------------------------------ */
/* One window (start i of the padded folded curve, Sect. 2.3.2).
 *
 * With the model m = 1 - depth * s_k inside the window and 1 outside,
 *   chi2 = chi2_0 - 2 depth c + depth^2 b,
 *   c = sum_k w (1 - y) s_k,   b = sum_k w s_k^2   (k over the window),
 * which is the paper's chi2_out + chi2_in with the edge term removed, since
 * chi2_out = chi2_0 - sum_window w (y-1)^2 (expanding the square).
 *
 * depth_mode 0 (weighted least squares): depth = c/b, clamped at 0, and the
 * improvement is dchi2 = depth * c.
 * depth_mode 1 (moving average, Sect. 2.3.3): depth = (mean deficit in the
 * window) / (mean of the ideal transit) = sum_window (1 - y) / sum_k s_k,
 * clamped at 0, and dchi2 = 2 depth c - depth^2 b.  The window deficit sum is
 * formed exactly: every 1 - y is an integer multiple of 2^-53, so the sum is
 * carried as a 128-bit integer and rounded once.                           */
typedef struct { double dchi2, depth; } window_fit;

static window_fit oracle_window(const double *r_s, const double *w_s,
                                const int64_t *u_s, int64_t n, int64_t i,
                                int64_t d, const double *s, double s1,
                                int depth_mode)
{
    double c = 0.0, b = 0.0;
    __int128 usum = 0;
    for (int64_t k = 0; k < d; ++k) {
        int64_t pos = i + k;
        if (pos >= n) pos -= n;
        c = fma(r_s[pos], s[k], c);
        double sk2 = s[k] * s[k];
        b = fma(w_s[pos], sk2, b);
        if (depth_mode == 1) usum += (__int128)u_s[pos];
    }
    window_fit f;
    if (depth_mode == 1) {
        double mean_deficit = ldexp((double)usum, -53);
        double depth = mean_deficit / s1;
        if (!(depth > 0.0)) depth = 0.0;
        f.depth = depth;
        f.dchi2 = (2.0 * depth) * c - (depth * depth) * b;
    } else {
        double depth = (c > 0.0) ? c / b : 0.0;
        f.depth = depth;
        f.dchi2 = depth * c;
    }
    return f;
}

/* ------------------------------------------------------------------------ */
/* The full search over an explicit list of periods.  Periods are
 * independent, so any subset of the grid gives the same per-period values
 * (OpenMP over periods only).  Per period the best window is the largest
 * dchi2 over durations in ascending order and starts in ascending order, the
 * first occurrence winning ties; chi2(P) = chi2_0 - dchi2 (Sect. 2.3,
 * minimum over duration and T0).                                           */
int oracle_tls_search(const double *t, const double *y, const double *dy, int64_t n,
                      const double *periods, int32_t n_periods,
                      const double *durations, int32_t n_durations,
                      const double *tmpl, int32_t n_tmpl,
                      double dt0, int envelope, double k_min, double k_max,
                      double q_cap, int depth_mode, int n_threads,
                      double *chi2_out, int32_t *best_dur, int32_t *best_start,
                      double *depth_out, double *t0_out, double *dchi2_out,
                      int64_t *n_evals_out)
{
    double chi2_0 = oracle_chi2_null(y, dy, n);
    double tmin = t[0];
    for (int64_t a = 1; a < n; ++a) if (t[a] < tmin) tmin = t[a];

    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t *u = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t a = 0; a < n; ++a) {
        w[a] = 1.0 / (dy[a] * dy[a]);
        r[a] = w[a] * (1.0 - y[a]);
        u[a] = (int64_t)((1.0 - y[a]) * TWO_POW_53);
    }
    int64_t total_evals = 0;

#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1) reduction(+ : total_evals)
    for (int32_t pn = 0; pn < n_periods; ++pn) {
        double period = periods[pn];
        int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        double *r_s = (double *)malloc(sizeof(double) * (size_t)n);
        double *w_s = (double *)malloc(sizeof(double) * (size_t)n);
        int64_t *u_s = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        double *s = (double *)malloc(sizeof(double) * (size_t)n);
        oracle_fold_sort(t, n, period, perm);
        for (int64_t k = 0; k < n; ++k) {
            r_s[k] = r[perm[k]];
            w_s[k] = w[perm[k]];
            u_s[k] = u[perm[k]];
        }
        double best = -INFINITY, best_depth = 0.0;
        int32_t bj = -1;
        int64_t bi = -1, bd = 0;
        for (int32_t j = 0; j < n_durations; ++j) {
            if (!oracle_duration_valid(period, durations[j], envelope, k_min, k_max, q_cap))
                continue;
            int64_t d = oracle_points_in_duration(n, period, durations[j]);
            oracle_resample(tmpl, n_tmpl, d, s);
            double s1 = 0.0;
            for (int64_t k = 0; k < d; ++k) s1 += s[k];
            int64_t stride = oracle_t0_stride(d, dt0);
            for (int64_t i = 0; i < n; i += stride) {
                window_fit f = oracle_window(r_s, w_s, u_s, n, i, d, s, s1, depth_mode);
                total_evals += 1;
                if (f.dchi2 > best) {
                    best = f.dchi2;
                    best_depth = f.depth;
                    bj = j;
                    bi = i;
                    bd = d;
                }
            }
        }
        if (bj < 0) {
            chi2_out[pn] = chi2_0;
            best_dur[pn] = -1;
            best_start[pn] = -1;
            depth_out[pn] = 0.0;
            t0_out[pn] = NAN;
            dchi2_out[pn] = 0.0;
        } else {
            chi2_out[pn] = chi2_0 - best;
            best_dur[pn] = bj;
            best_start[pn] = (int32_t)bi;
            depth_out[pn] = best_depth;
            dchi2_out[pn] = best;
            /* Mid-transit: the phase of the window's middle point, moved to
             * the first such epoch at or after the earliest time.          */
            int64_t mid = (bi + bd / 2) % n;
            double phic = oracle_phase(t[perm[mid]], period);
            double a = phic * period;
            t0_out[pn] = a + period * ceil((tmin - a) / period);
        }
        free(perm); free(r_s); free(w_s); free(u_s); free(s);
    }
    free(r); free(w); free(u);
    if (n_evals_out) *n_evals_out = total_evals;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Periodogram statistics (Sect. 2.4).
 *   SR(P)  = chi2_min / chi2(P)           (in (0, 1]; 1 at the best period)
 *   SDE_raw = (SR - <SR>) / sigma_SR      (population standard deviation)
 *   SDE    = SDE_raw - running median of SDE_raw over `window` points, the
 *            series edges extended with their end values.
 * The best period is the first index of the largest SDE.                   */
static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

int oracle_sde(const double *chi2, int32_t n, int32_t window,
               double *sr, double *sde_raw, double *sde, int32_t *best)
{
    double mn = chi2[0];
    for (int32_t a = 1; a < n; ++a) if (chi2[a] < mn) mn = chi2[a];
    for (int32_t a = 0; a < n; ++a)
        sr[a] = (chi2[a] == 0.0) ? 1.0 : mn / chi2[a];
    double sum = 0.0;
    for (int32_t a = 0; a < n; ++a) sum += sr[a];
    double mean = sum / (double)n;
    double var = 0.0;
    for (int32_t a = 0; a < n; ++a) {
        double d = sr[a] - mean;
        var += d * d;
    }
    double sd = sqrt(var / (double)n);
    for (int32_t a = 0; a < n; ++a)
        sde_raw[a] = (sd > 0.0) ? (sr[a] - mean) / sd : 0.0;
    int32_t half = window / 2;
    double *buf = (double *)malloc(sizeof(double) * (size_t)window);
    for (int32_t a = 0; a < n; ++a) {
        for (int32_t k = -half; k <= half; ++k) {
            int32_t idx = a + k;
            if (idx < 0) idx = 0;
            if (idx > n - 1) idx = n - 1;
            buf[k + half] = sde_raw[idx];
        }
        qsort(buf, (size_t)window, sizeof(double), cmp_double);
        sde[a] = sde_raw[a] - buf[half];
    }
    free(buf);
    int32_t b = 0;
    for (int32_t a = 1; a < n; ++a) if (sde[a] > sde[b]) b = a;
    *best = b;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Transit statistics at one window: the SNR and the per-transit and
 * odd/even depths the paper names (Sect. 1 and 2.5, SDE and SNR thresholds
 * of Sect. 3) without giving formulas; the reading is:
 *   - the window is the search's: padded positions start .. start + d - 1 of
 *     the curve folded at `period`, sorted position p mod n, "wrapped" when
 *     p >= n (the padding repeats the start of the folded curve);
 *   - window point k, input index idx, belongs to the transit of epoch
 *     e_k = floor(t_idx / period) - wrapped;
 *   - per epoch, over its points in ascending k, c_e = sum fma(r, s_k, .)
 *     and b_e = sum fma(w, s_k^2, .) with w = 1/dy^2, r = w (1 - y) and s the
 *     d-point template; depth_e = c_e / b_e, sigma_e = 1 / sqrt(b_e);
 *   - odd epochs, even epochs and all epochs pool c and b in ascending epoch
 *     order into the same depth and sigma; the odd/even mismatch is
 *     |depth_odd - depth_even| / sqrt(sigma_odd^2 + sigma_even^2);
 *   - SNR = max(C, 0) / sqrt(B) over all epochs: the fitted depth over its
 *     standard error, which is sqrt(chi2_0 - chi2) of the weighted
 *     least-squares fit of the window (Sect. 2.3.4);
 *   - the mid-transit time of epoch e is (e + phase_mid) period, phase_mid
 *     the phase of the window's middle point (position start + floor(d/2)),
 *     plus 1 when that position is wrapped.
 * stats[8] = snr, depth, depth_odd, depth_even, sigma_odd, sigma_even,
 * odd_even_sigma, phase_mid (NaN where a side has no transit);
 * ints[3] = points in the window, transits (epochs with points), first
 * epoch.  The per-transit arrays receive the epochs with points in
 * ascending order, at most max_transits of them.  Returns 1 when more
 * transits exist than max_transits, else 0.                              */
int oracle_transit_stats(const double *t, const double *y, const double *dy, int64_t n,
                         double period, int64_t d, int64_t start,
                         const double *tmpl, int32_t n_tmpl, double *stats, int64_t *ints,
                         int64_t max_transits, int64_t *epoch, double *t_mid, double *depth,
                         double *sigma, int64_t *count)
{
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *s = (double *)malloc(sizeof(double) * (size_t)d);
    int64_t *ek = (int64_t *)malloc(sizeof(int64_t) * (size_t)d);
    oracle_fold_sort(t, n, period, perm);
    oracle_resample(tmpl, n_tmpl, d, s);
    int64_t emin = 0, emax = 0;
    for (int64_t k = 0; k < d; ++k) {
        int64_t p = start + k;
        int wrapped = p >= n;
        int32_t idx = perm[wrapped ? p - n : p];
        ek[k] = (int64_t)floor(t[idx] / period) - wrapped;
        if (k == 0 || ek[k] < emin) emin = ek[k];
        if (k == 0 || ek[k] > emax) emax = ek[k];
    }
    int64_t nep = emax - emin + 1;
    double *ce = (double *)calloc((size_t)nep, sizeof(double));
    double *be = (double *)calloc((size_t)nep, sizeof(double));
    int64_t *ne = (int64_t *)calloc((size_t)nep, sizeof(int64_t));
    for (int64_t k = 0; k < d; ++k) {
        int64_t p = start + k;
        int32_t idx = perm[p >= n ? p - n : p];
        double w = 1.0 / (dy[idx] * dy[idx]);
        double r = w * (1.0 - y[idx]);
        int64_t j = ek[k] - emin;
        ce[j] = fma(r, s[k], ce[j]);
        double sk2 = s[k] * s[k];
        be[j] = fma(w, sk2, be[j]);
        ne[j] += 1;
    }
    int64_t pm = start + d / 2;
    double phase_mid = oracle_phase(t[perm[pm >= n ? pm - n : pm]], period) + (pm >= n ? 1.0 : 0.0);
    double c_all = 0.0, b_all = 0.0, c_odd = 0.0, b_odd = 0.0, c_even = 0.0, b_even = 0.0;
    int64_t nt = 0;
    for (int64_t j = 0; j < nep; ++j) {
        if (ne[j] == 0) continue;
        int64_t e = emin + j;
        if (nt < max_transits) {
            epoch[nt] = e;
            t_mid[nt] = ((double)e + phase_mid) * period;
            depth[nt] = ce[j] / be[j];
            sigma[nt] = 1.0 / sqrt(be[j]);
            count[nt] = ne[j];
        }
        ++nt;
        c_all += ce[j];
        b_all += be[j];
        if (((e % 2) + 2) % 2 == 1) {
            c_odd += ce[j];
            b_odd += be[j];
        } else {
            c_even += ce[j];
            b_even += be[j];
        }
    }
    double d_odd = b_odd > 0.0 ? c_odd / b_odd : NAN, s_odd = b_odd > 0.0 ? 1.0 / sqrt(b_odd) : NAN;
    double d_even = b_even > 0.0 ? c_even / b_even : NAN, s_even = b_even > 0.0 ? 1.0 / sqrt(b_even) : NAN;
    stats[0] = (c_all > 0.0 ? c_all : 0.0) / sqrt(b_all);
    stats[1] = c_all / b_all;
    stats[2] = d_odd;
    stats[3] = d_even;
    stats[4] = s_odd;
    stats[5] = s_even;
    stats[6] = (b_odd > 0.0 && b_even > 0.0) ? fabs(d_odd - d_even) / sqrt(s_odd * s_odd + s_even * s_even) : NAN;
    stats[7] = phase_mid;
    ints[0] = d;
    ints[1] = nt;
    ints[2] = nt > 0 ? emin : 0;
    for (int64_t j = 0; j < nep; ++j) if (ne[j] > 0) { ints[2] = emin + j; break; }
    free(perm); free(s); free(ek); free(ce); free(be); free(ne);
    return nt > max_transits ? 1 : 0;
}
