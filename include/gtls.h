/*
 * gtls.h -- C ABI of the MI355X (gfx950) Transit Least Squares search.
 *
 * The library implements the search the GTLS paper (Hu, Ge, Jin, Willis,
 * "GTLS: A GPU-accelerated method for periodic transit detection") builds
 * its GPU pipeline around: for every trial period, fold the light curve and
 * sort it by phase (Sect. 2.3.1), pad it cyclically (Sect. 2.3.2), slide a
 * limb-darkened transit template of every trial duration over it, fit a depth
 * and a chi-square per window (Sect. 2.3.3-2.3.4), keep the minimum over
 * duration and T0, and turn chi2(P) into the SDE periodogram (Sect. 2.4).
 *
 * Conventions shared by every call:
 *   - All sizes are explicit.  Arrays are contiguous, C order, FP64 unless
 *     stated.  Days are the time unit of times, periods and durations.
 *   - Ownership: the caller owns every input and output buffer; the library
 *     never frees them and keeps no pointer after a call returns.  A context
 *     owns its device scratch (grown on demand, freed by gtls_destroy).
 *   - Host-pointer calls are synchronous.  *_dev calls take device pointers,
 *     enqueue work on the context's stream and return; results are valid
 *     after gtls_sync (or any later synchronisation of that stream).
 *   - Errors: a negative gtls_status; gtls_last_error(ctx) then holds a
 *     message.  On error the contents of outputs are unspecified, except that
 *     tls_search sets out->best_period to -1.
 *   - A context is not thread-safe: use one context per host thread.
 */
#ifndef GTLS_H
#define GTLS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GTLS_OK = 0,
    GTLS_EINVAL = -1,    /* an argument failed validation                 */
    GTLS_ENOMEM = -2,    /* device or host allocation failed              */
    GTLS_EDEVICE = -3,   /* no usable gfx950 device, or a HIP call failed */
    GTLS_EINTERNAL = -4  /* a kernel left a result unfilled               */
} gtls_status;

/* Arithmetic of the flux path.  Time and phase are FP64 in both. */
enum { GTLS_FP64 = 0, GTLS_FP32C = 1 };

/* Depth rule per window.
 * WLS: weighted least-squares depth c/b (clamped at 0).
 * MEAN: the moving-average depth of Sect. 2.3.3, taken as the window's mean
 *       deficit over the template's mean (clamped at 0), from prefix sums. */
enum { GTLS_DEPTH_WLS = 0, GTLS_DEPTH_MEAN = 1 };

typedef struct gtls_ctx gtls_ctx;

typedef struct {
    double dt0;            /* T0 step as a fraction of the transit's points
                              (Sect. 2.5, N_skip = n_IT * dt0, floored, >= 1);
                              0 evaluates every offset                        */
    int32_t envelope;      /* 1: k_min P^(-2/3) <= T14/P <= k_max P^(-2/3),
                              P in seconds (Sect. 2.2.2); 0: only q_cap      */
    double k_min, k_max;   /* s^(2/3); defaults 20.05 and 620.84              */
    double q_cap;          /* T14/P upper cap, default 0.15, always applied   */
    int32_t depth_mode;    /* GTLS_DEPTH_WLS (default) or GTLS_DEPTH_MEAN      */
    int32_t precision;     /* GTLS_FP64 (default) or GTLS_FP32C                */
    int32_t median_window; /* odd running-median width of the SDE detrend, 91 */
    int32_t batch_route_min; /* batched calls only: curves of at least this many
                              points are searched one after the other by the
                              single-curve kernels instead of the persistent
                              launch (identical results); default 3000, where
                              the two take about the same time; 0: every curve
                              in the persistent launch                        */
} gtls_params;

/* Per-period outputs (arrays of n_periods, caller-owned) and summaries.
 *   chi2[n]       minimum chi-square over durations and T0 at period n
 *   best_dur[n]   index into duration_grid of that minimum, -1 if no duration
 *                 passes the envelope at this period
 *   best_start[n] window start as an index into the phase-sorted order of
 *                 this period (the padded curve, Sect. 2.3.2), -1 if none
 *   depth[n]      fitted depth of that window (fraction of unit flux)
 *   t0[n]         mid-transit: the phase of the window's middle point,
 *                 moved to the first epoch at or after min(time); NaN if none
 *   sr, sde_raw, sde [n]  signal residue chi2_min/chi2, its standardised
 *                 form, and that minus its running median (Sect. 2.4)
 *   chi2_null     sum of w (y - 1)^2, the flat-model chi-square
 *   best_period   first index of the largest SDE
 *   sde_max       SDE at best_period
 *   n_evals       number of (period, duration, T0) windows evaluated
 *   n_macs        template multiply-adds of those windows (sum of D)
 * Any array pointer may be NULL to skip that output (host calls only). */
typedef struct {
    double *chi2;
    int32_t *best_dur;
    int32_t *best_start;
    double *depth;
    double *t0;
    double *sr;
    double *sde_raw;
    double *sde;
    double chi2_null;
    int32_t best_period;
    double sde_max;
    int64_t n_evals;
    int64_t n_macs;
} gtls_result;

/* Scalar summary written to device memory by tls_search_dev. */
typedef struct {
    double chi2_null;
    double sde_max;
    int64_t n_evals;
    int64_t n_macs;
    int32_t best_period;
    int32_t pad_;
} gtls_summary;

/* Per-stage kernel timing, accumulated while profiling is on.  Stages:
 * 0 per-point preparation and chi2_0, 1 fold + sort + padding, 2 template
 * slide on every T0 offset (stride 1) and the task list of strided T0
 * grids, 3 per-period reduction, 4 periodogram statistics, 5 template slide
 * on strided T0 grids. */
#define GTLS_N_STAGES 6
typedef struct {
    double ms[8];          /* summed kernel time per stage (HIP events on the
                              context's stream, bracketing each launch)    */
    int64_t launches[8];   /* kernel launches per stage                    */
} gtls_profile;

/* Create a context on HIP device `device`.  hip_stream is a hipStream_t to
 * run on, or NULL for a stream the context creates.  Returns GTLS_EDEVICE
 * when no gfx950 device is visible.  *ctx is NULL on failure. */
gtls_status gtls_create(gtls_ctx **ctx, int device, void *hip_stream);

/* Release a context and its device scratch.  NULL is a no-op. */
void gtls_destroy(gtls_ctx *ctx);

/* Message of the last failed call on ctx (or of the last failed
 * gtls_create when ctx is NULL).  Valid until the next call on ctx. */
const char *gtls_last_error(const gtls_ctx *ctx);

/* Turn per-stage timing on (1) or off (0); turning it on clears the
 * counters.  Timing adds two event records per launch on the stream. */
gtls_status gtls_profile_enable(gtls_ctx *ctx, int on);

/* Wait for the stream and return the accumulated per-stage timing. */
gtls_status gtls_profile_read(gtls_ctx *ctx, gtls_profile *out);

/* Fill p with the defaults listed in gtls_params. */
void gtls_params_default(gtls_params *p);

/* Wait for all work enqueued on the context's stream. */
gtls_status gtls_sync(gtls_ctx *ctx);

/* The whole search on host arrays (Sect. 2.3-2.4).
 *   time, flux, dy [n]: one light curve; time need not be sorted, dy > 0,
 *     everything finite, |1 - flux| < 1024, 3 <= n <= 2^27.
 *   period_grid [n_periods]: strictly increasing, > 0 (days).
 *   duration_grid [n_durations]: > 0, non-decreasing (days).
 *   tmpl [n_tmpl]: unit-depth transit samples at x_m = (m + 1/2)/n_tmpl,
 *     values in (0, 1], maximum exactly 1, n_tmpl >= 2.
 *   params: NULL for defaults.
 * Writes the outputs of gtls_result.  Synchronous. */
gtls_status tls_search(gtls_ctx *ctx, const double *time, const double *flux,
                       const double *dy, int64_t n, const double *period_grid,
                       int32_t n_periods, const double *duration_grid,
                       int32_t n_durations, const double *tmpl, int32_t n_tmpl,
                       const gtls_params *params, gtls_result *out);

/* Same search on device arrays, enqueued on the context's stream.
 * Inputs are device pointers of the sizes above; the seven per-period
 * outputs (chi2, best_dur, best_start, depth, t0, sde_raw, sde) are device
 * arrays of n_periods and must all be non-NULL (sr may be NULL); summary is a
 * device pointer.  Validation reads only sizes and params (device data is not
 * inspected); invalid device data gives unspecified results.  The call waits
 * once for the stream, after the per-curve preparation (whether the weights
 * are constant picks the kernels), then enqueues the rest and returns. */
gtls_status tls_search_dev(gtls_ctx *ctx, const double *time, const double *flux,
                           const double *dy, int64_t n, const double *period_grid,
                           int32_t n_periods, const double *duration_grid,
                           int32_t n_durations, const double *tmpl, int32_t n_tmpl,
                           const gtls_params *params, double *chi2, int32_t *best_dur,
                           int32_t *best_start, double *depth, double *t0, double *sr,
                           double *sde_raw, double *sde, gtls_summary *summary);

/* tls_search_dev without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Arguments, outputs and results are those of
 * tls_search_dev.  Every scratch region (per-point arrays, template rows,
 * the sort and padding of each launch's periods, the SR array when sr is
 * NULL) comes from one static device array of 256 MiB that the library holds
 * on each GPU it runs on until the process ends; no hipMalloc, hipFree or
 * allocating library routine is called.  Limit: the per-curve arrays
 * (24 B per point), the template rows for every D up to q_cap n (about
 * 4 (q_cap n)^2 bytes in FP64, half in FP32C) and at least one period's sort
 * and padding (about 24 B per point) must fit in the 256 MiB, i.e. curves of
 * up to about 50,000 points at q_cap = 0.15 in FP64; larger calls return
 * GTLS_ENOMEM and leave the outputs unwritten.  Profiling must be off
 * (GTLS_EINVAL).
 * All calls on one GPU share its array: calls that overlap in time on one
 * GPU (several host threads, or several streams without ordering) race and
 * give undefined results; calls ordered on one stream are safe. */
gtls_status tls_search_dev_noalloc(gtls_ctx *ctx, const double *time, const double *flux,
                                   const double *dy, int64_t n, const double *period_grid,
                                   int32_t n_periods, const double *duration_grid,
                                   int32_t n_durations, const double *tmpl, int32_t n_tmpl,
                                   const gtls_params *params, double *chi2, int32_t *best_dur,
                                   int32_t *best_start, double *depth, double *t0, double *sr,
                                   double *sde_raw, double *sde, gtls_summary *summary);

/* Batched survey: many light curves searched in one persistent launch over
 * (curve, period) work items (Sect. 2.3-2.4 per curve); with
 * params->batch_route_min > 0 (default 3000), curves of at least that many
 * points are searched one after the other by the single-curve kernels
 * instead (faster for long curves; identical results).
 *   offsets [n_curves + 1], host: curve c owns points
 *     [offsets[c], offsets[c + 1]) of time/flux/dy; offsets[0] = 0, each
 *     curve has 3 <= n_c <= 2^27 points (same rules as tls_search).
 *   period_offsets [n_curves + 1], host: curve c's grid is
 *     periods[period_offsets[c] .. period_offsets[c + 1]), at least one
 *     period, strictly increasing; period_offsets[0] = 0.
 *   duration_grid, tmpl, params: shared by all curves.
 * Per-period outputs use the same CSR layout as periods (length
 * period_offsets[n_curves]); best_period in summaries[c] indexes curve c's
 * grid.  Each curve's results equal those of tls_search on that curve.
 * Host arrays; any per-period output may be NULL; summaries may be NULL.
 * Synchronous. */
gtls_status tls_search_batch(gtls_ctx *ctx, const int64_t *offsets, const double *time,
                             const double *flux, const double *dy, int32_t n_curves,
                             const int64_t *period_offsets, const double *periods,
                             const double *duration_grid, int32_t n_durations,
                             const double *tmpl, int32_t n_tmpl, const gtls_params *params,
                             double *chi2, int32_t *best_dur, int32_t *best_start, double *depth,
                             double *t0, double *sde, gtls_summary *summaries);

/* tls_search_batch on device arrays: offsets and period_offsets stay host
 * arrays; every other array is a device pointer and all outputs (chi2,
 * best_dur, best_start, depth, t0, sr, sde_raw, sde, summaries) must be
 * non-NULL.  The kernels after the per-curve preparation run as one captured
 * HIP graph that is replayed while the arguments stay the same.  Returns
 * after enqueueing (call gtls_sync); each curve routed to the single-curve
 * kernels (batch_route_min) waits once for the stream, as tls_search_dev
 * does. */
gtls_status tls_search_batch_dev(gtls_ctx *ctx, const int64_t *offsets, const double *time,
                                 const double *flux, const double *dy, int32_t n_curves,
                                 const int64_t *period_offsets, const double *periods,
                                 const double *duration_grid, int32_t n_durations,
                                 const double *tmpl, int32_t n_tmpl, const gtls_params *params,
                                 double *chi2, int32_t *best_dur, int32_t *best_start,
                                 double *depth, double *t0, double *sr, double *sde_raw,
                                 double *sde, gtls_summary *summaries);

/* Fold and phase-sort only (Sect. 2.3.1): perm[k * n + i] is the input index
 * of the i-th point in phase order at periods[k]; ties in phase keep input
 * order.  Host arrays; perm has n_periods * n entries. */
gtls_status tls_fold_sort(gtls_ctx *ctx, const double *time, int64_t n,
                          const double *periods, int32_t n_periods, int32_t *perm);

/* Statistics of one transit window: the SNR and the per-transit and
 * odd/even depths that Sect. 1, 2.5 and 3 name without formulas.  The window
 * is the search's: the duration's D points (D from the period and duration
 * as in the search) from sorted position `start` of the curve folded at
 * `period`, sorted position p mod n, "wrapped" when p >= n.  Window point k
 * (input index i) belongs to the transit of epoch floor(t_i / period) - 1
 * if wrapped, else floor(t_i / period).  Per transit, over its points in
 * ascending k, c = sum w (1 - y) s_k and b = sum w s_k^2 (w = 1/dy^2, s the
 * D-point template, fused multiply-adds); depth = c / b, sigma = 1/sqrt(b).
 * Odd epochs, even epochs and all epochs pool c and b (C, B) in ascending
 * epoch order.  Reading: SNR = max(C, 0) / sqrt(B), the pooled depth over
 * its standard error, i.e. sqrt(chi2_0 - chi2) of the window's weighted
 * least-squares fit; the mid-transit time of epoch e is (e + phase_mid) *
 * period.  Values are FP64 whatever params would say. */
typedef struct {
    double snr;            /* max(C, 0) / sqrt(B)                                    */
    double depth;          /* C / B, all transits (not clamped)                      */
    double depth_odd;      /* pooled over odd epochs; NaN when there is none         */
    double depth_even;     /* pooled over even epochs; NaN when there is none        */
    double sigma_odd;      /* 1/sqrt(B_odd); NaN when there is none                  */
    double sigma_even;     /* 1/sqrt(B_even); NaN when there is none                 */
    double odd_even_sigma; /* |depth_odd - depth_even| / sqrt(sigma_odd^2 + sigma_even^2); NaN if a side is empty */
    double phase_mid;      /* phase of the window's middle point (position start + D/2), +1 if wrapped */
    int64_t n_in;          /* D, the window's points                                 */
    int64_t n_transits;    /* epochs with at least one window point                  */
    int64_t first_epoch;   /* the lowest such epoch                                  */
} gtls_transit_stats;

/* Transit statistics at one window, host arrays.
 *   time, flux, dy [n]: the light curve (rules of tls_search);
 *   period, duration: days, > 0 (typically period_grid[best] and
 *     duration_grid[best_dur] of a search); start in [0, n): the window's
 *     first sorted position (best_start of that search);
 *   tmpl [n_tmpl]: as in tls_search;
 *   stats: written on success and when the transits exceed max_transits;
 *   epoch, t_mid, depth, sigma, count [max_transits] (any may be NULL when
 *     max_transits is 0): the transits with points, ascending epoch.
 * Returns GTLS_EINVAL (with stats filled and n_transits set) when there are
 * more than max_transits transits.  Synchronous. */
gtls_status tls_transit_stats(gtls_ctx *ctx, const double *time, const double *flux,
                              const double *dy, int64_t n, double period, double duration,
                              const double *tmpl, int32_t n_tmpl, int64_t start,
                              gtls_transit_stats *stats, int64_t max_transits, int64_t *epoch,
                              double *t_mid, double *depth, double *sigma, int64_t *count);

/* Periodogram statistics alone (Sect. 2.4) on a host chi2 array of n > 0
 * values: sr, sde_raw, sde [n] (any may be NULL) and the first argmax of sde.
 * window must be odd and >= 1. */
gtls_status tls_sde(gtls_ctx *ctx, const double *chi2, int32_t n, int32_t window,
                    double *sr, double *sde_raw, double *sde, int32_t *best);

/* Two-stage search (Sect. 2.5): the whole period grid with the T0 step
 * params->dt0, then every T0 offset (dt0 = 0) on the n_refine periods with
 * the largest first-stage SDE (ties: lower index).  At those periods the
 * second-stage chi2, best duration, start, depth and T0 replace the first-
 * stage ones, and sr, sde_raw, sde, best_period and sde_max are computed
 * over the merged chi2.  n_evals / n_macs count both stages.  Arguments as
 * in tls_search; n_refine >= 0 (0: the first stage alone; more than
 * n_periods: every period); refined [n_periods] (may be NULL) receives 1 at
 * the second-stage periods, else 0.  Synchronous. */
gtls_status tls_search_refined(gtls_ctx *ctx, const double *time, const double *flux,
                               const double *dy, int64_t n, const double *period_grid,
                               int32_t n_periods, const double *duration_grid,
                               int32_t n_durations, const double *tmpl, int32_t n_tmpl,
                               const gtls_params *params, int32_t n_refine,
                               gtls_result *out, uint8_t *refined);

/* ---------------- learned period proposal ---------------- */
/* A small 1D CNN ranks log-period bins so the full search can run on the
 * periods of the top-ranked bins only (the full grid stays the fallback).
 * Input: a 4096-bin view of the light curve (per-bin median flux, minus 1,
 * over 1.4826 x the curve's median absolute deviation; empty bins 0).
 * Network: 5 x [conv1d, 32 channels, kernel 7, padding 3, GELU (erf)],
 * mean over positions, linear 32 -> 512, softmax cross-entropy.  BF16
 * operands with FP32 accumulation on the matrix cores; FP32 master weights
 * and Adam (beta 0.9/0.999, eps 1e-8).  Parameters are one flat FP32 vector:
 * W0, b0, ..., W4, b4 (W_l shaped 32 x C_in x 7), Wf (512 x 32), bf (512). */
#define GTLS_CNN_VIEW 4096
#define GTLS_CNN_BINS 512
typedef struct gtls_cnn gtls_cnn;

/* Number of parameters (45,952). */
int64_t gtls_cnn_num_params(void);

/* Create a network on ctx's device from host FP32 initial parameters
 * (gtls_cnn_num_params values; the caller chooses the random init). */
gtls_status gtls_cnn_create(gtls_ctx *ctx, const float *init_params, gtls_cnn **net);

/* Release a network.  NULL is a no-op. */
void gtls_cnn_destroy(gtls_cnn *net);

/* Views of n_curves curves in CSR layout (offsets [n_curves + 1], host):
 * time non-decreasing within each curve, at least one point each.  Writes
 * views [n_curves][4096] (host).  Synchronous. */
gtls_status gtls_cnn_view(gtls_ctx *ctx, const int64_t *offsets, const double *time,
                          const double *flux, int32_t n_curves, float *views);

/* logits [B][512] for views [B][4096] (host arrays).  Synchronous. */
gtls_status gtls_cnn_forward(gtls_cnn *net, const float *views, int32_t B, float *logits);

/* Mean cross-entropy of the batch against labels [B] (bins 0..511) and its
 * gradient (flat like the parameters; grads may be NULL).  No update. */
gtls_status gtls_cnn_gradients(gtls_cnn *net, const float *views, const int32_t *labels,
                               int32_t B, float *loss, float *grads);

/* One Adam step at learning rate lr on the batch; *loss is its mean loss. */
gtls_status gtls_cnn_train_step(gtls_cnn *net, const float *views, const int32_t *labels,
                                int32_t B, float lr, float *loss);

/* Copy the FP32 master parameters to host. */
gtls_status gtls_cnn_get_params(gtls_cnn *net, float *params);

/* The k highest-scoring bins per view, best first (ties: lower bin):
 * bins [B][k], 1 <= k <= 512. */
gtls_status gtls_cnn_topk(gtls_cnn *net, const float *views, int32_t B, int32_t k, int32_t *bins);

/* Save the network (FP32 parameters, Adam moments and step count) to a file
 * at path, or load such a file into net (same architecture; the loaded
 * network continues training exactly where the saved one stopped).
 * GTLS_EINVAL when the file cannot be written or read, or is not a
 * checkpoint of this network. */
gtls_status gtls_cnn_save(gtls_cnn *net, const char *path);
gtls_status gtls_cnn_load(gtls_cnn *net, const char *path);

/* Search pruned by the learned proposal: the curve's view, the network's k
 * best of 512 geometric log-period bins over [bin_pmin, bin_pmax] (a period
 * outside the range counts in the first or last bin), then tls_search on the
 * grid periods inside those bins.  When that subset is empty or its
 * periodogram peaks below accept_sde, the whole grid is searched instead
 * (the fallback, which also gives the full-grid result).
 *   Arguments as tls_search (host arrays; time non-decreasing, as the view
 *   needs), net from gtls_cnn_create on the same context, 1 <= k <= 512.
 *   out: the per-period arrays over the whole grid; periods not searched get
 *   chi2 NaN, best_dur and best_start -1, depth 0, t0, sr, sde_raw and sde
 *   NaN.  SR and SDE are those of the searched set, best_period indexes the
 *   whole grid, n_evals and n_macs count every search made.
 *   searched [n_periods] (may be NULL): 1 where a period was searched.
 *   fell_back (may be NULL): 1 when the whole grid was searched.
 * Synchronous. */
gtls_status tls_search_pruned(gtls_ctx *ctx, gtls_cnn *net, const double *time, const double *flux,
                              const double *dy, int64_t n, const double *period_grid,
                              int32_t n_periods, const double *duration_grid, int32_t n_durations,
                              const double *tmpl, int32_t n_tmpl, const gtls_params *params,
                              double bin_pmin, double bin_pmax, int32_t k, double accept_sde,
                              gtls_result *out, uint8_t *searched, int32_t *fell_back);

/* ---------------- host-side helpers (no device needed) ---------------- */

/* Cubic frequency grid of Sect. 2.2.1 as ascending periods in days.
 * baseline_days S > 0, os > 0, stellar mass/radius in solar units.
 * pmin_days = 0 uses the Roche limit f_max; pmax_days = 0 uses S/2.
 * Writes at most cap periods; *n_out is the full count (call with cap = 0
 * to size).  GTLS_EINVAL if cap is non-zero and too small. */
gtls_status gtls_period_grid_ofir(double baseline_days, double os, double m_sun,
                                  double r_sun, double pmin_days, double pmax_days,
                                  double *out, int32_t cap, int32_t *n_out);

/* n log-spaced durations (days) between the envelope extremes over
 * [pmin_days, pmax_days] (Sect. 2.2.2). */
gtls_status gtls_duration_grid(double pmin_days, double pmax_days, int32_t n,
                               double k_min, double k_max, double q_cap, double *out);

/* m samples of a unit-depth quadratic-limb-darkened transit (u1, u2), planet
 * radius p (stellar radii), impact parameter b, at x = (k + 1/2)/m of the
 * T1-T4 chord; the largest sample is exactly 1. */
gtls_status gtls_template_quadratic(double u1, double u2, double p, double b,
                                    int32_t m, double *out);

#ifdef __cplusplus
}
#endif

#endif /* GTLS_H */
