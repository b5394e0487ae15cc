// C ABI of the search: argument validation, contexts, and the host-pointer
// wrappers around the device pipeline in kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "gtls_impl.hpp"

namespace {

thread_local std::string g_create_error;

gtls_status fail(gtls_ctx* ctx, gtls_status code, const std::string& msg) {
    if (ctx) ctx->err = msg;
    else g_create_error = msg;
    return code;
}

gtls_status hip_fail(gtls_ctx* ctx, hipError_t e, const char* where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(ctx, e == hipErrorOutOfMemory ? GTLS_ENOMEM : GTLS_EDEVICE, m);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

gtls_status check_params(gtls_ctx* ctx, const gtls_params& p) {
    if (!(p.dt0 >= 0.0) || !std::isfinite(p.dt0)) return fail(ctx, GTLS_EINVAL, "dt0 must be finite and >= 0");
    if (!(p.q_cap > 0.0) || !(p.q_cap <= 1.0)) return fail(ctx, GTLS_EINVAL, "q_cap must be in (0, 1]");
    if (p.envelope != 0 && p.envelope != 1) return fail(ctx, GTLS_EINVAL, "envelope must be 0 or 1");
    if (p.envelope && (!(p.k_min > 0.0) || !(p.k_max >= p.k_min) || !std::isfinite(p.k_max)))
        return fail(ctx, GTLS_EINVAL, "envelope needs 0 < k_min <= k_max");
    if (p.depth_mode != GTLS_DEPTH_WLS && p.depth_mode != GTLS_DEPTH_MEAN)
        return fail(ctx, GTLS_EINVAL, "unknown depth_mode");
    if (p.precision != GTLS_FP64 && p.precision != GTLS_FP32C) return fail(ctx, GTLS_EINVAL, "unknown precision");
    if (p.median_window < 1 || p.median_window > 1023 || (p.median_window % 2) == 0)
        return fail(ctx, GTLS_EINVAL, "median_window must be odd and in [1, 1023]");
    if (p.batch_route_min < 0) return fail(ctx, GTLS_EINVAL, "batch_route_min must be >= 0");
    return GTLS_OK;
}

gtls_status check_sizes(gtls_ctx* ctx, int64_t n, int32_t np, int32_t nd, int32_t nt) {
    // the strided slide addresses a padded curve (at most 2 n + 1088 points) with 32-bit byte offsets
    if (n < 3 || n > (1 << 27)) return fail(ctx, GTLS_EINVAL, "n must be in [3, 2^27]");
    if (np < 1) return fail(ctx, GTLS_EINVAL, "n_periods must be >= 1");
    if (nd < 1) return fail(ctx, GTLS_EINVAL, "n_durations must be >= 1");
    if (nt < 2) return fail(ctx, GTLS_EINVAL, "n_tmpl must be >= 2");
    return GTLS_OK;
}

gtls_status check_host_data(gtls_ctx* ctx, const double* t, const double* y, const double* dy, int64_t n,
                            const double* per, int32_t np, const double* dur, int32_t nd, const double* tm,
                            int32_t nt) {
    if (!t || !y || !dy || !per || !dur || !tm) return fail(ctx, GTLS_EINVAL, "null input array");
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(t[i]) || !std::isfinite(y[i])) return fail(ctx, GTLS_EINVAL, "non-finite time or flux");
        if (!(std::fabs(1.0 - y[i]) < 1024.0)) return fail(ctx, GTLS_EINVAL, "flux must satisfy |1 - y| < 1024");
        if (!(dy[i] > 0.0) || !std::isfinite(dy[i])) return fail(ctx, GTLS_EINVAL, "dy must be finite and > 0");
        if (!(1.0 / (dy[i] * dy[i]) < 1e300)) return fail(ctx, GTLS_EINVAL, "dy too small");
    }
    for (int32_t k = 0; k < np; ++k) {
        if (!(per[k] > 0.0) || !std::isfinite(per[k])) return fail(ctx, GTLS_EINVAL, "periods must be finite and > 0");
        if (k > 0 && !(per[k] > per[k - 1])) return fail(ctx, GTLS_EINVAL, "periods must be strictly increasing");
    }
    for (int32_t k = 0; k < nd; ++k) {
        if (!(dur[k] > 0.0) || !std::isfinite(dur[k])) return fail(ctx, GTLS_EINVAL, "durations must be finite and > 0");
        if (k > 0 && !(dur[k] >= dur[k - 1])) return fail(ctx, GTLS_EINVAL, "durations must be non-decreasing");
    }
    double mx = 0.0;
    for (int32_t k = 0; k < nt; ++k) {
        if (!(tm[k] > 0.0) || !(tm[k] <= 1.0)) return fail(ctx, GTLS_EINVAL, "template values must be in (0, 1]");
        mx = std::fmax(mx, tm[k]);
    }
    if (mx != 1.0) return fail(ctx, GTLS_EINVAL, "template maximum must be exactly 1");
    return GTLS_OK;
}

}  // namespace

extern "C" {

void gtls_params_default(gtls_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->dt0 = 0.0;
    p->envelope = 1;
    p->k_min = 20.05;
    p->k_max = 620.84;
    p->q_cap = 0.15;
    p->depth_mode = GTLS_DEPTH_WLS;
    p->precision = GTLS_FP64;
    p->median_window = 91;
    p->batch_route_min = 3000;
}

gtls_status gtls_create(gtls_ctx** out, int device, void* hip_stream) {
    if (!out) return fail(nullptr, GTLS_EINVAL, "ctx pointer is null");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) return fail(nullptr, GTLS_EDEVICE, "no HIP device visible");
    if (device < 0 || device >= count) return fail(nullptr, GTLS_EDEVICE, "device index out of range");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return fail(nullptr, GTLS_EDEVICE, hipGetErrorString(e));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, GTLS_EDEVICE, std::string("library is built for gfx950, device is ") + prop.gcnArchName);
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(nullptr, GTLS_EDEVICE, hipGetErrorString(e));
    gtls_ctx* ctx = new gtls_ctx();
    ctx->device = device;
    ctx->num_cus = prop.multiProcessorCount;     // sizes the persistent kernels
    e = gtls::static_scratch_address(device, &ctx->static_scratch);
    if (e != hipSuccess) {
        delete ctx;
        return fail(nullptr, GTLS_EDEVICE, std::string("static scratch address: ") + hipGetErrorString(e));
    }
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete ctx;
            return fail(nullptr, GTLS_EDEVICE, hipGetErrorString(e));
        }
        ctx->own_stream = true;
    }
    *out = ctx;
    return GTLS_OK;
}

void gtls_destroy(gtls_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->bcache.exec) (void)hipGraphExecDestroy(ctx->bcache.exec);
    for (gtls::DeviceBuffer* b : {&ctx->curve, &ctx->batch, &ctx->io, &ctx->sde_tmp, &ctx->table, &ctx->bcurve,
                                  &ctx->bscratch})
        if (b->ptr) (void)hipFree(b->ptr);
    for (auto& p : ctx->pending) {
        ctx->event_pool.push_back(p.start);
        ctx->event_pool.push_back(p.stop);
    }
    for (hipEvent_t ev : ctx->event_pool) (void)hipEventDestroy(ev);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

const char* gtls_last_error(const gtls_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

gtls_status gtls_profile_enable(gtls_ctx* ctx, int on) {
    if (!ctx) return GTLS_EINVAL;
    hipError_t e = gtls::profile_collect(ctx);
    if (e != hipSuccess) return hip_fail(ctx, e, "profile");
    for (int k = 0; k < 8; ++k) {
        ctx->prof_ms[k] = 0.0;
        ctx->prof_launches[k] = 0;
    }
    ctx->profiling = on != 0;
    return GTLS_OK;
}

gtls_status gtls_profile_read(gtls_ctx* ctx, gtls_profile* out) {
    if (!ctx || !out) return GTLS_EINVAL;
    hipError_t e = gtls::profile_collect(ctx);
    if (e != hipSuccess) return hip_fail(ctx, e, "profile");
    for (int k = 0; k < 8; ++k) {
        out->ms[k] = ctx->prof_ms[k];
        out->launches[k] = ctx->prof_launches[k];
    }
    return GTLS_OK;
}

gtls_status gtls_sync(gtls_ctx* ctx) {
    if (!ctx) return GTLS_EINVAL;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    return e == hipSuccess ? GTLS_OK : hip_fail(ctx, e, "stream synchronize");
}

gtls_status tls_search_dev(gtls_ctx* ctx, const double* time, const double* flux, const double* dy, int64_t n,
                           const double* period_grid, int32_t n_periods, const double* duration_grid,
                           int32_t n_durations, const double* tmpl, int32_t n_tmpl, const gtls_params* params,
                           double* chi2, int32_t* best_dur, int32_t* best_start, double* depth, double* t0,
                           double* sr, double* sde_raw, double* sde, gtls_summary* summary) {
    if (!ctx) return GTLS_EINVAL;
    gtls_params prm;
    if (params) prm = *params;
    else gtls_params_default(&prm);
    gtls_status st = check_sizes(ctx, n, n_periods, n_durations, n_tmpl);
    if (st != GTLS_OK) return st;
    if ((st = check_params(ctx, prm)) != GTLS_OK) return st;
    if (!time || !flux || !dy || !period_grid || !duration_grid || !tmpl || !chi2 || !best_dur || !best_start ||
        !depth || !t0 || !sde_raw || !sde || !summary)
        return fail(ctx, GTLS_EINVAL, "null device pointer");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "set device");
    // SR is needed internally; use scratch when the caller passes none.
    double* srp = sr;
    if (!srp) {
        e = gtls::ensure(ctx, ctx->sde_tmp, align256(sizeof(double) * (size_t)n_periods));
        if (e != hipSuccess) return hip_fail(ctx, e, "sde scratch");
        srp = (double*)ctx->sde_tmp.ptr;
    }
    gtls::SearchArgs a{time, flux, dy, n, period_grid, n_periods, duration_grid, n_durations, tmpl, n_tmpl, prm,
                       chi2, best_dur, best_start, depth, t0, srp, sde_raw, sde, summary};
    e = gtls::run_search(ctx, a);
    if (e != hipSuccess) return hip_fail(ctx, e, "search");
    return GTLS_OK;
}

gtls_status tls_search_dev_noalloc(gtls_ctx* ctx, const double* time, const double* flux, const double* dy, int64_t n,
                           const double* period_grid, int32_t n_periods, const double* duration_grid,
                           int32_t n_durations, const double* tmpl, int32_t n_tmpl, const gtls_params* params,
                           double* chi2, int32_t* best_dur, int32_t* best_start, double* depth, double* t0,
                           double* sr, double* sde_raw, double* sde, gtls_summary* summary) {
    if (!ctx) return GTLS_EINVAL;
    gtls_params prm;
    if (params) prm = *params;
    else gtls_params_default(&prm);
    gtls_status st = check_sizes(ctx, n, n_periods, n_durations, n_tmpl);
    if (st != GTLS_OK) return st;
    if ((st = check_params(ctx, prm)) != GTLS_OK) return st;
    if (!time || !flux || !dy || !period_grid || !duration_grid || !tmpl || !chi2 || !best_dur || !best_start ||
        !depth || !t0 || !sde_raw || !sde || !summary)
        return fail(ctx, GTLS_EINVAL, "null device pointer");
    if (ctx->profiling) return fail(ctx, GTLS_EINVAL, "profiling is on (it creates HIP events); turn it off");
    if (!ctx->static_scratch) return fail(ctx, GTLS_EDEVICE, "static scratch unavailable on this device");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "set device");
    // Every scratch region comes from the static array; SR too when the
    // caller passes none.
    char* base = ctx->static_scratch;
    size_t bytes = gtls::kStaticScratchBytes;
    double* srp = sr;
    if (!srp) {
        const size_t b = align256(sizeof(double) * (size_t)n_periods);
        if (b >= bytes) return fail(ctx, GTLS_ENOMEM, "n_periods too large for the static scratch");
        srp = (double*)base;
        base += b;
        bytes -= b;
    }
    gtls::SearchArgs a{time, flux, dy, n, period_grid, n_periods, duration_grid, n_durations, tmpl, n_tmpl, prm,
                       chi2, best_dur, best_start, depth, t0, srp, sde_raw, sde, summary, base, bytes};
    e = gtls::run_search(ctx, a);
    if (e == hipErrorOutOfMemory)
        return fail(ctx, GTLS_ENOMEM,
                    "curve too large for the static scratch of " + std::to_string(gtls::kStaticScratchBytes >> 20) +
                        " MiB (per-curve arrays, template rows up to q_cap n points and one period's sort and "
                        "padding must fit)");
    if (e != hipSuccess) return hip_fail(ctx, e, "search");
    return GTLS_OK;
}

gtls_status tls_search(gtls_ctx* ctx, const double* time, const double* flux, const double* dy, int64_t n,
                       const double* period_grid, int32_t n_periods, const double* duration_grid,
                       int32_t n_durations, const double* tmpl, int32_t n_tmpl, const gtls_params* params,
                       gtls_result* out) {
    if (!ctx) return GTLS_EINVAL;
    if (out) out->best_period = -1;
    if (!out) return fail(ctx, GTLS_EINVAL, "out is null");
    gtls_params prm;
    if (params) prm = *params;
    else gtls_params_default(&prm);
    gtls_status st = check_sizes(ctx, n, n_periods, n_durations, n_tmpl);
    if (st != GTLS_OK) return st;
    if ((st = check_params(ctx, prm)) != GTLS_OK) return st;
    st = check_host_data(ctx, time, flux, dy, n, period_grid, n_periods, duration_grid, n_durations, tmpl, n_tmpl);
    if (st != GTLS_OK) return st;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "set device");

    const size_t np = (size_t)n_periods, nn = (size_t)n;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const size_t o_t = take(8 * nn), o_y = take(8 * nn), o_dy = take(8 * nn), o_p = take(8 * np),
                 o_d = take(8 * (size_t)n_durations), o_tm = take(8 * (size_t)n_tmpl), o_chi2 = take(8 * np),
                 o_bd = take(4 * np), o_bs = take(4 * np), o_dep = take(8 * np), o_t0 = take(8 * np),
                 o_sr = take(8 * np), o_raw = take(8 * np), o_sde = take(8 * np), o_sum = take(sizeof(gtls_summary));
    e = gtls::ensure(ctx, ctx->io, o);
    if (e != hipSuccess) return hip_fail(ctx, e, "device buffers");
    char* b = (char*)ctx->io.ptr;
    hipStream_t s = ctx->stream;
    struct Up { size_t off; const void* src; size_t bytes; } ups[] = {
        {o_t, time, 8 * nn}, {o_y, flux, 8 * nn}, {o_dy, dy, 8 * nn}, {o_p, period_grid, 8 * np},
        {o_d, duration_grid, 8 * (size_t)n_durations}, {o_tm, tmpl, 8 * (size_t)n_tmpl}};
    for (const Up& u : ups) {
        e = hipMemcpyAsync(b + u.off, u.src, u.bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(ctx, e, "copy to device");
    }
    gtls::SearchArgs a{(double*)(b + o_t), (double*)(b + o_y), (double*)(b + o_dy), n, (double*)(b + o_p),
                       n_periods, (double*)(b + o_d), n_durations, (double*)(b + o_tm), n_tmpl, prm,
                       (double*)(b + o_chi2), (int32_t*)(b + o_bd), (int32_t*)(b + o_bs), (double*)(b + o_dep),
                       (double*)(b + o_t0), (double*)(b + o_sr), (double*)(b + o_raw), (double*)(b + o_sde),
                       (gtls_summary*)(b + o_sum)};
    e = gtls::run_search(ctx, a);
    if (e != hipSuccess) return hip_fail(ctx, e, "search");
    struct Down { void* dst; size_t off; size_t bytes; } downs[] = {
        {out->chi2, o_chi2, 8 * np}, {out->best_dur, o_bd, 4 * np}, {out->best_start, o_bs, 4 * np},
        {out->depth, o_dep, 8 * np}, {out->t0, o_t0, 8 * np}, {out->sr, o_sr, 8 * np},
        {out->sde_raw, o_raw, 8 * np}, {out->sde, o_sde, 8 * np}};
    for (const Down& d : downs) {
        if (!d.dst) continue;
        e = hipMemcpyAsync(d.dst, b + d.off, d.bytes, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return hip_fail(ctx, e, "copy to host");
    }
    gtls_summary sum;
    e = hipMemcpyAsync(&sum, b + o_sum, sizeof(sum), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(ctx, e, "copy to host");
    out->chi2_null = sum.chi2_null;
    out->best_period = sum.best_period;
    out->sde_max = sum.sde_max;
    out->n_evals = sum.n_evals;
    out->n_macs = sum.n_macs;
    if (sum.best_period < 0) return fail(ctx, GTLS_EINTERNAL, "no best period produced");
    return GTLS_OK;
}

static gtls_status check_batch_sizes(gtls_ctx* ctx, const int64_t* offsets, int32_t nc, const int64_t* poff,
                                     int32_t nd, int32_t nt) {
    if (!offsets || !poff) return fail(ctx, GTLS_EINVAL, "null offsets");
    if (nc < 1) return fail(ctx, GTLS_EINVAL, "n_curves must be >= 1");
    if (nd < 1 || nd > 64) return fail(ctx, GTLS_EINVAL, "batched search takes 1..64 durations");
    if (nt < 2) return fail(ctx, GTLS_EINVAL, "n_tmpl must be >= 2");
    if (offsets[0] != 0 || poff[0] != 0) return fail(ctx, GTLS_EINVAL, "offsets must start at 0");
    for (int32_t c = 0; c < nc; ++c) {
        const int64_t n = offsets[c + 1] - offsets[c];
        if (n < 3 || n > (1 << 27)) return fail(ctx, GTLS_EINVAL, "each curve needs 3 <= n <= 2^27 points");
        if (poff[c + 1] - poff[c] < 1) return fail(ctx, GTLS_EINVAL, "each curve needs at least one period");
    }
    if (poff[nc] > 0x7fffffff) return fail(ctx, GTLS_EINVAL, "too many periods in one batch");
    return GTLS_OK;
}

gtls_status tls_search_batch_dev(gtls_ctx* ctx, const int64_t* offsets, const double* time, const double* flux,
                                 const double* dy, int32_t n_curves, const int64_t* period_offsets,
                                 const double* periods, const double* duration_grid, int32_t n_durations,
                                 const double* tmpl, int32_t n_tmpl, const gtls_params* params, double* chi2,
                                 int32_t* best_dur, int32_t* best_start, double* depth, double* t0, double* sr,
                                 double* sde_raw, double* sde, gtls_summary* summaries) {
    if (!ctx) return GTLS_EINVAL;
    gtls_params prm;
    if (params) prm = *params;
    else gtls_params_default(&prm);
    gtls_status st = check_batch_sizes(ctx, offsets, n_curves, period_offsets, n_durations, n_tmpl);
    if (st != GTLS_OK) return st;
    if ((st = check_params(ctx, prm)) != GTLS_OK) return st;
    if (!time || !flux || !dy || !periods || !duration_grid || !tmpl || !chi2 || !best_dur || !best_start ||
        !depth || !t0 || !sr || !sde_raw || !sde || !summaries)
        return fail(ctx, GTLS_EINVAL, "null device pointer");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "set device");
    gtls::BatchArgsHost a{offsets, period_offsets, n_curves, time, flux, dy, periods, duration_grid, n_durations,
                          tmpl, n_tmpl, prm, chi2, best_dur, best_start, depth, t0, sr, sde_raw, sde, summaries};
    e = gtls::run_search_batch(ctx, a);
    if (e != hipSuccess) return hip_fail(ctx, e, "batched search");
    return GTLS_OK;
}

gtls_status tls_search_batch(gtls_ctx* ctx, const int64_t* offsets, const double* time, const double* flux,
                             const double* dy, int32_t n_curves, const int64_t* period_offsets, const double* periods,
                             const double* duration_grid, int32_t n_durations, const double* tmpl, int32_t n_tmpl,
                             const gtls_params* params, double* chi2, int32_t* best_dur, int32_t* best_start,
                             double* depth, double* t0, double* sde, gtls_summary* summaries) {
    if (!ctx) return GTLS_EINVAL;
    gtls_params prm;
    if (params) prm = *params;
    else gtls_params_default(&prm);
    gtls_status st = check_batch_sizes(ctx, offsets, n_curves, period_offsets, n_durations, n_tmpl);
    if (st != GTLS_OK) return st;
    if ((st = check_params(ctx, prm)) != GTLS_OK) return st;
    for (int32_t c = 0; c < n_curves; ++c) {
        const int64_t o = offsets[c], po = period_offsets[c];
        st = check_host_data(ctx, time + o, flux + o, dy + o, offsets[c + 1] - o, periods + po,
                             (int32_t)(period_offsets[c + 1] - po), duration_grid, n_durations, tmpl, n_tmpl);
        if (st != GTLS_OK) return st;
    }
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "set device");
    const size_t npts = (size_t)offsets[n_curves], np = (size_t)period_offsets[n_curves], nc = (size_t)n_curves;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const size_t o_t = take(8 * npts), o_y = take(8 * npts), o_dy = take(8 * npts), o_p = take(8 * np),
                 o_d = take(8 * (size_t)n_durations), o_tm = take(8 * (size_t)n_tmpl), o_chi2 = take(8 * np),
                 o_bd = take(4 * np), o_bs = take(4 * np), o_dep = take(8 * np), o_t0 = take(8 * np),
                 o_sr = take(8 * np), o_raw = take(8 * np), o_sde = take(8 * np),
                 o_sum = take(sizeof(gtls_summary) * nc);
    e = gtls::ensure(ctx, ctx->io, o);
    if (e != hipSuccess) return hip_fail(ctx, e, "device buffers");
    char* b = (char*)ctx->io.ptr;
    hipStream_t s = ctx->stream;
    struct Up { size_t off; const void* src; size_t bytes; } ups[] = {
        {o_t, time, 8 * npts}, {o_y, flux, 8 * npts}, {o_dy, dy, 8 * npts}, {o_p, periods, 8 * np},
        {o_d, duration_grid, 8 * (size_t)n_durations}, {o_tm, tmpl, 8 * (size_t)n_tmpl}};
    for (const Up& u : ups) {
        e = hipMemcpyAsync(b + u.off, u.src, u.bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(ctx, e, "copy to device");
    }
    gtls::BatchArgsHost a{offsets, period_offsets, n_curves, (double*)(b + o_t), (double*)(b + o_y),
                          (double*)(b + o_dy), (double*)(b + o_p), (double*)(b + o_d), n_durations,
                          (double*)(b + o_tm), n_tmpl, prm, (double*)(b + o_chi2), (int32_t*)(b + o_bd),
                          (int32_t*)(b + o_bs), (double*)(b + o_dep), (double*)(b + o_t0), (double*)(b + o_sr),
                          (double*)(b + o_raw), (double*)(b + o_sde), (gtls_summary*)(b + o_sum)};
    e = gtls::run_search_batch(ctx, a);
    if (e != hipSuccess) return hip_fail(ctx, e, "batched search");
    struct Down { void* dst; size_t off; size_t bytes; } downs[] = {
        {chi2, o_chi2, 8 * np}, {best_dur, o_bd, 4 * np}, {best_start, o_bs, 4 * np}, {depth, o_dep, 8 * np},
        {t0, o_t0, 8 * np}, {sde, o_sde, 8 * np}, {summaries, o_sum, sizeof(gtls_summary) * nc}};
    for (const Down& d : downs) {
        if (!d.dst) continue;
        e = hipMemcpyAsync(d.dst, b + d.off, d.bytes, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return hip_fail(ctx, e, "copy to host");
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(ctx, e, "copy to host");
    return GTLS_OK;
}

gtls_status tls_fold_sort(gtls_ctx* ctx, const double* time, int64_t n, const double* periods, int32_t n_periods,
                          int32_t* perm) {
    if (!ctx) return GTLS_EINVAL;
    if (!time || !periods || !perm) return fail(ctx, GTLS_EINVAL, "null argument");
    if (n < 1 || n > 0x7fffffff || n_periods < 1) return fail(ctx, GTLS_EINVAL, "bad sizes");
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(time[i])) return fail(ctx, GTLS_EINVAL, "non-finite time");
    for (int32_t k = 0; k < n_periods; ++k)
        if (!(periods[k] > 0.0) || !std::isfinite(periods[k])) return fail(ctx, GTLS_EINVAL, "bad period");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "set device");
    const size_t o_t = 0, o_p = align256(8 * (size_t)n), o_perm = align256(o_p + 8 * (size_t)n_periods),
                 total = align256(o_perm + 4 * (size_t)n * n_periods);
    e = gtls::ensure(ctx, ctx->io, total);
    if (e != hipSuccess) return hip_fail(ctx, e, "device buffers");
    char* b = (char*)ctx->io.ptr;
    hipStream_t s = ctx->stream;
    e = hipMemcpyAsync(b + o_t, time, 8 * (size_t)n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b + o_p, periods, 8 * (size_t)n_periods, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "copy to device");
    e = gtls::run_fold_sort(ctx, (double*)(b + o_t), n, (double*)(b + o_p), n_periods, (int32_t*)(b + o_perm));
    if (e != hipSuccess) return hip_fail(ctx, e, "fold sort");
    e = hipMemcpyAsync(perm, b + o_perm, 4 * (size_t)n * n_periods, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(ctx, e, "copy to host");
    return GTLS_OK;
}

gtls_status tls_transit_stats(gtls_ctx* ctx, const double* time, const double* flux, const double* dy, int64_t n,
                              double period, double duration, const double* tmpl, int32_t n_tmpl, int64_t start,
                              gtls_transit_stats* stats, int64_t max_transits, int64_t* epoch, double* t_mid,
                              double* depth, double* sigma, int64_t* count) {
    if (!ctx) return GTLS_EINVAL;
    if (!stats) return fail(ctx, GTLS_EINVAL, "null stats");
    gtls_status st = check_sizes(ctx, n, 1, 1, n_tmpl);
    if (st != GTLS_OK) return st;
    if (!(period > 0.0) || !std::isfinite(period) || !(duration > 0.0) || !std::isfinite(duration))
        return fail(ctx, GTLS_EINVAL, "period and duration must be finite and > 0");
    st = check_host_data(ctx, time, flux, dy, n, &period, 1, &duration, 1, tmpl, n_tmpl);
    if (st != GTLS_OK) return st;
    if (start < 0 || start >= n) return fail(ctx, GTLS_EINVAL, "start must be in [0, n)");
    if (max_transits < 0) return fail(ctx, GTLS_EINVAL, "max_transits must be >= 0");
    if (max_transits > 0 && (!epoch || !t_mid || !depth || !sigma || !count))
        return fail(ctx, GTLS_EINVAL, "null per-transit array");
    // window points as in the search: D = floor(n duration / period + 1/2) in [1, n]
    const double q = duration / period;
    double dd = std::floor((double)n * q + 0.5);
    const int64_t d = dd < 1.0 ? 1 : (dd > (double)n ? n : (int64_t)dd);
    // epochs lie between floor(min t / P) - 1 and floor(max t / P)
    double tmin = time[0], tmax = time[0];
    for (int64_t i = 1; i < n; ++i) {
        tmin = std::min(tmin, time[i]);
        tmax = std::max(tmax, time[i]);
    }
    const double span_epochs = std::floor(tmax / period) - std::floor(tmin / period) + 2.0;
    if (!(span_epochs < 1e8)) return fail(ctx, GTLS_EINVAL, "more than 1e8 epochs in the time span");
    const int64_t nep_max = (int64_t)span_epochs;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "set device");
    const size_t nn = (size_t)n, mt = (size_t)max_transits;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const size_t o_t = take(8 * nn), o_y = take(8 * nn), o_dy = take(8 * nn), o_tm = take(8 * (size_t)n_tmpl),
                 o_p = take(8), o_st = take(sizeof(gtls_transit_stats)), o_ep = take(8 * mt), o_tmid = take(8 * mt),
                 o_dep = take(8 * mt), o_sig = take(8 * mt), o_cnt = take(8 * mt);
    e = gtls::ensure(ctx, ctx->io, o);
    if (e != hipSuccess) return hip_fail(ctx, e, "device buffers");
    char* b = (char*)ctx->io.ptr;
    hipStream_t s = ctx->stream;
    e = hipMemcpyAsync(b + o_t, time, 8 * nn, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b + o_y, flux, 8 * nn, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b + o_dy, dy, 8 * nn, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b + o_tm, tmpl, 8 * (size_t)n_tmpl, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b + o_p, &period, 8, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "copy to device");
    e = gtls::run_transit_stats(ctx, (double*)(b + o_t), (double*)(b + o_y), (double*)(b + o_dy), n,
                                (double*)(b + o_p), d, start, (double*)(b + o_tm), n_tmpl, nep_max, max_transits,
                                (gtls_transit_stats*)(b + o_st), (int64_t*)(b + o_ep), (double*)(b + o_tmid),
                                (double*)(b + o_dep), (double*)(b + o_sig), (int64_t*)(b + o_cnt));
    if (e != hipSuccess) return hip_fail(ctx, e, "transit statistics");
    e = hipMemcpyAsync(stats, b + o_st, sizeof(gtls_transit_stats), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(ctx, e, "copy to host");
    const size_t k = (size_t)std::min<int64_t>(stats->n_transits, max_transits);
    if (k > 0) {
        e = hipMemcpyAsync(epoch, b + o_ep, 8 * k, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(t_mid, b + o_tmid, 8 * k, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(depth, b + o_dep, 8 * k, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(sigma, b + o_sig, 8 * k, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(count, b + o_cnt, 8 * k, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(ctx, e, "copy to host");
    }
    if (stats->n_transits > max_transits) return fail(ctx, GTLS_EINVAL, "more transits than max_transits");
    return GTLS_OK;
}

gtls_status tls_sde(gtls_ctx* ctx, const double* chi2, int32_t n, int32_t window, double* sr, double* sde_raw,
                    double* sde, int32_t* best) {
    if (!ctx) return GTLS_EINVAL;
    if (!chi2 || n < 1) return fail(ctx, GTLS_EINVAL, "chi2 must be a non-empty array");
    if (window < 1 || window > 1023 || window % 2 == 0) return fail(ctx, GTLS_EINVAL, "window must be odd, 1..1023");
    for (int32_t i = 0; i < n; ++i)
        if (!(chi2[i] >= 0.0) || !std::isfinite(chi2[i])) return fail(ctx, GTLS_EINVAL, "chi2 must be finite, >= 0");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "set device");
    const size_t nn = (size_t)n, o_c = 0, o_sr = align256(8 * nn), o_raw = align256(o_sr + 8 * nn),
                 o_sde = align256(o_raw + 8 * nn), o_sum = align256(o_sde + 8 * nn),
                 total = align256(o_sum + sizeof(gtls_summary));
    e = gtls::ensure(ctx, ctx->io, total);
    if (e != hipSuccess) return hip_fail(ctx, e, "device buffers");
    char* b = (char*)ctx->io.ptr;
    hipStream_t s = ctx->stream;
    e = hipMemcpyAsync(b + o_c, chi2, 8 * nn, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "copy to device");
    e = gtls::run_sde(ctx, (double*)(b + o_c), n, window, (double*)(b + o_sr), (double*)(b + o_raw),
                      (double*)(b + o_sde), (gtls_summary*)(b + o_sum));
    if (e != hipSuccess) return hip_fail(ctx, e, "sde");
    gtls_summary sum;
    struct Down { void* dst; size_t off; } downs[] = {{sr, o_sr}, {sde_raw, o_raw}, {sde, o_sde}};
    for (const Down& d : downs) {
        if (!d.dst) continue;
        e = hipMemcpyAsync(d.dst, b + d.off, 8 * nn, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return hip_fail(ctx, e, "copy to host");
    }
    e = hipMemcpyAsync(&sum, b + o_sum, sizeof(sum), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(ctx, e, "copy to host");
    if (best) *best = sum.best_period;
    return GTLS_OK;
}

gtls_status tls_search_pruned(gtls_ctx* ctx, gtls_cnn* net, const double* time, const double* flux, const double* dy,
                              int64_t n, const double* period_grid, int32_t n_periods, const double* duration_grid,
                              int32_t n_durations, const double* tmpl, int32_t n_tmpl, const gtls_params* params,
                              double bin_pmin, double bin_pmax, int32_t k, double accept_sde, gtls_result* out,
                              uint8_t* searched, int32_t* fell_back) {
    if (!ctx) return GTLS_EINVAL;
    if (out) out->best_period = -1;
    if (!out || !net) return fail(ctx, GTLS_EINVAL, "out and net must not be null");
    if (k < 1 || k > GTLS_CNN_BINS) return fail(ctx, GTLS_EINVAL, "k must be in [1, 512]");
    if (!(bin_pmin > 0.0) || !(bin_pmax > bin_pmin) || !std::isfinite(bin_pmax))
        return fail(ctx, GTLS_EINVAL, "bins need 0 < bin_pmin < bin_pmax");
    if (!std::isfinite(accept_sde)) return fail(ctx, GTLS_EINVAL, "accept_sde must be finite");
    if (n_periods < 1 || n < 3 || !time || !flux || !period_grid) return fail(ctx, GTLS_EINVAL, "empty input");
    gtls_params prm;
    if (params) prm = *params;
    else gtls_params_default(&prm);
    const size_t np = (size_t)n_periods;
    // The network's k best bins for this curve.
    std::vector<float> view(GTLS_CNN_VIEW);
    const int64_t off[2] = {0, n};
    gtls_status st = gtls_cnn_view(ctx, off, time, flux, 1, view.data());
    if (st != GTLS_OK) return st;
    std::vector<int32_t> bins((size_t)k);
    st = gtls_cnn_topk(net, view.data(), 1, k, bins.data());
    if (st != GTLS_OK) return st;
    std::vector<uint8_t> chosen(GTLS_CNN_BINS, 0);
    for (int32_t b : bins) chosen[(size_t)b] = 1;
    // Grid periods inside the chosen bins (geometric bins over [bin_pmin, bin_pmax]).
    std::vector<int32_t> idx;
    const double lr = std::log(bin_pmax / bin_pmin);
    for (size_t i = 0; i < np; ++i) {
        double b = std::floor(std::log(period_grid[i] / bin_pmin) / lr * (double)GTLS_CNN_BINS);
        b = b < 0.0 ? 0.0 : (b > GTLS_CNN_BINS - 1 ? GTLS_CNN_BINS - 1 : b);
        if (chosen[(size_t)b]) idx.push_back((int32_t)i);
    }
    std::vector<double> chi2(np, NAN), depth(np, 0.0), t0(np, NAN), sr(np, NAN), raw(np, NAN), sde(np, NAN);
    std::vector<int32_t> bd(np, -1), bs(np, -1);
    int32_t fb = 1;
    int32_t best = -1;
    double sde_max = NAN, chi2_null = 0.0;
    int64_t evals = 0, macs = 0;
    if (!idx.empty()) {
        // Search of the subset; accepted when its periodogram peaks at or above accept_sde.
        const size_t m = idx.size();
        std::vector<double> per(m), sc(m), sdp(m), st0(m), ssr(m), sraw(m), ssde(m);
        std::vector<int32_t> sbd(m), sbs(m);
        for (size_t i = 0; i < m; ++i) per[i] = period_grid[idx[i]];
        gtls_result r{};
        r.chi2 = sc.data();
        r.best_dur = sbd.data();
        r.best_start = sbs.data();
        r.depth = sdp.data();
        r.t0 = st0.data();
        r.sr = ssr.data();
        r.sde_raw = sraw.data();
        r.sde = ssde.data();
        st = tls_search(ctx, time, flux, dy, n, per.data(), (int32_t)m, duration_grid, n_durations, tmpl, n_tmpl,
                        &prm, &r);
        if (st != GTLS_OK) return st;
        evals = r.n_evals;
        macs = r.n_macs;
        chi2_null = r.chi2_null;
        if (r.sde_max >= accept_sde) {
            fb = 0;
            for (size_t i = 0; i < m; ++i) {
                const size_t g = (size_t)idx[i];
                chi2[g] = sc[i];
                bd[g] = sbd[i];
                bs[g] = sbs[i];
                depth[g] = sdp[i];
                t0[g] = st0[i];
                sr[g] = ssr[i];
                raw[g] = sraw[i];
                sde[g] = ssde[i];
            }
            best = idx[(size_t)r.best_period];
            sde_max = r.sde_max;
        }
    }
    if (fb) {
        // Fallback: the whole grid.
        gtls_result r{};
        r.chi2 = chi2.data();
        r.best_dur = bd.data();
        r.best_start = bs.data();
        r.depth = depth.data();
        r.t0 = t0.data();
        r.sr = sr.data();
        r.sde_raw = raw.data();
        r.sde = sde.data();
        st = tls_search(ctx, time, flux, dy, n, period_grid, n_periods, duration_grid, n_durations, tmpl, n_tmpl,
                        &prm, &r);
        if (st != GTLS_OK) return st;
        evals += r.n_evals;
        macs += r.n_macs;
        chi2_null = r.chi2_null;
        best = r.best_period;
        sde_max = r.sde_max;
    }
    struct Out { void* dst; const void* src; size_t bytes; } outs[] = {
        {out->chi2, chi2.data(), 8 * np}, {out->best_dur, bd.data(), 4 * np}, {out->best_start, bs.data(), 4 * np},
        {out->depth, depth.data(), 8 * np}, {out->t0, t0.data(), 8 * np}, {out->sr, sr.data(), 8 * np},
        {out->sde_raw, raw.data(), 8 * np}, {out->sde, sde.data(), 8 * np}};
    for (const Out& o : outs)
        if (o.dst) std::memcpy(o.dst, o.src, o.bytes);
    if (searched) {
        std::memset(searched, fb ? 1 : 0, np);
        if (!fb)
            for (int32_t i : idx) searched[i] = 1;
    }
    if (fell_back) *fell_back = fb;
    out->chi2_null = chi2_null;
    out->best_period = best;
    out->sde_max = sde_max;
    out->n_evals = evals;
    out->n_macs = macs;
    return GTLS_OK;
}

gtls_status tls_search_refined(gtls_ctx* ctx, const double* time, const double* flux, const double* dy, int64_t n,
                               const double* period_grid, int32_t n_periods, const double* duration_grid,
                               int32_t n_durations, const double* tmpl, int32_t n_tmpl, const gtls_params* params,
                               int32_t n_refine, gtls_result* out, uint8_t* refined) {
    if (!ctx) return GTLS_EINVAL;
    if (out) out->best_period = -1;
    if (!out) return fail(ctx, GTLS_EINVAL, "out is null");
    if (n_refine < 0) return fail(ctx, GTLS_EINVAL, "n_refine must be >= 0");
    if (n_periods < 1) return fail(ctx, GTLS_EINVAL, "n_periods must be >= 1");
    gtls_params prm;
    if (params) prm = *params;
    else gtls_params_default(&prm);
    const size_t np = (size_t)n_periods;
    // Stage 1: the whole grid with the coarse T0 step.
    std::vector<double> chi2(np), depth(np), t0(np), sr(np), raw(np), sde(np);
    std::vector<int32_t> bd(np), bs(np);
    gtls_result c{};
    c.chi2 = chi2.data();
    c.best_dur = bd.data();
    c.best_start = bs.data();
    c.depth = depth.data();
    c.t0 = t0.data();
    c.sr = sr.data();
    c.sde_raw = raw.data();
    c.sde = sde.data();
    gtls_status st = tls_search(ctx, time, flux, dy, n, period_grid, n_periods, duration_grid, n_durations, tmpl,
                                n_tmpl, &prm, &c);
    if (st != GTLS_OK) return st;
    // Candidates: the n_refine largest coarse SDE values (ties: lower index),
    // searched again in ascending period order.
    const size_t k = std::min(np, (size_t)n_refine);
    std::vector<int32_t> idx(np);
    for (size_t i = 0; i < np; ++i) idx[i] = (int32_t)i;
    std::partial_sort(idx.begin(), idx.begin() + (std::ptrdiff_t)k, idx.end(), [&](int32_t a, int32_t b) {
        return sde[a] > sde[b] || (sde[a] == sde[b] && a < b);
    });
    idx.resize(k);
    std::sort(idx.begin(), idx.end());
    uint64_t evals = c.n_evals, macs = c.n_macs;
    if (k > 0) {
        // Stage 2: every T0 offset on the candidates; their results replace the coarse ones.
        std::vector<double> per(k), fchi2(k), fdepth(k), ft0(k);
        std::vector<int32_t> fbd(k), fbs(k);
        for (size_t i = 0; i < k; ++i) per[i] = period_grid[idx[i]];
        gtls_params fine = prm;
        fine.dt0 = 0.0;
        gtls_result f{};
        f.chi2 = fchi2.data();
        f.best_dur = fbd.data();
        f.best_start = fbs.data();
        f.depth = fdepth.data();
        f.t0 = ft0.data();
        st = tls_search(ctx, time, flux, dy, n, per.data(), (int32_t)k, duration_grid, n_durations, tmpl, n_tmpl,
                        &fine, &f);
        if (st != GTLS_OK) return st;
        for (size_t i = 0; i < k; ++i) {
            chi2[idx[i]] = fchi2[i];
            bd[idx[i]] = fbd[i];
            bs[idx[i]] = fbs[i];
            depth[idx[i]] = fdepth[i];
            t0[idx[i]] = ft0[i];
        }
        evals += f.n_evals;
        macs += f.n_macs;
        // The periodogram statistics over the merged chi2.
        int32_t best = -1;
        st = tls_sde(ctx, chi2.data(), n_periods, prm.median_window, sr.data(), raw.data(), sde.data(), &best);
        if (st != GTLS_OK) return st;
        c.best_period = best;
        c.sde_max = sde[(size_t)best];
    }
    struct Out { void* dst; const void* src; size_t bytes; } outs[] = {
        {out->chi2, chi2.data(), 8 * np}, {out->best_dur, bd.data(), 4 * np}, {out->best_start, bs.data(), 4 * np},
        {out->depth, depth.data(), 8 * np}, {out->t0, t0.data(), 8 * np}, {out->sr, sr.data(), 8 * np},
        {out->sde_raw, raw.data(), 8 * np}, {out->sde, sde.data(), 8 * np}};
    for (const Out& o : outs)
        if (o.dst) std::memcpy(o.dst, o.src, o.bytes);
    if (refined) {
        std::memset(refined, 0, np);
        for (int32_t i : idx) refined[i] = 1;
    }
    out->chi2_null = c.chi2_null;
    out->best_period = c.best_period;
    out->sde_max = c.sde_max;
    out->n_evals = evals;
    out->n_macs = macs;
    return GTLS_OK;
}

}  // extern "C"
