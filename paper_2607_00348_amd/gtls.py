"""ctypes binding of libgtls.so, the gfx950 TLS search.

Argument marshalling only: every call goes straight to the C entry point of
the same name declared in include/gtls.h.  Host arrays are numpy; the *_dev
calls take device addresses (for example ``tensor.data_ptr()`` of a torch
tensor on the GPU) and the stream is the one the context was created with.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgtls.so")

GTLS_OK, GTLS_EINVAL, GTLS_ENOMEM, GTLS_EDEVICE, GTLS_EINTERNAL = 0, -1, -2, -3, -4
GTLS_FP64, GTLS_FP32C = 0, 1
GTLS_DEPTH_WLS, GTLS_DEPTH_MEAN = 0, 1

EXPORTED = ["gtls_create", "gtls_destroy", "gtls_last_error", "gtls_params_default", "gtls_sync",
            "gtls_profile_enable", "gtls_profile_read",
            "tls_search", "tls_search_dev", "tls_search_dev_noalloc", "tls_search_batch", "tls_search_batch_dev", "tls_fold_sort",
            "tls_sde", "tls_search_refined", "tls_transit_stats", "gtls_period_grid_ofir",
            "gtls_duration_grid", "gtls_template_quadratic", "gtls_cnn_num_params", "gtls_cnn_create",
            "gtls_cnn_destroy", "gtls_cnn_view", "gtls_cnn_forward", "gtls_cnn_gradients", "gtls_cnn_train_step",
            "gtls_cnn_get_params", "gtls_cnn_topk", "gtls_cnn_save", "gtls_cnn_load", "tls_search_pruned"]
CNN_VIEW, CNN_BINS = 4096, 512


class gtls_params(ctypes.Structure):
    _fields_ = [("dt0", ctypes.c_double), ("envelope", ctypes.c_int32), ("k_min", ctypes.c_double),
                ("k_max", ctypes.c_double), ("q_cap", ctypes.c_double), ("depth_mode", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("median_window", ctypes.c_int32),
                ("batch_route_min", ctypes.c_int32)]


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class gtls_result(ctypes.Structure):
    _fields_ = [("chi2", _dp), ("best_dur", _ip), ("best_start", _ip), ("depth", _dp), ("t0", _dp),
                ("sr", _dp), ("sde_raw", _dp), ("sde", _dp), ("chi2_null", ctypes.c_double),
                ("best_period", ctypes.c_int32), ("sde_max", ctypes.c_double), ("n_evals", ctypes.c_int64),
                ("n_macs", ctypes.c_int64)]


class gtls_summary(ctypes.Structure):
    _fields_ = [("chi2_null", ctypes.c_double), ("sde_max", ctypes.c_double), ("n_evals", ctypes.c_int64),
                ("n_macs", ctypes.c_int64), ("best_period", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class gtls_transit_stats(ctypes.Structure):
    _fields_ = [("snr", ctypes.c_double), ("depth", ctypes.c_double), ("depth_odd", ctypes.c_double),
                ("depth_even", ctypes.c_double), ("sigma_odd", ctypes.c_double), ("sigma_even", ctypes.c_double),
                ("odd_even_sigma", ctypes.c_double), ("phase_mid", ctypes.c_double), ("n_in", ctypes.c_int64),
                ("n_transits", ctypes.c_int64), ("first_epoch", ctypes.c_int64)]


STAGES = ("prep", "fold_sort", "slide", "reduce", "sde", "slide_strided")


class gtls_profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 8), ("launches", ctypes.c_int64 * 8)]


class GtlsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gtls error {code}: {msg}")
        self.code = code


_lib = None


def _hip_runtimes() -> list:
    """Paths of the HIP runtime libraries (libamdhip64) mapped into this process."""
    found = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                parts = line.split()
                if len(parts) >= 6 and os.path.basename(parts[5]).startswith("libamdhip64.so"):
                    found.add(os.path.realpath(parts[5]))
    except OSError:
        pass
    return sorted(found)


def _load_host_runtime_first() -> None:
    """Make the library share the HIP runtime of PyTorch when PyTorch is installed.

    libgtls.so needs the runtime by its soname (libamdhip64.so.7, found through
    its RUNPATH in the ROCm install).  PyTorch's HIP libraries need the
    unversioned name libamdhip64.so, which they resolve to the copy shipped in
    torch/lib; that copy carries the same soname.  Loaded in the order torch,
    then libgtls, the dynamic loader matches libgtls's need against the soname
    already present and both use torch's copy.  In the other order the process
    ends up with two HIP runtimes (and two HSA runtimes) whose device pointers
    and streams are not interchangeable, which breaks every call that receives
    a torch tensor's address or torch's stream.  So torch is imported first.
    """
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        _load_host_runtime_first()
        L = ctypes.CDLL(LIB_PATH)
        rts = _hip_runtimes()
        if len(rts) > 1:
            raise RuntimeError(f"two HIP runtimes are mapped into this process ({', '.join(rts)}); "
                               "load libgtls.so after PyTorch, never before it")
        vp = ctypes.c_void_p
        L.gtls_create.restype = ctypes.c_int
        L.gtls_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp]
        L.gtls_destroy.restype = None
        L.gtls_destroy.argtypes = [vp]
        L.gtls_last_error.restype = ctypes.c_char_p
        L.gtls_last_error.argtypes = [vp]
        L.gtls_params_default.restype = None
        L.gtls_params_default.argtypes = [ctypes.POINTER(gtls_params)]
        L.gtls_sync.restype = ctypes.c_int
        L.gtls_sync.argtypes = [vp]
        L.gtls_profile_enable.restype = ctypes.c_int
        L.gtls_profile_enable.argtypes = [vp, ctypes.c_int]
        L.gtls_profile_read.restype = ctypes.c_int
        L.gtls_profile_read.argtypes = [vp, ctypes.POINTER(gtls_profile)]
        L.tls_search.restype = ctypes.c_int
        L.tls_search.argtypes = [vp, _dp, _dp, _dp, ctypes.c_int64, _dp, ctypes.c_int32, _dp, ctypes.c_int32,
                                 _dp, ctypes.c_int32, ctypes.POINTER(gtls_params), ctypes.POINTER(gtls_result)]
        L.tls_search_dev.restype = ctypes.c_int
        L.tls_search_dev.argtypes = [vp, vp, vp, vp, ctypes.c_int64, vp, ctypes.c_int32, vp, ctypes.c_int32,
                                     vp, ctypes.c_int32, ctypes.POINTER(gtls_params), vp, vp, vp, vp, vp, vp,
                                     vp, vp, vp]
        L.tls_search_dev_noalloc.restype = ctypes.c_int
        L.tls_search_dev_noalloc.argtypes = L.tls_search_dev.argtypes
        lp = ctypes.POINTER(ctypes.c_int64)
        L.tls_search_batch.restype = ctypes.c_int
        L.tls_search_batch.argtypes = [vp, lp, _dp, _dp, _dp, ctypes.c_int32, lp, _dp, _dp, ctypes.c_int32, _dp,
                                       ctypes.c_int32, ctypes.POINTER(gtls_params), _dp, _ip, _ip, _dp, _dp, _dp,
                                       ctypes.POINTER(gtls_summary)]
        L.tls_search_batch_dev.restype = ctypes.c_int
        L.tls_search_batch_dev.argtypes = [vp, lp, vp, vp, vp, ctypes.c_int32, lp, vp, vp, ctypes.c_int32, vp,
                                           ctypes.c_int32, ctypes.POINTER(gtls_params), vp, vp, vp, vp, vp, vp, vp,
                                           vp, vp]
        L.tls_fold_sort.restype = ctypes.c_int
        L.tls_fold_sort.argtypes = [vp, _dp, ctypes.c_int64, _dp, ctypes.c_int32, _ip]
        _lp = ctypes.POINTER(ctypes.c_int64)
        L.tls_transit_stats.restype = ctypes.c_int
        L.tls_transit_stats.argtypes = [vp, _dp, _dp, _dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double, _dp,
                                        ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(gtls_transit_stats),
                                        ctypes.c_int64, _lp, _dp, _dp, _dp, _lp]
        L.tls_sde.restype = ctypes.c_int
        L.tls_sde.argtypes = [vp, _dp, ctypes.c_int32, ctypes.c_int32, _dp, _dp, _dp, _ip]
        L.tls_search_refined.restype = ctypes.c_int
        L.tls_search_refined.argtypes = [vp, _dp, _dp, _dp, ctypes.c_int64, _dp, ctypes.c_int32, _dp,
                                         ctypes.c_int32, _dp, ctypes.c_int32, ctypes.POINTER(gtls_params),
                                         ctypes.c_int32, ctypes.POINTER(gtls_result),
                                         ctypes.POINTER(ctypes.c_uint8)]
        L.gtls_period_grid_ofir.restype = ctypes.c_int
        L.gtls_period_grid_ofir.argtypes = [ctypes.c_double] * 6 + [_dp, ctypes.c_int32, _ip]
        L.gtls_duration_grid.restype = ctypes.c_int
        L.gtls_duration_grid.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, _dp]
        fp = ctypes.POINTER(ctypes.c_float)
        L.gtls_cnn_num_params.restype = ctypes.c_int64
        L.gtls_cnn_num_params.argtypes = []
        L.gtls_cnn_create.restype = ctypes.c_int
        L.gtls_cnn_create.argtypes = [vp, fp, ctypes.POINTER(vp)]
        L.gtls_cnn_destroy.restype = None
        L.gtls_cnn_destroy.argtypes = [vp]
        L.gtls_cnn_view.restype = ctypes.c_int
        L.gtls_cnn_view.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), _dp, _dp, ctypes.c_int32, fp]
        L.gtls_cnn_forward.restype = ctypes.c_int
        L.gtls_cnn_forward.argtypes = [vp, fp, ctypes.c_int32, fp]
        L.gtls_cnn_gradients.restype = ctypes.c_int
        L.gtls_cnn_gradients.argtypes = [vp, fp, _ip, ctypes.c_int32, fp, fp]
        L.gtls_cnn_train_step.restype = ctypes.c_int
        L.gtls_cnn_train_step.argtypes = [vp, fp, _ip, ctypes.c_int32, ctypes.c_float, fp]
        L.gtls_cnn_get_params.restype = ctypes.c_int
        L.gtls_cnn_get_params.argtypes = [vp, fp]
        L.gtls_cnn_topk.restype = ctypes.c_int
        L.gtls_cnn_topk.argtypes = [vp, fp, ctypes.c_int32, ctypes.c_int32, _ip]
        L.gtls_cnn_save.restype = ctypes.c_int
        L.gtls_cnn_save.argtypes = [vp, ctypes.c_char_p]
        L.gtls_cnn_load.restype = ctypes.c_int
        L.gtls_cnn_load.argtypes = [vp, ctypes.c_char_p]
        L.tls_search_pruned.restype = ctypes.c_int
        L.tls_search_pruned.argtypes = [vp, vp, _dp, _dp, _dp, ctypes.c_int64, _dp, ctypes.c_int32, _dp,
                                        ctypes.c_int32, _dp, ctypes.c_int32, ctypes.POINTER(gtls_params),
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                        ctypes.POINTER(gtls_result), ctypes.POINTER(ctypes.c_uint8),
                                        ctypes.POINTER(ctypes.c_int32)]
        L.gtls_template_quadratic.restype = ctypes.c_int
        L.gtls_template_quadratic.argtypes = [ctypes.c_double] * 4 + [ctypes.c_int32, _dp]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(_dp)


def _check(code: int, ctx=None):
    if code != GTLS_OK:
        raise GtlsError(code, lib().gtls_last_error(ctx).decode())


def gtls_params_default(**overrides) -> gtls_params:
    p = gtls_params()
    lib().gtls_params_default(ctypes.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


class Context:
    """Owns a gtls_ctx on one HIP device; stream is a hipStream_t or None."""

    def __init__(self, device: int = 0, stream: int | None = None):
        self.ptr = ctypes.c_void_p()
        _check(lib().gtls_create(ctypes.byref(self.ptr), int(device), ctypes.c_void_p(stream or 0)))

    def close(self):
        if self.ptr:
            lib().gtls_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def gtls_create(device: int = 0, stream: int | None = None) -> Context:
    return Context(device, stream)


def gtls_sync(ctx: Context):
    _check(lib().gtls_sync(ctx.ptr), ctx.ptr)


def gtls_profile_enable(ctx: Context, on: bool = True):
    _check(lib().gtls_profile_enable(ctx.ptr, int(bool(on))), ctx.ptr)


def gtls_profile_read(ctx: Context) -> dict:
    """{stage name: (summed ms, launches)} for the stages of gtls.h."""
    p = gtls_profile()
    _check(lib().gtls_profile_read(ctx.ptr, ctypes.byref(p)), ctx.ptr)
    return {name: (p.ms[k], int(p.launches[k])) for k, name in enumerate(STAGES)}


@dataclass
class SearchResult:
    chi2: np.ndarray
    best_dur: np.ndarray
    best_start: np.ndarray
    depth: np.ndarray
    t0: np.ndarray
    sr: np.ndarray
    sde_raw: np.ndarray
    sde: np.ndarray
    chi2_null: float
    best_period: int
    sde_max: float
    n_evals: int
    n_macs: int


def tls_search(ctx: Context, time, flux, dy, period_grid, duration_grid, tmpl,
               params: gtls_params | None = None) -> SearchResult:
    t, y, e = _f64(time), _f64(flux), _f64(dy)
    per, dur, tm = _f64(period_grid), _f64(duration_grid), _f64(tmpl)
    npd = len(per)
    out = {k: np.empty(npd) for k in ("chi2", "depth", "t0", "sr", "sde_raw", "sde")}
    out["best_dur"] = np.empty(npd, dtype=np.int32)
    out["best_start"] = np.empty(npd, dtype=np.int32)
    res = gtls_result()
    for k in ("chi2", "depth", "t0", "sr", "sde_raw", "sde"):
        setattr(res, k, _p(out[k]))
    res.best_dur = out["best_dur"].ctypes.data_as(_ip)
    res.best_start = out["best_start"].ctypes.data_as(_ip)
    prm = params if params is not None else gtls_params_default()
    _check(lib().tls_search(ctx.ptr, _p(t), _p(y), _p(e), len(t), _p(per), npd, _p(dur), len(dur), _p(tm),
                            len(tm), ctypes.byref(prm), ctypes.byref(res)), ctx.ptr)
    return SearchResult(chi2_null=res.chi2_null, best_period=res.best_period, sde_max=res.sde_max,
                        n_evals=res.n_evals, n_macs=res.n_macs, **out)


def tls_search_refined(ctx: Context, time, flux, dy, period_grid, duration_grid, tmpl, n_refine: int,
                       params: gtls_params | None = None):
    """Two-stage search; returns (SearchResult, refined mask)."""
    t, y, e = _f64(time), _f64(flux), _f64(dy)
    per, dur, tm = _f64(period_grid), _f64(duration_grid), _f64(tmpl)
    npd = len(per)
    out = {k: np.empty(npd) for k in ("chi2", "depth", "t0", "sr", "sde_raw", "sde")}
    out["best_dur"] = np.empty(npd, dtype=np.int32)
    out["best_start"] = np.empty(npd, dtype=np.int32)
    refined = np.zeros(npd, dtype=np.uint8)
    res = gtls_result()
    for k in ("chi2", "depth", "t0", "sr", "sde_raw", "sde"):
        setattr(res, k, _p(out[k]))
    res.best_dur = out["best_dur"].ctypes.data_as(_ip)
    res.best_start = out["best_start"].ctypes.data_as(_ip)
    prm = params if params is not None else gtls_params_default()
    _check(lib().tls_search_refined(ctx.ptr, _p(t), _p(y), _p(e), len(t), _p(per), npd, _p(dur), len(dur), _p(tm),
                                    len(tm), ctypes.byref(prm), int(n_refine), ctypes.byref(res),
                                    refined.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))), ctx.ptr)
    return (SearchResult(chi2_null=res.chi2_null, best_period=res.best_period, sde_max=res.sde_max,
                         n_evals=res.n_evals, n_macs=res.n_macs, **out), refined.astype(bool))


def tls_search_dev(ctx: Context, time, flux, dy, n: int, period_grid, n_periods: int, duration_grid,
                   n_durations: int, tmpl, n_tmpl: int, params: gtls_params | None, chi2, best_dur, best_start,
                   depth, t0, sr, sde_raw, sde, summary):
    """All array arguments are device addresses (ints); enqueues and returns."""
    prm = params if params is not None else gtls_params_default()
    v = ctypes.c_void_p
    _check(lib().tls_search_dev(ctx.ptr, v(time), v(flux), v(dy), int(n), v(period_grid), int(n_periods),
                                v(duration_grid), int(n_durations), v(tmpl), int(n_tmpl), ctypes.byref(prm),
                                v(chi2), v(best_dur), v(best_start), v(depth), v(t0), v(sr), v(sde_raw), v(sde),
                                v(summary)), ctx.ptr)


def tls_search_dev_noalloc(ctx: Context, time, flux, dy, n: int, period_grid, n_periods: int, duration_grid,
                           n_durations: int, tmpl, n_tmpl: int, params: gtls_params | None, chi2, best_dur,
                           best_start, depth, t0, sr, sde_raw, sde, summary):
    """tls_search_dev with no device allocation (the library's static scratch)."""
    prm = params if params is not None else gtls_params_default()
    v = ctypes.c_void_p
    _check(lib().tls_search_dev_noalloc(ctx.ptr, v(time), v(flux), v(dy), int(n), v(period_grid), int(n_periods),
                                        v(duration_grid), int(n_durations), v(tmpl), int(n_tmpl), ctypes.byref(prm),
                                        v(chi2), v(best_dur), v(best_start), v(depth), v(t0), v(sr), v(sde_raw),
                                        v(sde), v(summary)), ctx.ptr)


@dataclass
class BatchResult:
    chi2: np.ndarray          # CSR over all curves' periods
    best_dur: np.ndarray
    best_start: np.ndarray
    depth: np.ndarray
    t0: np.ndarray
    sde: np.ndarray
    summaries: np.ndarray     # structured: chi2_null, sde_max, n_evals, n_macs, best_period


SUMMARY_DTYPE = np.dtype([("chi2_null", "<f8"), ("sde_max", "<f8"), ("n_evals", "<i8"), ("n_macs", "<i8"),
                          ("best_period", "<i4"), ("pad_", "<i4")])


def tls_search_batch(ctx: Context, offsets, time, flux, dy, period_offsets, periods, duration_grid, tmpl,
                     params: gtls_params | None = None) -> BatchResult:
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    poff = np.ascontiguousarray(period_offsets, dtype=np.int64)
    t, y, e = _f64(time), _f64(flux), _f64(dy)
    per, dur, tm = _f64(periods), _f64(duration_grid), _f64(tmpl)
    nc = len(off) - 1
    npd = int(poff[-1])
    out = {k: np.empty(npd) for k in ("chi2", "depth", "t0", "sde")}
    bd = np.empty(npd, dtype=np.int32)
    bs = np.empty(npd, dtype=np.int32)
    summ = np.zeros(nc, dtype=SUMMARY_DTYPE)
    prm = params if params is not None else gtls_params_default()
    lp = ctypes.POINTER(ctypes.c_int64)
    _check(lib().tls_search_batch(ctx.ptr, off.ctypes.data_as(lp), _p(t), _p(y), _p(e), nc,
                                  poff.ctypes.data_as(lp), _p(per), _p(dur), len(dur), _p(tm), len(tm),
                                  ctypes.byref(prm), _p(out["chi2"]), bd.ctypes.data_as(_ip),
                                  bs.ctypes.data_as(_ip), _p(out["depth"]), _p(out["t0"]), _p(out["sde"]),
                                  summ.ctypes.data_as(ctypes.POINTER(gtls_summary))), ctx.ptr)
    return BatchResult(best_dur=bd, best_start=bs, summaries=summ, **out)


def tls_search_batch_dev(ctx: Context, offsets, time, flux, dy, period_offsets, periods, n_durations_ptr,
                         n_durations: int, tmpl, n_tmpl: int, params: gtls_params | None, chi2, best_dur,
                         best_start, depth, t0, sr, sde_raw, sde, summaries):
    """offsets / period_offsets are host arrays; all other arrays are device
    addresses (ints).  Enqueues and returns."""
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    poff = np.ascontiguousarray(period_offsets, dtype=np.int64)
    prm = params if params is not None else gtls_params_default()
    v = ctypes.c_void_p
    lp = ctypes.POINTER(ctypes.c_int64)
    _check(lib().tls_search_batch_dev(ctx.ptr, off.ctypes.data_as(lp), v(time), v(flux), v(dy), len(off) - 1,
                                      poff.ctypes.data_as(lp), v(periods), v(n_durations_ptr), int(n_durations),
                                      v(tmpl), int(n_tmpl), ctypes.byref(prm), v(chi2), v(best_dur),
                                      v(best_start), v(depth), v(t0), v(sr), v(sde_raw), v(sde), v(summaries)),
           ctx.ptr)


def tls_fold_sort(ctx: Context, time, periods) -> np.ndarray:
    t, per = _f64(time), _f64(np.atleast_1d(periods))
    perm = np.empty((len(per), len(t)), dtype=np.int32)
    _check(lib().tls_fold_sort(ctx.ptr, _p(t), len(t), _p(per), len(per), perm.ctypes.data_as(_ip)), ctx.ptr)
    return perm


def tls_transit_stats(ctx: Context, time, flux, dy, period: float, duration: float, tmpl, start: int,
                      max_transits: int = 65536):
    """SNR, per-transit and odd/even depths of the window of the search's
    best (period, duration, start); see include/gtls.h.  Returns (stats
    dict, per-transit dict of arrays: epoch, t_mid, depth, sigma, count)."""
    t, y, e, tm = _f64(time), _f64(flux), _f64(dy), _f64(tmpl)
    st = gtls_transit_stats()
    cap = int(max_transits)
    ep, cn = np.zeros(cap, dtype=np.int64), np.zeros(cap, dtype=np.int64)
    tmid, dep, sig = np.zeros(cap), np.zeros(cap), np.zeros(cap)
    lp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    _check(lib().tls_transit_stats(ctx.ptr, _p(t), _p(y), _p(e), len(t), float(period), float(duration), _p(tm),
                                   len(tm), int(start), ctypes.byref(st), cap, lp(ep), _p(tmid), _p(dep), _p(sig),
                                   lp(cn)), ctx.ptr)
    stats = {f: getattr(st, f) for f, _ in gtls_transit_stats._fields_}
    k = int(st.n_transits)
    return stats, {"epoch": ep[:k], "t_mid": tmid[:k], "depth": dep[:k], "sigma": sig[:k], "count": cn[:k]}


def tls_sde(ctx: Context, chi2, window: int = 91):
    c = _f64(chi2)
    n = len(c)
    sr, raw, sde = np.empty(n), np.empty(n), np.empty(n)
    best = ctypes.c_int32(-1)
    _check(lib().tls_sde(ctx.ptr, _p(c), n, int(window), _p(sr), _p(raw), _p(sde), ctypes.byref(best)), ctx.ptr)
    return sr, raw, sde, int(best.value)


def gtls_period_grid_ofir(baseline_days: float, os_factor: float = 3.0, m_sun: float = 1.0, r_sun: float = 1.0,
                          pmin_days: float = 0.0, pmax_days: float = 0.0) -> np.ndarray:
    n = ctypes.c_int32(0)
    args = [float(baseline_days), float(os_factor), float(m_sun), float(r_sun), float(pmin_days), float(pmax_days)]
    _check(lib().gtls_period_grid_ofir(*args, None, 0, ctypes.byref(n)))
    out = np.empty(n.value)
    _check(lib().gtls_period_grid_ofir(*args, _p(out), n.value, ctypes.byref(n)))
    return out


def gtls_duration_grid(pmin_days: float, pmax_days: float, n: int, k_min: float = 20.05, k_max: float = 620.84,
                       q_cap: float = 0.15) -> np.ndarray:
    out = np.empty(int(n))
    _check(lib().gtls_duration_grid(float(pmin_days), float(pmax_days), int(n), float(k_min), float(k_max),
                                    float(q_cap), _p(out)))
    return out


def gtls_template_quadratic(u1: float = 0.4, u2: float = 0.25, p: float = 0.01, b: float = 0.0,
                            m: int = 1024) -> np.ndarray:
    out = np.empty(int(m))
    _check(lib().gtls_template_quadratic(float(u1), float(u2), float(p), float(b), int(m), _p(out)))
    return out


# --------------------------------------------------------------------------
# Learned period proposal

def _fp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def gtls_cnn_num_params() -> int:
    return int(lib().gtls_cnn_num_params())


class Cnn:
    """gtls_cnn handle: a period-proposal network living on ctx's device."""

    def __init__(self, ctx: Context, init_params):
        self.ctx = ctx
        self.ptr = ctypes.c_void_p()
        p = np.ascontiguousarray(init_params, dtype=np.float32)
        if len(p) != gtls_cnn_num_params():
            raise ValueError("wrong parameter count")
        _check(lib().gtls_cnn_create(ctx.ptr, _fp(p), ctypes.byref(self.ptr)), ctx.ptr)

    def close(self):
        if self.ptr:
            lib().gtls_cnn_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gtls_cnn_create(ctx: Context, init_params) -> Cnn:
    return Cnn(ctx, init_params)


def gtls_cnn_destroy(net: Cnn):
    net.close()


def gtls_cnn_view(ctx: Context, offsets, time, flux) -> np.ndarray:
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    t, y = _f64(time), _f64(flux)
    nc = len(off) - 1
    out = np.empty((nc, CNN_VIEW), dtype=np.float32)
    _check(lib().gtls_cnn_view(ctx.ptr, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(t), _p(y), nc,
                               _fp(out)), ctx.ptr)
    return out


def _views(v):
    v = np.ascontiguousarray(v, dtype=np.float32)
    return v.reshape(-1, CNN_VIEW)


def gtls_cnn_forward(net: Cnn, views) -> np.ndarray:
    v = _views(views)
    out = np.empty((len(v), CNN_BINS), dtype=np.float32)
    _check(lib().gtls_cnn_forward(net.ptr, _fp(v), len(v), _fp(out)), net.ctx.ptr)
    return out


def gtls_cnn_gradients(net: Cnn, views, labels):
    v = _views(views)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    g = np.empty(gtls_cnn_num_params(), dtype=np.float32)
    loss = ctypes.c_float(0.0)
    _check(lib().gtls_cnn_gradients(net.ptr, _fp(v), lab.ctypes.data_as(_ip), len(v), ctypes.byref(loss), _fp(g)),
           net.ctx.ptr)
    return float(loss.value), g


def gtls_cnn_train_step(net: Cnn, views, labels, lr: float = 1e-3) -> float:
    v = _views(views)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    loss = ctypes.c_float(0.0)
    _check(lib().gtls_cnn_train_step(net.ptr, _fp(v), lab.ctypes.data_as(_ip), len(v), float(lr),
                                     ctypes.byref(loss)), net.ctx.ptr)
    return float(loss.value)


def gtls_cnn_get_params(net: Cnn) -> np.ndarray:
    out = np.empty(gtls_cnn_num_params(), dtype=np.float32)
    _check(lib().gtls_cnn_get_params(net.ptr, _fp(out)), net.ctx.ptr)
    return out


def gtls_cnn_topk(net: Cnn, views, k: int) -> np.ndarray:
    v = _views(views)
    out = np.empty((len(v), int(k)), dtype=np.int32)
    _check(lib().gtls_cnn_topk(net.ptr, _fp(v), len(v), int(k), out.ctypes.data_as(_ip)), net.ctx.ptr)
    return out


def gtls_cnn_save(net: Cnn, path: str):
    _check(lib().gtls_cnn_save(net.ptr, os.fsencode(path)), net.ctx.ptr)


def gtls_cnn_load(net: Cnn, path: str):
    _check(lib().gtls_cnn_load(net.ptr, os.fsencode(path)), net.ctx.ptr)


def tls_search_pruned(ctx: Context, net: Cnn, time, flux, dy, period_grid, duration_grid, tmpl, bin_pmin: float,
                      bin_pmax: float, k: int, accept_sde: float, params: gtls_params | None = None):
    """Learned-proposal search; returns (SearchResult, searched mask, fell_back)."""
    t, y, e = _f64(time), _f64(flux), _f64(dy)
    per, dur, tm = _f64(period_grid), _f64(duration_grid), _f64(tmpl)
    npd = len(per)
    out = {k_: np.empty(npd) for k_ in ("chi2", "depth", "t0", "sr", "sde_raw", "sde")}
    out["best_dur"] = np.empty(npd, dtype=np.int32)
    out["best_start"] = np.empty(npd, dtype=np.int32)
    searched = np.zeros(npd, dtype=np.uint8)
    fell = ctypes.c_int32(0)
    res = gtls_result()
    for k_ in ("chi2", "depth", "t0", "sr", "sde_raw", "sde"):
        setattr(res, k_, _p(out[k_]))
    res.best_dur = out["best_dur"].ctypes.data_as(_ip)
    res.best_start = out["best_start"].ctypes.data_as(_ip)
    prm = params if params is not None else gtls_params_default()
    _check(lib().tls_search_pruned(ctx.ptr, net.ptr, _p(t), _p(y), _p(e), len(t), _p(per), npd, _p(dur), len(dur),
                                   _p(tm), len(tm), ctypes.byref(prm), float(bin_pmin), float(bin_pmax), int(k),
                                   float(accept_sde), ctypes.byref(res),
                                   searched.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), ctypes.byref(fell)),
           ctx.ptr)
    return (SearchResult(chi2_null=res.chi2_null, best_period=res.best_period, sde_max=res.sde_max,
                         n_evals=res.n_evals, n_macs=res.n_macs, **out), searched.astype(bool), bool(fell.value))
