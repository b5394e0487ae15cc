"""Plain FP64 reference of the TLS search described by GTLS (Hu et al.).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP library in ``paper_2607_00348_amd``: the search core is the plain C in
``tls_oracle.c`` (loaded here with ctypes), and the period grid, the duration
grid and the transit template are written below from the paper's text.

What each function follows:

* ``period_grid_ofir`` -- Sect. 2.2.1, the cubic frequency sampling
  f_i = (A i / 3 + C)^3 with f_min = 2/S, the Roche-limit f_max and the
  equations for A, C and N.
* ``duration_grid`` -- Sect. 2.2.2, the envelope k_min P^(-2/3) <= T14/P <=
  min(k_max P^(-2/3), q_cap); log-spaced durations between its extremes over
  the period range.
* ``template_quadratic`` -- the ideal transit of Sect. 2.1 / 2.3.3: a
  quadratic-limb-darkened occultation normalised to unit depth.  The paper
  gives no parameters for it; the occulted flux is the radial integral of the
  intensity over the part of each stellar annulus the planet covers, computed
  with adaptive quadrature (scipy.integrate.quad).
* ``tls_search`` / ``fold_sort`` / ``sde`` -- thin ctypes calls into the C core.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtls_oracle.so")
SRC_PATH = os.path.join(HERE, "tls_oracle.c")

# Physical constants of the grid helpers (SI).  The paper does not state the
# values it used; these are the common ones.
G_SI = 6.674e-11
M_SUN = 1.989e30
R_SUN = 6.957e8
DAY = 86400.0

# Default envelope of Sect. 2.2.2 (s^(2/3)) and the T14/P cap.
K_MIN = 20.05
K_MAX = 620.84
Q_CAP = 0.15


def build(verbose: bool = False) -> str:
    """Compile the C core into ``libtls_oracle.so`` (CPU only)."""
    cmd = ["gcc", "-O2", "-mfma", "-ffp-contract=off", "-fopenmp", "-shared",
           "-fPIC", "-o", LIB_PATH, SRC_PATH, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or (
                os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH)):
            build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lp = ctypes.POINTER(ctypes.c_int64)
        L.oracle_chi2_null.restype = ctypes.c_double
        L.oracle_chi2_null.argtypes = [dp, dp, ctypes.c_int64]
        L.oracle_phase.restype = ctypes.c_double
        L.oracle_phase.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_fold_sort.restype = None
        L.oracle_fold_sort.argtypes = [dp, ctypes.c_int64, ctypes.c_double, ip]
        L.oracle_duration_valid.restype = ctypes.c_int
        L.oracle_duration_valid.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.oracle_points_in_duration.restype = ctypes.c_int64
        L.oracle_points_in_duration.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double]
        L.oracle_t0_stride.restype = ctypes.c_int64
        L.oracle_t0_stride.argtypes = [ctypes.c_int64, ctypes.c_double]
        L.oracle_resample.restype = None
        L.oracle_resample.argtypes = [dp, ctypes.c_int32, ctypes.c_int64, dp]
        L.oracle_chi2_literal.restype = ctypes.c_double
        L.oracle_chi2_literal.argtypes = [dp, dp, ctypes.c_int64, ip, ctypes.c_int64,
                                          ctypes.c_int64, dp, ctypes.c_double]
        L.oracle_tls_search.restype = ctypes.c_int
        L.oracle_tls_search.argtypes = [dp, dp, dp, ctypes.c_int64, dp, ctypes.c_int32,
                                        dp, ctypes.c_int32, dp, ctypes.c_int32,
                                        ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                        ctypes.c_int, dp, ip, ip, dp, dp, dp, lp]
        L.oracle_sde.restype = ctypes.c_int
        L.oracle_sde.argtypes = [dp, ctypes.c_int32, ctypes.c_int32, dp, dp, dp, ip]
        L.oracle_transit_stats.restype = ctypes.c_int
        L.oracle_transit_stats.argtypes = [dp, dp, dp, ctypes.c_int64, ctypes.c_double, ctypes.c_int64,
                                           ctypes.c_int64, dp, ctypes.c_int32, dp, lp, ctypes.c_int64, lp, dp,
                                           dp, dp, lp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# Grids (Sect. 2.2)

def roche_fmax(m_sun: float = 1.0, r_sun: float = 1.0) -> float:
    """f_max = (1/2pi) sqrt(G M / (3 R)^3), in Hz (Sect. 2.2.1)."""
    gm = G_SI * (m_sun * M_SUN)
    a = 3.0 * (r_sun * R_SUN)
    return (1.0 / (2.0 * math.pi)) * math.sqrt(gm / (a * a * a))


def period_grid_ofir(baseline_days: float, os_factor: float = 3.0, m_sun: float = 1.0,
                     r_sun: float = 1.0, pmin_days: float = 0.0,
                     pmax_days: float = 0.0) -> np.ndarray:
    """Cubic frequency grid of Sect. 2.2.1, returned as periods in days, ascending.

    f_min = 2/S unless pmax_days > 0 (then 1/pmax); f_max is the Roche limit
    unless pmin_days > 0 (then 1/pmin).  A uses the baseline S in seconds and
    the oversampling factor.  Frequencies i = 1 .. ceil(N); periods outside
    [P_min, P_max] (inclusive) are dropped.
    """
    s = baseline_days * DAY
    gm = G_SI * (m_sun * M_SUN)
    r = r_sun * R_SUN
    fmin = (2.0 / s) if pmax_days <= 0.0 else 1.0 / (pmax_days * DAY)
    fmax = roche_fmax(m_sun, r_sun) if pmin_days <= 0.0 else 1.0 / (pmin_days * DAY)
    a = (2.0 * math.pi) ** (2.0 / 3.0) / math.pi * r / gm ** (1.0 / 3.0) / (s * os_factor)
    c = fmin ** (1.0 / 3.0) - a / 3.0
    n = (fmax ** (1.0 / 3.0) - fmin ** (1.0 / 3.0) + a / 3.0) * 3.0 / a
    count = int(math.ceil(n))
    pmin = 1.0 / fmax / DAY
    pmax = 1.0 / fmin / DAY
    out = []
    for i in range(count, 0, -1):         # descending frequency = ascending period
        x = a / 3.0 * i + c
        f = x * x * x
        p = 1.0 / f / DAY
        if pmin <= p <= pmax:
            out.append(p)
    return np.array(out, dtype=np.float64)


def duration_grid(pmin_days: float, pmax_days: float, n: int, k_min: float = K_MIN,
                  k_max: float = K_MAX, q_cap: float = Q_CAP) -> np.ndarray:
    """n durations (days), log-spaced between the envelope extremes over the
    period range: T_lo = k_min P_min^(1/3) (shortest allowed at the shortest
    period) and T_hi = min(k_max P_max^(-2/3), q_cap) P_max (Sect. 2.2.2)."""
    lo_q = k_min * (pmin_days * DAY) ** (-2.0 / 3.0)
    hi_q = min(k_max * (pmax_days * DAY) ** (-2.0 / 3.0), q_cap)
    t_lo = lo_q * pmin_days
    t_hi = hi_q * pmax_days
    if n == 1:
        return np.array([t_lo], dtype=np.float64)
    ratio = t_hi / t_lo
    return np.array([t_lo * ratio ** (j / (n - 1)) for j in range(n)], dtype=np.float64)


# --------------------------------------------------------------------------
# Template (unit-depth quadratic-limb-darkened transit)

def _intensity(r: float, u1: float, u2: float) -> float:
    mu = math.sqrt(max(0.0, 1.0 - r * r))
    return 1.0 - u1 * (1.0 - mu) - u2 * (1.0 - mu) ** 2


def _half_angle(r: float, z: float, p: float) -> float:
    """Half the angle of the stellar circle of radius r that lies inside a
    planet disk of radius p centred at distance z."""
    if r <= p - z:
        return math.pi
    if r <= z - p or r >= z + p:
        return 0.0
    c = (r * r + z * z - p * p) / (2.0 * r * z)
    return math.acos(min(1.0, max(-1.0, c)))


def occulted_fraction(z: float, p: float, u1: float, u2: float) -> float:
    """Fraction of the stellar flux hidden by the planet at separation z."""
    from scipy.integrate import quad
    if z >= 1.0 + p:
        return 0.0
    lo = max(0.0, z - p)
    hi = min(1.0, z + p)
    if hi <= lo:
        return 0.0
    pts = [x for x in (abs(z - p), z + p) if lo < x < hi]
    val, _ = quad(lambda r: _intensity(r, u1, u2) * 2.0 * r * _half_angle(r, z, p),
                  lo, hi, points=pts or None, epsabs=1e-15, epsrel=1e-13, limit=400)
    norm = math.pi * (1.0 - u1 / 3.0 - u2 / 6.0)
    return val / norm


def chord_separation(x: float, p: float, b: float) -> float:
    """Sky separation for the fraction x in [0, 1] of the T1..T4 chord
    (straight chord, a/R_star >> 1)."""
    half = math.sqrt((1.0 + p) ** 2 - b * b)
    xx = (2.0 * x - 1.0) * half
    return math.sqrt(b * b + xx * xx)


def template_quadratic(u1: float = 0.4, u2: float = 0.25, p: float = 0.01, b: float = 0.0,
                       m: int = 1024) -> np.ndarray:
    """m samples of the unit-depth transit at x_m = (m + 1/2)/M, normalised so
    the largest sample is exactly 1."""
    d = np.array([occulted_fraction(chord_separation((k + 0.5) / m, p, b), p, u1, u2)
                  for k in range(m)], dtype=np.float64)
    return d / d.max()


# --------------------------------------------------------------------------
# Search and periodogram (C core)

@dataclass
class SearchResult:
    chi2: np.ndarray
    best_dur: np.ndarray
    best_start: np.ndarray
    depth: np.ndarray
    t0: np.ndarray
    dchi2: np.ndarray
    chi2_null: float
    n_evals: int


def chi2_null(y, dy) -> float:
    y, dy = _f64(y), _f64(dy)
    return lib().oracle_chi2_null(_dp(y), _dp(dy), len(y))


def phase(t: float, period: float) -> float:
    return lib().oracle_phase(float(t), float(period))


def fold_sort(t, period: float) -> np.ndarray:
    t = _f64(t)
    perm = np.empty(len(t), dtype=np.int32)
    lib().oracle_fold_sort(_dp(t), len(t), float(period), _ip(perm))
    return perm


def duration_valid(period, dur, envelope=1, k_min=K_MIN, k_max=K_MAX, q_cap=Q_CAP) -> bool:
    return bool(lib().oracle_duration_valid(float(period), float(dur), int(envelope),
                                            float(k_min), float(k_max), float(q_cap)))


def points_in_duration(n: int, period: float, dur: float) -> int:
    return int(lib().oracle_points_in_duration(int(n), float(period), float(dur)))


def t0_stride(d: int, dt0: float) -> int:
    return int(lib().oracle_t0_stride(int(d), float(dt0)))


def resample(tmpl, d: int) -> np.ndarray:
    tmpl = _f64(tmpl)
    out = np.empty(d, dtype=np.float64)
    lib().oracle_resample(_dp(tmpl), len(tmpl), int(d), _dp(out))
    return out


def chi2_literal(y, dy, perm, i: int, d: int, s, depth: float) -> float:
    y, dy, s = _f64(y), _f64(dy), _f64(s)
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    return lib().oracle_chi2_literal(_dp(y), _dp(dy), len(y), _ip(perm), int(i), int(d),
                                     _dp(s), float(depth))


def tls_search(t, y, dy, periods, durations, tmpl, dt0: float = 0.0, envelope: int = 1,
               k_min: float = K_MIN, k_max: float = K_MAX, q_cap: float = Q_CAP,
               depth_mode: int = 0, threads: int | None = None) -> SearchResult:
    t, y, dy = _f64(t), _f64(y), _f64(dy)
    periods, durations, tmpl = _f64(periods), _f64(durations), _f64(tmpl)
    if np.any(np.abs(1.0 - y) >= 1024.0):
        raise ValueError("flux must satisfy |1 - y| < 1024")
    n_p = len(periods)
    chi2 = np.empty(n_p)
    bdur = np.empty(n_p, dtype=np.int32)
    bst = np.empty(n_p, dtype=np.int32)
    depth = np.empty(n_p)
    t0 = np.empty(n_p)
    dchi2 = np.empty(n_p)
    nev = ctypes.c_int64(0)
    if threads is None:
        threads = os.cpu_count() or 1
    lib().oracle_tls_search(_dp(t), _dp(y), _dp(dy), len(t), _dp(periods), n_p,
                            _dp(durations), len(durations), _dp(tmpl), len(tmpl),
                            float(dt0), int(envelope), float(k_min), float(k_max),
                            float(q_cap), int(depth_mode), int(threads), _dp(chi2),
                            _ip(bdur), _ip(bst), _dp(depth), _dp(t0), _dp(dchi2),
                            ctypes.byref(nev))
    return SearchResult(chi2, bdur, bst, depth, t0, dchi2, chi2_null(y, dy), int(nev.value))


def sde(chi2, window: int = 91):
    """Returns (sr, sde_raw, sde, best_index)."""
    chi2 = _f64(chi2)
    n = len(chi2)
    sr, raw, out = np.empty(n), np.empty(n), np.empty(n)
    best = ctypes.c_int32(0)
    lib().oracle_sde(_dp(chi2), n, int(window), _dp(sr), _dp(raw), _dp(out), ctypes.byref(best))
    return sr, raw, out, int(best.value)


def tls_search_two_stage(t, y, dy, periods, durations, tmpl, dt0: float, n_refine: int, window: int = 91,
                         **kw):
    """Two-stage search (Sect. 2.5): the whole grid with T0 step dt0, then
    every T0 offset on the n_refine periods of largest first-stage SDE (ties:
    lower index); their results replace the first-stage ones and the SDE
    periodogram is taken over the merged chi2.  Returns (SearchResult,
    (sr, sde_raw, sde, best), refined mask)."""
    periods = _f64(periods)
    coarse = tls_search(t, y, dy, periods, durations, tmpl, dt0=dt0, **kw)
    _, _, sde0, _ = sde(coarse.chi2, window)
    order = sorted(range(len(periods)), key=lambda i: (-sde0[i], i))
    pick = np.array(sorted(order[:max(0, min(n_refine, len(periods)))]), dtype=np.int64)
    res = SearchResult(coarse.chi2.copy(), coarse.best_dur.copy(), coarse.best_start.copy(),
                       coarse.depth.copy(), coarse.t0.copy(), coarse.dchi2.copy(), coarse.chi2_null,
                       coarse.n_evals)
    refined = np.zeros(len(periods), dtype=bool)
    if len(pick):
        fine = tls_search(t, y, dy, periods[pick], durations, tmpl, dt0=0.0, **kw)
        for a, k in enumerate(pick):
            res.chi2[k] = fine.chi2[a]
            res.best_dur[k] = fine.best_dur[a]
            res.best_start[k] = fine.best_start[a]
            res.depth[k] = fine.depth[a]
            res.t0[k] = fine.t0[a]
            res.dchi2[k] = fine.dchi2[a]
        res.n_evals += fine.n_evals
        refined[pick] = True
    return res, sde(res.chi2, window), refined


TRANSIT_STATS_KEYS = ("snr", "depth", "depth_odd", "depth_even", "sigma_odd", "sigma_even", "odd_even_sigma",
                      "phase_mid")


def transit_stats(t, y, dy, period: float, d: int, start: int, tmpl, max_transits: int = 1 << 20):
    """SNR, per-transit and odd/even depths of the window of d points that
    starts at sorted position `start` of the curve folded at `period` (the
    reading is stated at oracle_transit_stats in tls_oracle.c).  Returns
    (stats dict, per-transit dict of arrays: epoch, t_mid, depth, sigma,
    count)."""
    t, y, dy, tmpl = _f64(t), _f64(y), _f64(dy), _f64(tmpl)
    st = np.zeros(8)
    ints = np.zeros(3, dtype=np.int64)
    cap = int(max_transits)
    ep = np.zeros(cap, dtype=np.int64)
    tm, de, sg = np.zeros(cap), np.zeros(cap), np.zeros(cap)
    cn = np.zeros(cap, dtype=np.int64)
    lp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    rc = lib().oracle_transit_stats(_dp(t), _dp(y), _dp(dy), len(t), float(period), int(d), int(start),
                                    _dp(tmpl), len(tmpl), _dp(st), lp(ints), cap, lp(ep), _dp(tm), _dp(de),
                                    _dp(sg), lp(cn))
    if rc != 0:
        raise ValueError("more transits than max_transits")
    stats = dict(zip(TRANSIT_STATS_KEYS, (float(v) for v in st)))
    stats.update(n_in=int(ints[0]), n_transits=int(ints[1]), first_epoch=int(ints[2]))
    k = int(ints[1])
    return stats, {"epoch": ep[:k], "t_mid": tm[:k], "depth": de[:k], "sigma": sg[:k], "count": cn[:k]}
