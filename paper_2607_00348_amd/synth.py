"""Seeded synthetic light curves of the shapes the GTLS paper benchmarks on.

This module only *makes inputs*.  It holds none of the search's arithmetic
(no fold, sort, grid, template resampling, chi-square or SDE); the transit it
injects is a forward model of the data: the stellar intensity of a quadratic
limb-darkening law integrated over the planet disk on a polar midpoint grid.

Both the HIP library's tests/benchmark and the CPU oracle's tests take their
light curves from here, so the two sides always see identical inputs.

Workloads (Kepler long cadence = 29.4 min):

* ``curve_90d``    -- 90-day curve, 4409 cadences from t = 0, 200 ppm white
  noise, one 600 ppm transit (P = 7.3 d, T14 = 3 h, T0 = 1.7 d).
* ``curve_3000d``  -- 3000-day curve, 146 939 cadences, >= 10 % removed in
  1-5 day gaps, 100 ppm white + 30 ppm AR(1) red noise (tau = 0.5 d), one
  Earth-like transit (P = 365 d, 84 ppm, T14 = 13 h, T0 = 121.3 d).
* ``curve_tess``   -- 350 days of 2-min cadence starting at t = 2458325.0
  (BJD-scale times), a 1-day gap every 13.7 d, 500 ppm white noise, a grazing
  transit (b = 0.9, P = 0.7 d, 300 ppm).
* ``curve_random`` -- a generic curve with seeded length/noise/transit.
* ``injection_curve`` -- a 4-year, 30-min, 110 ppm white-noise set, half of
  it with one injected transit of P < 14 d (injection-recovery tests).
* ``proposal_curve`` -- 3000-day curves with the 3000-day curve's gaps and
  noise, 70 % carrying a transit (learned period proposal).

Flux is produced in FP64, rounded to FP32 (the instruments' precision), and
returned as FP64 holding FP32 values.
"""
from __future__ import annotations

import math

import numpy as np

KEPLER_CADENCE_DAYS = 29.4 / 1440.0
TESS_CADENCE_DAYS = 2.0 / 1440.0


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# Transit forward model (data generation only)

def _disk_deficit(z: np.ndarray, p: float, u1: float, u2: float,
                  n_rho: int = 48, n_theta: int = 96) -> np.ndarray:
    """Flux fraction blocked by a planet of radius p (stellar radii) whose
    centre is at sky separation z, by midpoint integration over the planet
    disk in polar coordinates (rho, theta) around the planet centre."""
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    rho = (np.arange(n_rho) + 0.5) / n_rho * p
    th = (np.arange(n_theta) + 0.5) / n_theta * 2.0 * math.pi
    d_area = (p / n_rho) * (2.0 * math.pi / n_theta) * rho          # rho drho dtheta
    cx = rho[:, None] * np.cos(th)[None, :]
    cy = rho[:, None] * np.sin(th)[None, :]
    total = math.pi * (1.0 - u1 / 3.0 - u2 / 6.0)
    out = np.zeros_like(z)
    for k0 in range(0, len(z), 2048):
        zz = z[k0:k0 + 2048, None, None]
        r2 = (zz + cx[None]) ** 2 + cy[None] ** 2
        inside = r2 < 1.0
        mu = np.sqrt(np.clip(1.0 - r2, 0.0, None))
        inten = 1.0 - u1 * (1.0 - mu) - u2 * (1.0 - mu) ** 2
        out[k0:k0 + 2048] = (np.where(inside, inten, 0.0) * d_area[None, :, None]).sum(axis=(1, 2))
    return out / total


def radius_for_depth(depth: float, b: float, u1: float, u2: float) -> float:
    """Planet radius whose deepest point (separation b) blocks `depth`."""
    p = math.sqrt(depth)
    for _ in range(6):
        dd = float(_disk_deficit(np.array([b]), p, u1, u2)[0])
        p *= math.sqrt(depth / dd)
    return p


def transit_deficit(t: np.ndarray, period: float, t0: float, t14: float, depth: float,
                    u1: float, u2: float, b: float = 0.0) -> np.ndarray:
    """Positive flux deficit of a limb-darkened transit (straight chord,
    a/R_star >> 1), scaled so its deepest point equals `depth`."""
    p = radius_for_depth(depth, b, u1, u2)
    dt = np.mod(t - t0 + 0.5 * period, period) - 0.5 * period
    half = math.sqrt((1.0 + p) ** 2 - b * b)
    inside = np.abs(dt) < 0.5 * t14
    out = np.zeros_like(t, dtype=np.float64)
    if np.any(inside):
        x = 2.0 * dt[inside] / t14 * half
        z = np.sqrt(b * b + x * x)
        peak = float(_disk_deficit(np.array([b]), p, u1, u2)[0])
        out[inside] = depth * _disk_deficit(z, p, u1, u2) / peak
    return out


def grazing_t14(period: float, b: float, p: float, m_sun: float = 1.0, r_sun: float = 1.0) -> float:
    """T14 of a circular orbit around a star of the given mass/radius (days)."""
    g, msun, rsun = 6.674e-11, 1.989e30, 6.957e8
    ps = period * 86400.0
    a = (g * m_sun * msun * ps * ps / (4.0 * math.pi ** 2)) ** (1.0 / 3.0) / (r_sun * rsun)
    return period / math.pi * math.asin(min(1.0, math.sqrt((1.0 + p) ** 2 - b * b) / a))


def _to_fp32_flux(y: np.ndarray) -> np.ndarray:
    return y.astype(np.float32).astype(np.float64)


def _curve(t, y, dy, **meta):
    return {"t": np.ascontiguousarray(t, dtype=np.float64),
            "y": np.ascontiguousarray(y, dtype=np.float64),
            "dy": np.ascontiguousarray(dy, dtype=np.float64),
            "meta": meta}


# --------------------------------------------------------------------------
# Workload curves

def curve_90d(seed: int = 0, noise: bool = True, inject: bool = True) -> dict:
    n = 4409
    t = np.arange(n, dtype=np.float64) * KEPLER_CADENCE_DAYS
    g = rng(seed)
    sigma = 200e-6
    y = np.ones(n)
    tr = dict(period=7.3, t0=1.7, t14=0.125, depth=600e-6, u1=0.4, u2=0.25, b=0.0)
    if inject:
        y = y - transit_deficit(t, **tr)
    if noise:
        y = y + sigma * g.standard_normal(n)
    return _curve(t, _to_fp32_flux(y), np.full(n, sigma), transit=tr if inject else None,
                  sigma=sigma, name="kepler_90d")


def curve_3000d(seed: int = 1, inject: bool = True) -> dict:
    n_full = int(round(3000.0 / KEPLER_CADENCE_DAYS))           # 146 939 cadences
    t = np.arange(n_full, dtype=np.float64) * KEPLER_CADENCE_DAYS
    g = rng(seed)
    white, red, tau = 100e-6, 30e-6, 0.5
    phi = math.exp(-KEPLER_CADENCE_DAYS / tau)
    innov = red * math.sqrt(1.0 - phi * phi)
    e = g.standard_normal(n_full) * innov
    ar = np.empty(n_full)
    ar[0] = red * g.standard_normal()
    for k in range(1, n_full):                                    # AR(1) on the full grid
        ar[k] = phi * ar[k - 1] + e[k]
    y = 1.0 + white * g.standard_normal(n_full) + ar
    tr = dict(period=365.0, t0=121.3, t14=13.0 / 24.0, depth=84e-6, u1=0.4, u2=0.25, b=0.0)
    if inject:
        y = y - transit_deficit(t, **tr)
    keep = np.ones(n_full, dtype=bool)
    while keep.sum() > 0.9 * n_full:                              # 1-5 day gaps, >= 10 %
        start = g.uniform(0.0, 3000.0)
        length = g.uniform(1.0, 5.0)
        keep &= ~((t >= start) & (t < start + length))
    sig = math.sqrt(white ** 2 + red ** 2)
    return _curve(t[keep], _to_fp32_flux(y[keep]), np.full(int(keep.sum()), sig),
                  transit=tr if inject else None, sigma=sig, name="kepler_3000d")


def curve_tess(seed: int = 5, inject: bool = True) -> dict:
    t_start = 2458325.0
    n_full = int(round(350.0 / TESS_CADENCE_DAYS))              # 252 000 cadences
    t = t_start + np.arange(n_full, dtype=np.float64) * TESS_CADENCE_DAYS
    g = rng(seed)
    sigma = 500e-6
    keep = np.ones(n_full, dtype=bool)
    k = 1
    while 13.7 * k <= 350.0:                                      # 1-day gap every 13.7 d
        g0 = t_start + 13.7 * k
        keep &= ~((t >= g0 - 1.0) & (t < g0))
        k += 1
    b, depth, period = 0.9, 300e-6, 0.7
    p = radius_for_depth(depth, b, 0.4, 0.25)
    t14 = grazing_t14(period, b, p)
    tr = dict(period=period, t0=t_start + 0.31, t14=t14, depth=depth, u1=0.4, u2=0.25, b=b)
    y = 1.0 + sigma * g.standard_normal(n_full)
    if inject:
        y = y - transit_deficit(t, **tr)
    return _curve(t[keep], _to_fp32_flux(y[keep]), np.full(int(keep.sum()), sigma),
                  transit=tr if inject else None, sigma=sigma, name="tess_13sector")


def curve_random(seed: int, n: int | None = None, n_min: int = 64, n_max: int = 4000,
                 cadence: float = KEPLER_CADENCE_DAYS, sigma: float | None = None,
                 inject: bool | None = None, t_start: float = 0.0,
                 varying_dy: bool = False, shuffle: bool = False) -> dict:
    """Generic seeded curve: optional random time order, per-point errors and a
    random transit; used for parity at sizes the oracle finishes quickly."""
    g = rng(seed)
    if n is None:
        n = int(g.integers(n_min, n_max + 1))
    t = t_start + np.arange(n, dtype=np.float64) * cadence
    if sigma is None:
        sigma = float(math.exp(g.uniform(math.log(50e-6), math.log(2000e-6))))
    y = np.ones(n)
    tr = None
    if inject is None:
        inject = bool(g.uniform() < 0.5)
    span = n * cadence
    if inject:
        period = float(math.exp(g.uniform(math.log(0.6), math.log(max(0.7, span / 3.0)))))
        depth = float(g.uniform(2.0, 8.0) * sigma)
        tr = dict(period=period, t0=t_start + float(g.uniform(0.0, period)),
                  t14=float(min(0.12 * period, g.uniform(0.05, 0.4))), depth=depth,
                  u1=float(g.uniform(0.2, 0.6)), u2=float(g.uniform(0.1, 0.4)), b=0.0)
        y = y - transit_deficit(t, **tr)
    y = y + sigma * g.standard_normal(n)
    dy = np.full(n, sigma)
    if varying_dy:
        dy = sigma * g.uniform(0.5, 2.0, n)
    y = _to_fp32_flux(y)
    if shuffle:
        order = g.permutation(n)
        t, y, dy = t[order], y[order], dy[order]
    return _curve(t, y, dy, transit=tr, sigma=sigma, name=f"random_{seed}")


def random_chi2_series(seed: int, n: int) -> np.ndarray:
    """A positive periodogram-like series (chi2 per period) with a slow trend,
    noise and one dip, for SDE-only checks."""
    g = rng(seed)
    x = np.linspace(0.0, 1.0, n)
    base = 1000.0 * (1.0 + 0.05 * x) + g.normal(0.0, 2.0, n)
    k = int(g.integers(0, n))
    base[k] -= 40.0
    return base


def survey_curve(index: int, n_curves: int = 4096, seed: int = 2, n_min: int = 4000,
                 n_max: int = 147000) -> dict:
    """Curve `index` of the batched Kepler-like survey: length uniform in
    [n_min, n_max] cadences of 29.4 min, white noise with sigma log-uniform in
    [50, 2000] ppm (dy = sigma), and for the first 10 % of a seeded
    permutation of the curves an injected transit: P log-uniform in
    [1, 200] d (at most half the baseline), p ~ U(0.01, 0.1), u1 ~ U(0.2, 0.6),
    u2 ~ U(0.1, 0.4), b = 0, T14 of a circular orbit around a Sun-like star,
    T0 ~ U(0, P)."""
    perm = rng(seed).permutation(n_curves)
    injected = set(perm[: max(1, n_curves // 10)].tolist())
    g = rng(seed * 1_000_003 + index + 1)
    n = int(g.integers(n_min, n_max + 1))
    t = np.arange(n, dtype=np.float64) * KEPLER_CADENCE_DAYS
    sigma = float(math.exp(g.uniform(math.log(50e-6), math.log(2000e-6))))
    y = np.ones(n)
    tr = None
    if index in injected:
        span = n * KEPLER_CADENCE_DAYS
        period = float(math.exp(g.uniform(math.log(1.0), math.log(min(200.0, span / 2)))))
        p = float(g.uniform(0.01, 0.1))
        u1, u2 = float(g.uniform(0.2, 0.6)), float(g.uniform(0.1, 0.4))
        norm = 1.0 - u1 / 3.0 - u2 / 6.0
        depth = p * p * (1.0 - 0.0) / norm                           # central transit, limb-darkened centre
        t14 = grazing_t14(period, 0.0, p)
        tr = dict(period=period, t0=float(g.uniform(0.0, period)), t14=t14, depth=depth, u1=u1, u2=u2, b=0.0)
        y = y - transit_deficit(t, **tr)
    y = y + sigma * g.standard_normal(n)
    return _curve(t, _to_fp32_flux(y), np.full(n, sigma), transit=tr, sigma=sigma, name=f"survey_{index}")


def injection_curve(index: int, n_curves: int, seed: int = 7, days: float = 1461.0, cadence_min: float = 30.0,
                    sigma: float = 110e-6, pos_frac: float = 0.5, pmin: float = 0.5, pmax: float = 14.0,
                    p_min: float = 0.003, p_max: float = 0.012) -> dict:
    """Curve `index` of an injection-recovery set (the white-noise detection
    test of Sect. 3.1): `days` of `cadence_min` sampling from t = 0, white
    noise `sigma` (dy = sigma).  The first pos_frac of a seeded permutation
    of the n_curves are positives: one central (b = 0) limb-darkened transit
    with P log-uniform in [pmin, pmax] d, radius ratio log-uniform in
    [p_min, p_max] (central depth about 10-170 ppm), u1 ~ U(0.2, 0.6),
    u2 ~ U(0.1, 0.4), T14 of a circular orbit around a Sun-like star and
    T0 ~ U(0, P).  The rest are noise only."""
    perm = rng(seed).permutation(n_curves)
    positives = set(perm[: int(round(pos_frac * n_curves))].tolist())
    g = rng(seed * 1_000_003 + index + 1)
    cad = cadence_min / 1440.0
    n = int(math.floor(days / cad))
    t = np.arange(n, dtype=np.float64) * cad
    y = np.ones(n)
    tr = None
    if index in positives:
        period = float(math.exp(g.uniform(math.log(pmin), math.log(pmax))))
        p = float(math.exp(g.uniform(math.log(p_min), math.log(p_max))))
        u1, u2 = float(g.uniform(0.2, 0.6)), float(g.uniform(0.1, 0.4))
        depth = p * p / (1.0 - u1 / 3.0 - u2 / 6.0)
        tr = dict(period=period, t0=float(g.uniform(0.0, period)), t14=grazing_t14(period, 0.0, p), depth=depth,
                  u1=u1, u2=u2, b=0.0)
        y = y - transit_deficit(t, **tr)
    y = y + sigma * g.standard_normal(n)
    return _curve(t, _to_fp32_flux(y), np.full(n, sigma), transit=tr, sigma=sigma, name=f"injection_{index}")


def proposal_curve(index: int, seed: int = 3, pos_frac: float = 0.7) -> dict:
    """Curve `index` of the learned-proposal set: the 3000-day curve's cadence
    (29.4 min, 146,939 cadences from t = 0), gaps (uniform-start blocks of
    U(1, 5) d removed until >= 10 % of the cadences are gone) and noise
    (100 ppm white + AR(1) red noise of stationary sigma 30 ppm, tau = 0.5 d,
    dy = 104.4 ppm); a seeded fraction pos_frac of the curves carries one
    transit with the survey's parameter distribution and P <= 500 d: P
    log-uniform in [1, 500] d, p ~ U(0.01, 0.1), u1 ~ U(0.2, 0.6),
    u2 ~ U(0.1, 0.4), b = 0, T14 of a circular orbit around a Sun-like star,
    T0 ~ U(0, P)."""
    from scipy.signal import lfilter
    g = rng(seed * 1_000_003 + index + 1)
    n_full = int(round(3000.0 / KEPLER_CADENCE_DAYS))
    t = np.arange(n_full, dtype=np.float64) * KEPLER_CADENCE_DAYS
    white, red, tau = 100e-6, 30e-6, 0.5
    phi = math.exp(-KEPLER_CADENCE_DAYS / tau)
    e = g.standard_normal(n_full) * (red * math.sqrt(1.0 - phi * phi))
    e[0] = red * g.standard_normal()
    ar = lfilter([1.0], [1.0, -phi], e)                           # ar[k] = phi ar[k-1] + e[k]
    y = 1.0 + white * g.standard_normal(n_full) + ar
    tr = None
    if g.uniform() < pos_frac:
        period = float(math.exp(g.uniform(math.log(1.0), math.log(500.0))))
        p = float(g.uniform(0.01, 0.1))
        u1, u2 = float(g.uniform(0.2, 0.6)), float(g.uniform(0.1, 0.4))
        depth = p * p / (1.0 - u1 / 3.0 - u2 / 6.0)
        tr = dict(period=period, t0=float(g.uniform(0.0, period)), t14=grazing_t14(period, 0.0, p), depth=depth,
                  u1=u1, u2=u2, b=0.0)
        y = y - transit_deficit(t, **tr)
    keep = np.ones(n_full, dtype=bool)
    while keep.sum() > 0.9 * n_full:
        start = g.uniform(0.0, 3000.0)
        keep &= ~((t >= start) & (t < start + g.uniform(1.0, 5.0)))
    sig = math.sqrt(white ** 2 + red ** 2)
    return _curve(t[keep], _to_fp32_flux(y[keep]), np.full(int(keep.sum()), sig), transit=tr, sigma=sig,
                  name=f"proposal_{index}")


def cnn_init(seed: int = 0) -> np.ndarray:
    """Seeded initial parameters of the period-proposal network, flat in the
    order W0, b0, ..., W4, b4, Wf, bf (W_l: 32 x C_in x 7, Wf: 512 x 32):
    uniform in +-sqrt(6 / fan_in) for weights, zero biases.  The random draws
    live here so the GPU network and the CPU reference start identically."""
    g = rng(seed)
    parts = []
    for cin in (1, 32, 32, 32, 32):
        a = math.sqrt(6.0 / (cin * 7))
        parts.append(g.uniform(-a, a, 32 * cin * 7))
        parts.append(np.zeros(32))
    a = math.sqrt(6.0 / 32)
    parts.append(g.uniform(-a, a, 512 * 32))
    parts.append(np.zeros(512))
    return np.concatenate(parts).astype(np.float64)
