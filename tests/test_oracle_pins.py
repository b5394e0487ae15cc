"""Pins of the CPU oracle against things other than itself (CPU only).

Each test ties one oracle function to the paper's printed numbers, a closed
form, a library routine, brute force on tiny inputs or an invariant, so that
a plausible mistake (dropped term, wrong sign or index, transposed operand)
fails at least one of them.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import ndimage

from paper_2607_00348_amd import synth

DAY = 86400.0


# --------------------------------------------------------------------------
# Period grid (Sect. 2.2.1)

def test_roche_fmax_matches_paper(oracle, golden):
    g = golden["roche_fmax_hz"]
    assert abs(oracle.roche_fmax() - g["value"]) / g["value"] < g["rtol"]
    p = golden["shortest_period_days"]
    assert abs(1.0 / oracle.roche_fmax() / DAY - p["value"]) < p["atol"]


def test_grid_size_matches_paper(oracle, golden):
    g = golden["n_periods_1500d_os3"]
    grid = oracle.period_grid_ofir(1500.0, golden["oversampling_default"]["value"])
    assert abs(len(grid) - g["value"]) / g["value"] < g["rtol"]
    assert np.all(np.diff(grid) > 0)
    assert grid[-1] <= 750.0 and abs(grid[-1] - 750.0) < 1e-9
    assert grid[0] >= 1.0 / oracle.roche_fmax() / DAY


def test_grid_step_is_transit_duty_cycle(oracle):
    """Ofir's criterion: the frequency step equals the duty cycle of a central
    transit, R/(pi a) with a from Kepler's third law, over S * OS.  Derived
    here from the orbit, not from the grid's A constant."""
    s_days, os_f = 500.0, 3.0
    grid = oracle.period_grid_ofir(s_days, os_f)
    f = np.sort(1.0 / (grid * DAY))
    gm = oracle.G_SI * oracle.M_SUN
    for k in (10, len(f) // 3, len(f) // 2, len(f) - 10):
        fm = 0.5 * (f[k] + f[k + 1])
        a = (gm / (4 * math.pi ** 2 * fm ** 2)) ** (1.0 / 3.0)
        q = oracle.R_SUN / (math.pi * a)
        expected = q / (s_days * DAY * os_f)
        assert abs((f[k + 1] - f[k]) - expected) / expected < 1e-6


def test_grid_cube_roots_are_evenly_spaced(oracle):
    grid = oracle.period_grid_ofir(90.0, 3.0, pmin_days=0.5, pmax_days=45.0)
    c = np.sort((1.0 / (grid * DAY)) ** (1.0 / 3.0))
    d = np.diff(c)
    assert np.max(np.abs(d / d.mean() - 1.0)) < 1e-7


# --------------------------------------------------------------------------
# Duration envelope and stride (Sect. 2.2.2, Sect. 2.5)

def test_stride_worked_example(oracle, golden):
    ex = golden["skip_example"]
    assert oracle.t0_stride(ex["n_it"], ex["dt0"]) == ex["n_skip"]
    assert oracle.t0_stride(7, 0.0) == 1
    assert oracle.t0_stride(5, 0.1) == 1


def test_envelope_constants_are_radius_sums(oracle, golden):
    """k = (R_s + R_p) (4/(pi G M))^(1/3) with P in seconds (Sect. 2.2.2): the
    printed k's correspond to plausible radius sums in solar radii only in
    that unit convention."""
    per_rsun = oracle.R_SUN * (4.0 / (math.pi * oracle.G_SI * oracle.M_SUN)) ** (1.0 / 3.0)
    assert abs(per_rsun - 147.8) < 0.2
    for key, lo, hi in (("gtls_k_min", 0.1, 0.2), ("gtls_k_max", 4.0, 4.4),
                        ("tls_k_min", 0.25, 0.3), ("tls_k_max", 3.6, 3.8)):
        r = golden[key]["value"] / per_rsun
        assert lo < r < hi, (key, r)


def test_envelope_boundaries(oracle, golden):
    kmin, kmax, cap = (golden[k]["value"] for k in ("gtls_k_min", "gtls_k_max", "gtls_q_cap"))
    for p_days in (0.7, 3.0, 30.0, 400.0):
        ps = p_days * DAY
        q_lo = kmin * ps ** (-2.0 / 3.0)
        q_hi = min(kmax * ps ** (-2.0 / 3.0), cap)
        assert oracle.duration_valid(p_days, q_lo * p_days * (1 + 1e-9), 1, kmin, kmax, cap)
        assert not oracle.duration_valid(p_days, q_lo * p_days * (1 - 1e-9), 1, kmin, kmax, cap)
        assert oracle.duration_valid(p_days, q_hi * p_days * (1 - 1e-9), 1, kmin, kmax, cap)
        assert not oracle.duration_valid(p_days, q_hi * p_days * (1 + 1e-9), 1, kmin, kmax, cap)
        # envelope off: only the cap remains
        assert oracle.duration_valid(p_days, q_lo * p_days * 0.5, 0, kmin, kmax, cap)
        assert not oracle.duration_valid(p_days, cap * p_days * 1.0001, 0, kmin, kmax, cap)


def test_points_in_duration(oracle):
    assert oracle.points_in_duration(1024, 8.0, 10.0 * 8 / 1024) == 10
    assert oracle.points_in_duration(1024, 8.0, 10.5 * 8 / 1024) == 11   # exact half rounds up
    assert oracle.points_in_duration(1024, 8.0, 10.49 * 8 / 1024) == 10
    assert oracle.points_in_duration(1000, 10.0, 1e-6) == 1       # clamp low
    assert oracle.points_in_duration(10, 1.0, 5.0) == 10          # clamp high


def test_duration_grid_spans_envelope(oracle):
    d = oracle.duration_grid(0.5, 45.0, 12)
    assert len(d) == 12 and np.all(np.diff(d) > 0)
    r = d[1:] / d[:-1]
    assert np.max(np.abs(r / r[0] - 1)) < 1e-12                    # log-spaced
    # extremes lie on the envelope at the period extremes
    assert oracle.duration_valid(0.5, d[0] * (1 + 1e-9))
    assert not oracle.duration_valid(0.5, d[0] * (1 - 1e-6))
    assert oracle.duration_valid(45.0, d[-1] * (1 - 1e-9))
    assert not oracle.duration_valid(45.0, d[-1] * (1 + 1e-6))


# --------------------------------------------------------------------------
# Template (unit-depth quadratic limb-darkened transit)

def _lens_area(z, p):
    """Area of the intersection of the unit disk and a disk of radius p at
    distance z (textbook two-circle lens)."""
    if z >= 1 + p:
        return 0.0
    if z <= 1 - p:
        return math.pi * p * p
    k0 = math.acos((p * p + z * z - 1) / (2 * p * z))
    k1 = math.acos((1 - p * p + z * z) / (2 * z))
    return p * p * k0 + k1 - 0.5 * math.sqrt(max(0.0, 4 * z * z - (1 + z * z - p * p) ** 2))


@pytest.mark.parametrize("p", [0.05, 0.1, 0.3])
def test_uniform_source_is_lens_area(oracle, p):
    for z in np.linspace(0.0, 1.0 + p - 1e-6, 23):
        got = oracle.occulted_fraction(float(z), p, 0.0, 0.0)
        assert abs(got - _lens_area(float(z), p) / math.pi) < 1e-12


def test_small_planet_limit(oracle):
    p, u1, u2 = 1e-3, 0.4, 0.25
    for z in (0.0, 0.3, 0.6, 0.9):
        mu = math.sqrt(1 - z * z)
        approx = p * p * (1 - u1 * (1 - mu) - u2 * (1 - mu) ** 2) / (1 - u1 / 3 - u2 / 6)
        assert abs(oracle.occulted_fraction(z, p, u1, u2) / approx - 1) < 1e-5


def test_template_shape(oracle):
    tm = oracle.template_quadratic(0.4, 0.25, 0.05, 0.3, 256)
    assert tm.max() == 1.0 and np.all(tm > 0)
    assert np.max(np.abs(tm - tm[::-1])) < 1e-12                   # s(x) = s(1-x)
    assert np.all(np.diff(tm[:128]) >= -1e-15)                     # rises to the centre


def test_resample_is_linear_interpolation(oracle):
    g = synth.rng(3)
    tm = np.sort(g.uniform(0.1, 1.0, 64))
    for d in (1, 2, 7, 63, 64, 65, 500):
        s = oracle.resample(tm, d)
        x = (np.arange(d) + 0.5) / d
        xp = (np.arange(64) + 0.5) / 64
        assert np.allclose(s, np.interp(x, xp, tm), rtol=1e-14, atol=0)


# --------------------------------------------------------------------------
# Fold and sort (Sect. 2.3.1)

def test_fold_sort_matches_numpy_stable_argsort(oracle):
    c = synth.curve_random(11, n=3000, shuffle=True, t_start=2458000.0)
    for period in (0.613, 1.0, 7.3, 55.55):
        phi = c["t"] / period - np.floor(c["t"] / period)
        assert np.array_equal(oracle.fold_sort(c["t"], period),
                              np.argsort(phi, kind="stable").astype(np.int32))


def test_fold_sort_brute_force_with_ties(oracle):
    g = synth.rng(5)
    t = np.round(g.uniform(0, 20, 300), 1)        # many duplicate times -> phase ties
    for period in (0.5, 2.0, 3.7):
        phi = [oracle.phase(x, period) for x in t]
        order = list(range(len(t)))
        for a in range(1, len(order)):              # insertion sort on (phase, index)
            b = a
            while b > 0 and (phi[order[b - 1]], order[b - 1]) > (phi[order[b]], order[b]):
                order[b - 1], order[b] = order[b], order[b - 1]
                b -= 1
        assert list(oracle.fold_sort(t, period)) == order


def test_phase_is_fractional_part(oracle):
    for t, p in ((2458325.123456, 0.7), (0.0, 3.0), (10.0, 2.5), (123.456, 1e-3)):
        fr = Fraction(t) / Fraction(p)
        exact = fr - math.floor(fr)
        got = oracle.phase(t, p)
        assert 0.0 <= got < 1.0
        assert abs(Fraction(got) - exact) <= Fraction(2.0 ** -40) * max(1, abs(fr))


# --------------------------------------------------------------------------
# Window chi-square, depth fit and per-period minimum (Sect. 2.3.2-2.3.4)

def _literal_chi2(y, dy, perm, i, d, s, depth):
    model = np.ones(len(y))
    pos = (i + np.arange(d)) % len(y)
    model[perm[pos]] = 1.0 - depth * s
    return float(np.sum(((y - model) / dy) ** 2))


def _brute_force_period(y, dy, t, period, durs, tm, depth_mode, dt0, oracle):
    """Minimum over windows of the literal all-points chi2 at the best
    non-negative depth.  WLS: the chi2(depth) parabola is recovered from three
    literal evaluations and minimised on depth >= 0.  MEAN: depth is the
    exact window deficit sum over the template sum."""
    n = len(y)
    phi = t / period - np.floor(t / period)
    perm = np.argsort(phi, kind="stable")
    best = (math.inf, -1, -1)
    for j, dur in enumerate(durs):
        q = dur / period
        ps = period * DAY
        if not (q <= oracle.Q_CAP and oracle.K_MIN * ps ** (-2 / 3) <= q <= oracle.K_MAX * ps ** (-2 / 3)):
            continue
        d = int(min(max(math.floor(n * q + 0.5), 1), n))
        x = (np.arange(d) + 0.5) / d
        xp = (np.arange(len(tm)) + 0.5) / len(tm)
        s = np.interp(x, xp, tm)
        stride = 1 if dt0 <= 0 else max(1, int(math.floor(dt0 * d)))
        for i in range(0, n, stride):
            if depth_mode == 0:
                h = 1e-3
                c0 = _literal_chi2(y, dy, perm, i, d, s, 0.0)
                c1 = _literal_chi2(y, dy, perm, i, d, s, h)
                c2 = _literal_chi2(y, dy, perm, i, d, s, 2 * h)
                a2 = (c2 - 2 * c1 + c0) / (2 * h * h)
                a1 = (c1 - c0) / h - a2 * h
                dep = max(0.0, -a1 / (2 * a2))
            else:
                pos = (i + np.arange(d)) % n
                exact = sum(Fraction(1) - Fraction(v) for v in y[perm[pos]])
                dep = max(0.0, float(exact) / float(np.sum(s)))
            val = _literal_chi2(y, dy, perm, i, d, s, dep)
            if val < best[0] * (1 - 1e-12):
                best = (val, j, i)
    return best


@pytest.mark.parametrize("depth_mode", [0, 1])
@pytest.mark.parametrize("dt0", [0.0, 0.3])
def test_search_equals_brute_force_literal_chi2(oracle, depth_mode, dt0):
    c = synth.curve_random(21, n=150, sigma=1e-3, inject=True, varying_dy=True, shuffle=True)
    t, y, dy = c["t"], c["y"], c["dy"]
    tm = oracle.template_quadratic(0.4, 0.25, 0.03, 0.0, 64)
    periods = np.array([0.61, 0.77, 1.1, 1.5])
    durs = np.array([0.01, 0.03, 0.06, 0.1, 0.2])
    r = oracle.tls_search(t, y, dy, periods, durs, tm, dt0=dt0, depth_mode=depth_mode)
    for n_p, period in enumerate(periods):
        val, j, i = _brute_force_period(y, dy, t, period, durs, tm, depth_mode, dt0, oracle)
        assert abs(r.chi2[n_p] - val) <= 1e-9 * val
        assert (r.best_dur[n_p], r.best_start[n_p]) == (j, i)


def test_wls_depth_is_chi2_minimum(oracle):
    c = synth.curve_random(4, n=400, inject=True)
    tm = oracle.template_quadratic(0.4, 0.25, 0.02, 0.0, 128)
    periods = np.array([0.8, 1.3, 2.2])
    durs = oracle.duration_grid(0.8, 2.2, 6)
    r = oracle.tls_search(c["t"], c["y"], c["dy"], periods, durs, tm)
    for k, period in enumerate(periods):
        perm = oracle.fold_sort(c["t"], period)
        d = oracle.points_in_duration(len(c["t"]), period, durs[r.best_dur[k]])
        s = oracle.resample(tm, d)
        lit = oracle.chi2_literal(c["y"], c["dy"], perm, r.best_start[k], d, s, r.depth[k])
        assert abs(lit - r.chi2[k]) <= 1e-10 * lit
        for eps in (1e-6, 1e-5):
            for dd in (r.depth[k] * (1 + eps), r.depth[k] * (1 - eps)):
                assert oracle.chi2_literal(c["y"], c["dy"], perm, r.best_start[k], d, s, dd) >= lit * (1 - 1e-14)


def test_mean_depth_never_beats_wls(oracle):
    c = synth.curve_random(8, n=900, inject=True)
    tm = oracle.template_quadratic(0.4, 0.25, 0.02, 0.0, 128)
    periods = np.geomspace(0.6, 6.0, 40)
    durs = oracle.duration_grid(0.6, 6.0, 8)
    w = oracle.tls_search(c["t"], c["y"], c["dy"], periods, durs, tm, depth_mode=0)
    m = oracle.tls_search(c["t"], c["y"], c["dy"], periods, durs, tm, depth_mode=1)
    assert np.all(m.chi2 >= w.chi2 * (1 - 1e-14))


@pytest.mark.parametrize("depth_mode", [0, 1])
def test_flat_curve_gives_null_chi2_exactly(oracle, depth_mode):
    n = 700
    t = np.arange(n) * synth.KEPLER_CADENCE_DAYS
    y = np.full(n, 1.0 + 2.0 ** -11)       # brighter than the model everywhere
    dy = np.full(n, 2.0 ** -13)
    tm = oracle.template_quadratic(0.4, 0.25, 0.02, 0.0, 64)
    periods = np.geomspace(0.6, 5.0, 30)
    durs = oracle.duration_grid(0.6, 5.0, 6)
    r = oracle.tls_search(t, y, dy, periods, durs, tm, depth_mode=depth_mode)
    assert r.chi2_null == 16.0 * n                              # (2^-11 / 2^-13)^2 per point
    assert np.all(r.chi2 == r.chi2_null)
    assert np.all(r.depth == 0.0)
    ones = oracle.tls_search(t, np.ones(n), dy, periods, durs, tm, depth_mode=depth_mode)
    assert np.all(ones.chi2 == 0.0)


def test_split_transit_equals_centred_transit(oracle):
    """A noiseless box transit straddling phase 0 gives the same chi2(P) as the
    same transit moved to phase 0.5 (padding / wrap-around)."""
    n, period = 1000, 2.0
    t = np.arange(n) * (period / n) * 3.0                       # three cycles, exact phases
    def curve(centre):
        ph = np.mod(t / period - centre + 0.5, 1.0) - 0.5
        return np.where(np.abs(ph) < 0.02, 1.0 - 1e-3, 1.0)
    dy = np.full(n, 1e-3)
    tm = np.ones(16)
    durs = np.array([0.08])
    a = oracle.tls_search(t, curve(0.0), dy, np.array([period]), durs, tm, envelope=0)
    b = oracle.tls_search(t, curve(0.5), dy, np.array([period]), durs, tm, envelope=0)
    assert abs(a.chi2[0] - b.chi2[0]) <= 1e-12 * max(1.0, abs(b.chi2[0]))
    assert a.chi2[0] < a.chi2_null


def test_time_shift_invariance(oracle):
    c = synth.curve_random(31, n=1200, inject=True, sigma=300e-6)
    tm = oracle.template_quadratic(0.4, 0.25, 0.02, 0.0, 128)
    periods = np.geomspace(0.6, 8.0, 60)
    durs = oracle.duration_grid(0.6, 8.0, 8)
    a = oracle.tls_search(c["t"], c["y"], c["dy"], periods, durs, tm)
    shift = 123.456789
    b = oracle.tls_search(c["t"] + shift, c["y"], c["dy"], periods, durs, tm)
    assert np.allclose(a.chi2, b.chi2, rtol=1e-9, atol=0)
    assert np.argmin(a.chi2) == np.argmin(b.chi2)
    assert np.array_equal(a.best_dur, b.best_dur)
    k = int(np.argmin(a.chi2))
    dt = np.mod((b.t0[k] - a.t0[k]) - shift + 0.5 * periods[k], periods[k]) - 0.5 * periods[k]
    assert abs(dt) < 1e-6 * periods[k]


def test_scale_and_order_invariances(oracle):
    c = synth.curve_random(41, n=800, inject=True, varying_dy=True)
    tm = oracle.template_quadratic(0.4, 0.25, 0.02, 0.0, 128)
    periods = np.geomspace(0.6, 6.0, 50)
    durs = oracle.duration_grid(0.6, 6.0, 8)
    base = oracle.tls_search(c["t"], c["y"], c["dy"], periods, durs, tm)
    scaled = oracle.tls_search(c["t"], c["y"], c["dy"] * 4.0, periods, durs, tm)
    assert np.array_equal(scaled.chi2 * 16.0, base.chi2)        # dy * 2^2 -> chi2 * 2^-4
    assert np.array_equal(scaled.best_start, base.best_start)
    assert np.array_equal(oracle.sde(scaled.chi2)[2], oracle.sde(base.chi2)[2])
    perm = synth.rng(9).permutation(len(c["t"]))
    shuf = oracle.tls_search(c["t"][perm], c["y"][perm], c["dy"][perm], periods, durs, tm)
    assert np.allclose(shuf.chi2, base.chi2, rtol=1e-14, atol=0)
    assert np.array_equal(shuf.best_dur, base.best_dur)
    sub = oracle.tls_search(c["t"], c["y"], c["dy"], periods[7:19], durs, tm)
    assert np.array_equal(sub.chi2, base.chi2[7:19])
    assert np.array_equal(sub.best_start, base.best_start[7:19])
    dup = oracle.tls_search(c["t"], c["y"], c["dy"], periods, np.repeat(durs, 2), tm)
    assert np.array_equal(dup.chi2, base.chi2)
    assert np.array_equal(dup.best_dur, 2 * base.best_dur)


def test_chi2_null_is_correctly_summed(oracle):
    g = synth.rng(2)
    y = 1.0 + g.normal(0, 1e-3, 3000)
    dy = g.uniform(1e-4, 1e-3, 3000)
    exact = sum(Fraction(1) / (Fraction(e) * Fraction(e)) * (Fraction(v) - 1) ** 2 for v, e in zip(y, dy))
    assert abs(oracle.chi2_null(y, dy) - float(exact)) <= 1e-13 * float(exact)


# --------------------------------------------------------------------------
# Periodogram statistics (Sect. 2.4)

@pytest.mark.parametrize("window", [1, 5, 91])
def test_sde_matches_numpy_scipy(oracle, window):
    chi2 = synth.random_chi2_series(7, 3000)
    sr, raw, sde, best = oracle.sde(chi2, window)
    ref_sr = chi2.min() / chi2
    assert np.allclose(sr, ref_sr, rtol=1e-15, atol=0)
    ref_raw = (ref_sr - ref_sr.mean()) / ref_sr.std()
    assert np.allclose(raw, ref_raw, rtol=0, atol=1e-12)
    med = ndimage.median_filter(raw, size=window, mode="nearest")
    assert np.array_equal(sde, raw - med)
    assert best == int(np.argmax(sde))
    assert sr.max() == 1.0 and sr[np.argmin(chi2)] == 1.0


def test_sde_degenerate_constant(oracle):
    sr, raw, sde, best = oracle.sde(np.full(50, 7.0), 91)
    assert np.all(sr == 1.0) and np.all(raw == 0.0) and np.all(sde == 0.0) and best == 0


# --------------------------------------------------------------------------
# End-to-end recovery on the 90-day workload without noise

def test_noiseless_injection_recovered(oracle):
    c = synth.curve_90d(noise=False)
    tr = c["meta"]["transit"]
    p_rad = synth.radius_for_depth(tr["depth"], tr["b"], tr["u1"], tr["u2"])
    tm = oracle.template_quadratic(tr["u1"], tr["u2"], p_rad, tr["b"], 1024)
    span = c["t"][-1] - c["t"][0]
    periods = oracle.period_grid_ofir(span, 3.0, pmin_days=0.5, pmax_days=45.0)
    sel = np.abs(np.log(periods / 7.3)) < 0.35                  # 5.1 .. 10.4 d
    periods = periods[sel]
    durs = np.sort(np.r_[oracle.duration_grid(0.5, 45.0, 12), 0.125])
    r = oracle.tls_search(c["t"], c["y"], c["dy"], periods, durs, tm)
    k = int(np.argmin(r.chi2))
    assert abs(k - int(np.argmin(np.abs(periods - 7.3)))) <= 1
    assert abs(durs[r.best_dur[k]] - 0.125) < 1e-12
    assert abs(r.depth[k] / tr["depth"] - 1) < 0.02
    dt = np.mod(r.t0[k] - tr["t0"] + 0.5 * periods[k], periods[k]) - 0.5 * periods[k]
    assert abs(dt) < 0.02


# --------------------------------------------------------------------------
# Two-stage search (Sect. 2.5)

def _two_stage_case(oracle):
    c = synth.curve_random(21, n=1500, inject=True)
    span = c["t"].max() - c["t"].min()
    periods = oracle.period_grid_ofir(span, 2.0, pmin_days=0.5, pmax_days=span / 2)[::3]
    durs = oracle.duration_grid(periods[0], periods[-1], 8)
    tm = oracle.template_quadratic(0.4, 0.25, 0.02, 0.0, 128)
    return c, periods, durs, tm


def test_two_stage_limits(oracle):
    """Refining nothing is the coarse search; refining everything is the
    every-offset search; a partial refinement lowers chi2 only where it
    refines (stride-1 windows include the strided ones)."""
    c, periods, durs, tm = _two_stage_case(oracle)
    coarse = oracle.tls_search(c["t"], c["y"], c["dy"], periods, durs, tm, dt0=0.2)
    full = oracle.tls_search(c["t"], c["y"], c["dy"], periods, durs, tm, dt0=0.0)
    r0, (_, _, sde0, best0), ref0 = oracle.tls_search_two_stage(c["t"], c["y"], c["dy"], periods, durs, tm,
                                                               dt0=0.2, n_refine=0)
    assert not ref0.any() and np.array_equal(r0.chi2, coarse.chi2) and r0.n_evals == coarse.n_evals
    assert best0 == oracle.sde(coarse.chi2)[3]
    rall, (_, _, sdea, besta), refa = oracle.tls_search_two_stage(c["t"], c["y"], c["dy"], periods, durs, tm,
                                                                  dt0=0.2, n_refine=10 ** 6)
    assert refa.all()
    for k in ("chi2", "best_dur", "best_start", "depth"):
        assert np.array_equal(getattr(rall, k), getattr(full, k)), k
    assert besta == oracle.sde(full.chi2)[3]
    rk, (_, _, sdek, bestk), refk = oracle.tls_search_two_stage(c["t"], c["y"], c["dy"], periods, durs, tm,
                                                                dt0=0.2, n_refine=15)
    assert refk.sum() == 15
    assert np.all(rk.chi2[refk] <= coarse.chi2[refk]) and np.array_equal(rk.chi2[~refk], coarse.chi2[~refk])
    assert np.array_equal(rk.chi2[refk], full.chi2[refk])
    # the refined set is the 15 largest first-stage SDE values
    _, _, sdec, _ = oracle.sde(coarse.chi2)
    assert np.min(sdec[refk]) >= np.max(sdec[~refk])


# ---------------------------------------------------------------------------
# Transit statistics at one window (SNR, per-transit and odd/even depths).

def _stats_case(oracle, seed=5, n=900, period=3.7, d=23, start=None):
    g = np.random.default_rng(seed)
    t = np.sort(g.uniform(0.0, 60.0, n))
    y = 1.0 + 1e-3 * g.standard_normal(n)
    dy = np.exp(g.uniform(np.log(5e-4), np.log(2e-3), n))
    tm = oracle.template_quadratic(0.4, 0.25, 0.05, 0.0, 256)
    if start is None:
        start = n - d // 2          # a window that wraps round phase 0
    return t, y, dy, period, d, start, tm


def test_transit_stats_brute_force(oracle):
    """Per-transit depths and counts against numpy sums over the window
    points grouped by transit; SNR^2 against chi2_0 minus the literal chi2 of
    the window at the fitted depth."""
    t, y, dy, period, d, start, tm = _stats_case(oracle)
    n = len(t)
    st, per = oracle.transit_stats(t, y, dy, period, d, start, tm)
    perm = oracle.fold_sort(t, period)
    s = oracle.resample(tm, d)
    pos = start + np.arange(d)
    idx = perm[pos % n]
    ep = np.floor(t[idx] / period).astype(np.int64) - (pos >= n)
    w = 1.0 / dy[idx] ** 2
    r = w * (1.0 - y[idx])
    uniq = np.unique(ep)
    assert np.array_equal(per["epoch"], uniq)
    assert st["n_transits"] == len(uniq) and st["n_in"] == d and st["first_epoch"] == uniq[0]
    for a, e in enumerate(uniq):
        m = ep == e
        assert per["count"][a] == m.sum()
        assert per["depth"][a] == pytest.approx(np.sum(r[m] * s[m]) / np.sum(w[m] * s[m] ** 2), rel=1e-12)
        assert per["sigma"][a] == pytest.approx(1.0 / math.sqrt(np.sum(w[m] * s[m] ** 2)), rel=1e-12)
    # transits counted from the window's first phase group the points the same way
    ph0 = oracle.phase(t[idx[0]], period)
    ep2 = np.floor((t[idx] - ph0 * period) / period + 1e-9).astype(np.int64)
    for e in uniq:
        assert len(np.unique(ep2[ep == e])) == 1
    c, b = np.sum(r * s), np.sum(w * s * s)
    depth = c / b
    assert st["depth"] == pytest.approx(depth, rel=1e-12)
    chi2_0 = oracle.chi2_null(y, dy)
    chi2_fit = oracle.chi2_literal(y, dy, perm, start, d, s, depth)
    assert st["snr"] ** 2 == pytest.approx(chi2_0 - chi2_fit, rel=1e-8) if depth > 0 else st["snr"] == 0.0


def test_transit_stats_recovers_odd_even_depths(oracle):
    """Window points replaced by 1 - depth_e s_k with odd and even depths:
    every per-transit depth, the odd and even pools and the mismatch follow
    exactly."""
    t, y, dy, period, d, start, tm = _stats_case(oracle, seed=9)
    n = len(t)
    perm = oracle.fold_sort(t, period)
    s = oracle.resample(tm, d)
    pos = start + np.arange(d)
    idx = perm[pos % n]
    ep = np.floor(t[idx] / period).astype(np.int64) - (pos >= n)
    y = np.ones(n)
    dodd, deven = 3e-3, 1e-3
    y[idx] = 1.0 - np.where(ep % 2 == 1, dodd, deven) * s
    st, per = oracle.transit_stats(t, y, dy, period, d, start, tm)
    want = np.where(per["epoch"] % 2 == 1, dodd, deven)
    assert np.allclose(per["depth"], want, rtol=1e-12, atol=0)
    assert st["depth_odd"] == pytest.approx(dodd, rel=1e-12)
    assert st["depth_even"] == pytest.approx(deven, rel=1e-12)
    so, se = st["sigma_odd"], st["sigma_even"]
    assert st["odd_even_sigma"] == pytest.approx(abs(dodd - deven) / math.sqrt(so * so + se * se), rel=1e-12)
    # a depth shared by every transit: no mismatch, and the pooled depth is that depth
    y[idx] = 1.0 - 2e-3 * s
    st, _ = oracle.transit_stats(t, y, dy, period, d, start, tm)
    assert st["depth"] == pytest.approx(2e-3, rel=1e-12)
    assert st["odd_even_sigma"] == pytest.approx(0.0, abs=1e-9)


def test_transit_stats_scale_invariance(oracle):
    """dy * 2^k leaves every depth unchanged bit for bit and scales sigma by
    2^k and the SNR (depth over its standard error) by 2^-k."""
    t, y, dy, period, d, start, tm = _stats_case(oracle, seed=3, start=100)
    st0, p0 = oracle.transit_stats(t, y, dy, period, d, start, tm)
    st1, p1 = oracle.transit_stats(t, y, dy * 4.0, period, d, start, tm)
    assert np.array_equal(p0["depth"], p1["depth"]) and np.array_equal(p0["epoch"], p1["epoch"])
    assert np.array_equal(p0["sigma"] * 4.0, p1["sigma"])
    assert st0["snr"] == st1["snr"] * 4.0 and st0["depth_odd"] == st1["depth_odd"]


@pytest.mark.parametrize("start,d", [(0, 50), (333, 41), (1265, 30), (1275, 20), (1279, 7)])
def test_transit_stats_mid_times_exact(oracle, start, d):
    """Phase of the window's middle point and per-transit mid-times on a grid
    where every phase is a multiple of 1/128 (P = 2 d, cadence 1/64 d, ten
    epochs): the sorted order is known in closed form (phase bin, then
    epoch), so phase_mid and t_mid = (epoch + phase_mid) P follow exactly,
    with exact rational arithmetic, for windows whose middle point lies
    before the end of the sorted curve and for wrapped ones (middle point
    past the end: phase + 1, epochs counted one lower)."""
    period, per_epoch, epochs = 2.0, 128, 10
    n = per_epoch * epochs
    k = np.arange(n)
    t = k / 64.0
    y = np.ones(n)
    dy = np.full(n, 1e-3)
    tm = oracle.template_quadratic(0.4, 0.25, 0.05, 0.0, 64)
    st, per = oracle.transit_stats(t, y, dy, period, d, start, tm)

    def point_at(p):                     # input index at sorted position p (closed form)
        q = p % n
        return (q % epochs) * per_epoch + q // epochs

    pm = start + d // 2
    want_phase = Fraction(point_at(pm) % per_epoch, per_epoch) + (1 if pm >= n else 0)
    assert Fraction(st["phase_mid"]) == want_phase
    eps = sorted({point_at(p) // per_epoch - (1 if p >= n else 0) for p in range(start, start + d)})
    assert list(per["epoch"]) == eps
    for e, tmid in zip(per["epoch"], per["t_mid"]):
        assert Fraction(tmid) == (int(e) + want_phase) * Fraction(period)
    assert oracle.fold_sort(t, period)[pm % n] == point_at(pm)


def test_transit_stats_mid_times_at_injected_transits(oracle):
    """Noiseless curve with a symmetric transit every period: at the search's
    best window the reported mid-time of every transit lies within one
    cadence of the injected mid-time T0 + e P (the window is centred on the
    transit, and its middle point is the data point nearest the centre)."""
    cad = 0.02
    t = np.arange(0.0, 60.0, cad)
    tr = dict(period=5.3, t0=1.37, t14=0.24, depth=2e-3, u1=0.4, u2=0.25, b=0.0)
    y = 1.0 - synth.transit_deficit(t, **tr)
    dy = np.full(len(t), 1e-4)
    tm = oracle.template_quadratic(0.4, 0.25, math.sqrt(2e-3), 0.0, 256)
    periods = np.array([tr["period"]])
    durs = np.array([tr["t14"]])
    ref = oracle.tls_search(t, y, dy, periods, durs, tm, envelope=0, q_cap=0.15, threads=1)
    d = oracle.points_in_duration(len(t), tr["period"], tr["t14"])
    st, per = oracle.transit_stats(t, y, dy, tr["period"], d, int(ref.best_start[0]), tm)
    assert st["n_transits"] >= 11
    for e, tmid in zip(per["epoch"], per["t_mid"]):
        assert abs(tmid - (tr["t0"] + e * tr["period"])) <= cad, (e, tmid)
    # the search's T0 is the first of these mid-times at or after min(t)
    assert abs(ref.t0[0] - tr["t0"]) <= cad
