"""FP32C acceptance rule shared by the GPU tests: chi2 within rtol 1e-5 of
the oracle, identical best period, and per period the oracle's best window
or a certified near-tie (never at the best period).

A near-tie is certified when the oracle's own Delta chi2 at the window the GPU
chose falls short of the oracle's maximum by no more than the FP32C error
bound of the two windows.  The bound: r = w (1 - y), w and the template are
stored in FP32 (relative error u each, u = 2^-24) and the correlation sums
run in FP32 over blocks of at most 32 points added into FP64 (relative error
at most 32 u of the block's sum of magnitudes), so |dc| <= 34 u sum|r s| and
|db| <= 34 u sum w s^2; with delta the window's depth, |dDelta| <= 2 delta
|dc| + delta^2 |db| + 2 |c - delta b| |ddelta|, where the last term vanishes
for the weighted least-squares depth (stationary there) and, for the
moving-average depth, |ddelta| <= 2 u sum|1 - y| / sum s (compensated FP32
prefix sums).
"""
import numpy as np
import pytest

from paper_2607_00348_amd import gtls

RTOL32 = 1e-5
U32 = 2.0 ** -24


def window_delta(oracle, c, period, dur, start, tm, depth_mode):
    """FP64 Delta chi2 at one window and its FP32C error bound."""
    n = len(c["t"])
    d = oracle.points_in_duration(n, period, dur)
    s = oracle.resample(tm, d)
    perm = oracle.fold_sort(c["t"], period)
    idx = perm[(start + np.arange(d)) % n]
    w = 1.0 / c["dy"][idx] ** 2
    dev = 1.0 - c["y"][idx]
    cc = float(np.sum(w * dev * s))
    bb = float(np.sum(w * s * s))
    if depth_mode == gtls.GTLS_DEPTH_MEAN:
        delta = max(0.0, float(np.sum(dev)) / float(np.sum(s)))
        dchi2 = 2.0 * delta * cc - delta * delta * bb
        e_delta = 2.0 * U32 * float(np.sum(np.abs(1.0 - c["y"]))) / float(np.sum(s))
    else:
        delta = max(0.0, cc / bb)
        dchi2 = delta * cc
        e_delta = 0.0                      # the WLS optimum is stationary in delta
    k = 34.0 * U32
    e_c = k * float(np.sum(np.abs(w * dev * s)))
    e_b = k * bb
    bound = 2.0 * delta * e_c + delta * delta * e_b + 2.0 * abs(cc - delta * bb) * e_delta
    return dchi2, bound


def check_fp32c(oracle, c, periods, durs, tm, res, fx, label, depth_mode=0):
    rel = np.abs(res.chi2 - fx["chi2"]) / fx["chi2"]
    worst = float(np.max(rel))
    same = (res.best_dur == fx["best_dur"]) & (res.best_start == fx["best_start"])
    _, _, _, best = oracle.sde(fx["chi2"], 91)
    assert same[best], f"{label}: the best period's window differs"
    chi2_null = float(fx["chi2_null"])
    n_tie = 0
    for k in np.nonzero(~same)[0]:
        d_gpu, e_gpu = window_delta(oracle, c, periods[k], durs[int(res.best_dur[k])], int(res.best_start[k]), tm,
                                     depth_mode)
        d_ref, e_ref = window_delta(oracle, c, periods[k], durs[int(fx["best_dur"][k])], int(fx["best_start"][k]),
                                     tm, depth_mode)
        assert d_ref == pytest.approx(chi2_null - fx["chi2"][k], rel=1e-9, abs=1e-9 * chi2_null)
        assert d_ref - d_gpu <= e_gpu + e_ref, (label, int(k), d_ref - d_gpu, e_gpu + e_ref)
        n_tie += 1
    print(f"{label}: {len(periods)} periods, max chi2 rel err {worst:.2e}, certified near-tie windows {n_tie}",
          flush=True)
    assert worst <= RTOL32, (label, worst)
    assert res.best_period == best
    assert res.n_evals == int(fx["n_evals"])
