"""Injection-recovery harness: detection (precision, recall, ROC) and
parameter recovery (average relative errors) on seeded synthetic curves.

The detection test of Sect. 3.1: 4-year, 30-min white-noise curves (110 ppm)
of which half carry one injected transit with P < 14 d (``synth.injection_curve``);
a curve is flagged when its best peak has SDE >= 7 and SNR >= 5 (the
thresholds of the precision/recall table, Sect. 3.1).  Precision and recall
count curves (their definitions in Sect. 3.1: a flagged positive is a true
positive whatever period it found; the period-matched recall is reported
beside it), the ROC sweeps the SDE threshold (the TPR/FPR definitions of
Sect. 3.2), and the parameter errors follow the average-relative-error
equation of Sect. 3.3.1: period, duration and depth errors relative to the
larger of the two values, T0 relative to the injected period after moving
the injected T0 by whole periods to the observed epoch nearest the
recovered one.

Every search runs through the C ABI (``gtls``): the two-stage search of
Sect. 2.5 (coarse dt0 over the full grid, stride-1 refinement of the
best-SDE periods) and the transit statistics of the best window.  The
metric functions below are plain host arithmetic.

Run: ``python -m paper_2607_00348_amd.injection --curves 256`` prints one
JSON summary.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import gtls, synth

SDE_MIN, SNR_MIN = 7.0, 5.0


# ---------------------------------------------------------------------------
# Metrics (host arithmetic)

def detected(sde, snr, sde_min: float = SDE_MIN, snr_min: float = SNR_MIN) -> np.ndarray:
    """Flag of each curve: SDE and SNR both at or above their thresholds."""
    return (np.asarray(sde, dtype=np.float64) >= sde_min) & (np.asarray(snr, dtype=np.float64) >= snr_min)


def confusion(labels, flags) -> dict:
    """Counts of true/false positives/negatives (labels: curve is positive)."""
    lab = np.asarray(labels, dtype=bool)
    fl = np.asarray(flags, dtype=bool)
    return {"tp": int(np.sum(lab & fl)), "fp": int(np.sum(~lab & fl)), "tn": int(np.sum(~lab & ~fl)),
            "fn": int(np.sum(lab & ~fl))}


def precision_recall(c: dict) -> tuple[float, float]:
    """Precision and recall (Sect. 3.1); NaN where the denominator is zero."""
    p = c["tp"] / (c["tp"] + c["fp"]) if c["tp"] + c["fp"] else math.nan
    r = c["tp"] / (c["tp"] + c["fn"]) if c["tp"] + c["fn"] else math.nan
    return p, r


def roc(scores, labels) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """TPR and FPR (Sect. 3.2) of the rule 'score >= threshold' for every
    distinct score taken as threshold, in decreasing order, preceded by the
    point (0, 0) of an infinite threshold.  Returns (fpr, tpr, thresholds)."""
    s = np.asarray(scores, dtype=np.float64)
    lab = np.asarray(labels, dtype=bool)
    npos, nneg = int(lab.sum()), int((~lab).sum())
    order = np.argsort(-s, kind="stable")
    s_sorted, l_sorted = s[order], lab[order]
    tp = np.cumsum(l_sorted)
    fp = np.cumsum(~l_sorted)
    # the last index of each run of equal scores: all of them pass together
    last = np.r_[np.nonzero(np.diff(s_sorted))[0], len(s_sorted) - 1] if len(s_sorted) else np.array([], int)
    tpr = np.r_[0.0, tp[last] / npos if npos else np.full(len(last), math.nan)]
    fpr = np.r_[0.0, fp[last] / nneg if nneg else np.full(len(last), math.nan)]
    return fpr, tpr, np.r_[math.inf, s_sorted[last]]


def auc(fpr, tpr) -> float:
    """Area under the ROC polyline (trapezoids)."""
    f, t = np.asarray(fpr, dtype=np.float64), np.asarray(tpr, dtype=np.float64)
    return float(np.sum(np.diff(f) * (t[1:] + t[:-1]) * 0.5))


def are_ratio(recovered, expected) -> np.ndarray:
    """|r - e| / max(r, e) (Sect. 3.3.1: period, duration and depth); a
    negative recovered value counts as zero (error 1); both zero gives 0."""
    r = np.maximum(np.asarray(recovered, dtype=np.float64), 0.0)
    e = np.asarray(expected, dtype=np.float64)
    m = np.maximum(r, e)
    return np.where(m > 0, np.abs(r - e) / np.where(m > 0, m, 1.0), 0.0)


def are_t0(t0_r, t0_e, p_e, t_min, t_max) -> np.ndarray:
    """|T0_r - (T0_e + n P_e)| / P_e (Sect. 3.3.1): n is the whole number of
    periods that puts T0_e + n P_e inside [t_min, t_max] nearest T0_r; when
    no epoch falls inside, the nearest to T0_r over all n."""
    t0r = np.asarray(t0_r, dtype=np.float64)
    t0e = np.asarray(t0_e, dtype=np.float64)
    pe = np.asarray(p_e, dtype=np.float64)
    lo = np.ceil((t_min - t0e) / pe)
    hi = np.floor((t_max - t0e) / pe)
    n = np.round((t0r - t0e) / pe)
    n = np.where(lo <= hi, np.clip(n, lo, hi), n)
    return np.abs(t0r - (t0e + n * pe)) / pe


def period_match(p_r, p_e, tol: float = 0.01) -> np.ndarray:
    """Recovered period within tol (relative) of the injected one or of
    P/2, P/3, 2P, 3P (aliases the fold cannot tell apart)."""
    pr = np.asarray(p_r, dtype=np.float64)
    pe = np.asarray(p_e, dtype=np.float64)
    ok = np.zeros(pr.shape, dtype=bool)
    for h in (1.0, 0.5, 1.0 / 3.0, 2.0, 3.0):
        ok |= np.abs(pr - h * pe) <= tol * h * pe
    return ok


# ---------------------------------------------------------------------------
# The harness

def search_setup(days: float, cadence_min: float):
    """Blind-search grids of Sect. 3: the Ofir grid (oversampling 3) from
    0.5 d to half the baseline, 20 durations, one limb-darkened template."""
    span = (math.floor(days / (cadence_min / 1440.0)) - 1) * cadence_min / 1440.0
    grid = gtls.gtls_period_grid_ofir(span, 3.0, pmin_days=0.5, pmax_days=span / 2)
    durs = gtls.gtls_duration_grid(0.5, span / 2, 20)
    tm = gtls.gtls_template_quadratic(0.4, 0.25, 0.01, 0.0, 1024)
    return grid, durs, tm


def recover(ctx, curve: dict, grid, durs, tm, dt0: float, n_refine: int) -> dict:
    """Best peak of one curve (two-stage search when n_refine > 0) and the
    transit statistics of its window."""
    prm = gtls.gtls_params_default(dt0=dt0)
    if n_refine > 0:
        r, _ = gtls.tls_search_refined(ctx, curve["t"], curve["y"], curve["dy"], grid, durs, tm, n_refine, prm)
    else:
        r = gtls.tls_search(ctx, curve["t"], curve["y"], curve["dy"], grid, durs, tm, prm)
    b = r.best_period
    out = {"best_period": int(b), "period": float(grid[b]), "sde": float(r.sde_max), "snr": 0.0,
           "duration": math.nan, "depth": 0.0, "t0": math.nan, "n_evals": int(r.n_evals)}
    j = int(r.best_dur[b])
    if j >= 0:
        st, _ = gtls.tls_transit_stats(ctx, curve["t"], curve["y"], curve["dy"], float(grid[b]), float(durs[j]),
                                       tm, int(r.best_start[b]))
        out.update(snr=float(st["snr"]), duration=float(durs[j]), depth=float(r.depth[b]), t0=float(r.t0[b]))
    return out


def summarize(recs: list, truths: list, t_min: float, t_max: float, sde_min: float = SDE_MIN,
              snr_min: float = SNR_MIN) -> dict:
    """Detection counts, the Sect. 3.1-3.3 metrics and the ROC of per-curve results
    (truth None: a negative curve)."""
    lab = np.array([tr is not None for tr in truths])
    sde = np.array([r["sde"] for r in recs])
    snr = np.array([r["snr"] for r in recs])
    flag = detected(sde, snr, sde_min, snr_min)
    c = confusion(lab, flag)
    prec, rec = precision_recall(c)
    fpr, tpr, thr = roc(sde, lab)
    out = {"n_curves": len(recs), "n_positive": int(lab.sum()), "sde_min": sde_min, "snr_min": snr_min, **c,
           "precision": prec, "recall": rec, "roc_auc_sde": auc(fpr, tpr),
           "roc_sde": {"fpr": fpr.tolist(), "tpr": tpr.tolist(), "threshold": thr.tolist()}}
    pos = np.nonzero(lab)[0]
    if len(pos):
        pe = np.array([truths[i]["period"] for i in pos])
        pr = np.array([recs[i]["period"] for i in pos])
        match = period_match(pr, pe)
        out["recall_period_match"] = float(np.mean(flag[pos] & match))
        d_r = np.array([recs[i]["duration"] for i in pos])
        d_r = np.where(np.isfinite(d_r), d_r, 0.0)
        t0_r = np.array([recs[i]["t0"] for i in pos])
        errs = {"P": are_ratio(pr, pe),
                "D": are_ratio(d_r, np.array([truths[i]["t14"] for i in pos])),
                "Dp": are_ratio(np.array([recs[i]["depth"] for i in pos]), np.array([truths[i]["depth"] for i in pos])),
                "T0": np.where(np.isfinite(t0_r),
                               are_t0(np.where(np.isfinite(t0_r), t0_r, 0.0),
                                      np.array([truths[i]["t0"] for i in pos]), pe, t_min, t_max), 1.0)}
        out["are_all_positives"] = {k: float(np.mean(v)) for k, v in errs.items()}
        hit = flag[pos] & match
        out["are_period_matched"] = ({k: float(np.mean(v[hit])) for k, v in errs.items()} if hit.any() else None)
    return out


def run(n_curves: int, seed: int = 7, days: float = 1461.0, cadence_min: float = 30.0, sigma: float = 110e-6,
        dt0: float = 0.1, n_refine: int = 200, log=None) -> dict:
    grid, durs, tm = search_setup(days, cadence_min)
    ctx = gtls.Context(0)
    recs, truths = [], []
    t_search = 0.0
    t_min = t_max = 0.0
    for i in range(n_curves):
        c = synth.injection_curve(i, n_curves, seed=seed, days=days, cadence_min=cadence_min, sigma=sigma)
        t_min, t_max = float(c["t"][0]), float(c["t"][-1])
        t0 = time.perf_counter()
        recs.append(recover(ctx, c, grid, durs, tm, dt0, n_refine))
        t_search += time.perf_counter() - t0
        truths.append(c["meta"]["transit"])
        if log and (i + 1) % 16 == 0:
            log(f"{i + 1} of {n_curves} curves searched ({t_search:.1f} s)")
    ctx.close()
    out = summarize(recs, truths, t_min, t_max)
    out.update({"days": days, "cadence_min": cadence_min, "sigma_ppm": sigma * 1e6, "grid_periods": int(len(grid)),
                "durations": int(len(durs)), "dt0": dt0, "n_refine": n_refine, "search_seconds": t_search,
                "curves_per_hour": 3600.0 * n_curves / t_search if t_search > 0 else None})
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--curves", type=int, default=256)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--days", type=float, default=1461.0)
    ap.add_argument("--cadence-min", type=float, default=30.0)
    ap.add_argument("--sigma-ppm", type=float, default=110.0)
    ap.add_argument("--dt0", type=float, default=0.1)
    ap.add_argument("--refine", type=int, default=200, help="periods refined at stride 1 (0: one stage)")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    res = run(a.curves, a.seed, a.days, a.cadence_min, a.sigma_ppm * 1e-6, a.dt0, a.refine,
              log=lambda m: print(f"[injection] {m}", file=sys.stderr, flush=True))
    s = json.dumps(res)
    print(s, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(s + "\n")


if __name__ == "__main__":
    main()
