"""Learned period proposal: data, training and evaluation driver.

The network (a small 1D CNN, see include/gtls.h) ranks 512 log-period bins
of a curve from its 4096-bin view; the full TLS search then runs only on the
grid periods inside the top-k bins.  Labels are the best period (largest SDE)
of the full-grid search, computed with the batched GPU search (which is
bit-exact against the CPU oracle).  Everything here calls the C ABI through
``gtls``; the oracle is not used.

Two workloads:

* 90-day stand-in curves (``training_curve``, periods 0.5-45 d):
  ``python -m paper_2607_00348_amd.learned --train 8192 --test 1024`` writes a
  JSON summary: recall@k of the network and of the prior-only ranking (is the
  full-grid best period's bin among the top k), the final recall of the best
  period (curves whose pruned search peaks below SDE ``--accept`` fall back to
  the full grid, which also judges recall), and the curves/hour and speed-up of
  view + network + pruned search + fallback over the plain full-grid search.
* 3000-day curves (``synth.proposal_curve``, periods 0.5-1500 d, 418,590-period
  grid): ``label`` writes the full-grid labels of a range of curves, ``eval``
  trains on them (optionally after pretraining on the injected-period bins of
  further curves) and scores held-out curves against the full grid, the
  prior-only ranking and the coarse two-stage pass.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import gtls, synth

PMIN, PMAX = 0.5, 45.0          # 90-day Kepler-like curves: grid 0.5 .. 45 d
N_BINS = 512
N_CAD = 4409


def bin_edges() -> np.ndarray:
    return PMIN * (PMAX / PMIN) ** (np.arange(N_BINS + 1) / N_BINS)


def period_bin(p: np.ndarray) -> np.ndarray:
    return np.clip(np.floor(np.log(np.asarray(p) / PMIN) / math.log(PMAX / PMIN) * N_BINS), 0, N_BINS - 1).astype(
        np.int32)


def training_curve(index: int, seed: int) -> dict:
    """90-day, 29.4-min cadence curve; sigma log-uniform in [100, 400] ppm;
    70 % carry a transit with P log-uniform in [0.6, 40] d, depth 2-8 sigma
    per point, T14 of a circular orbit around a Sun-like star."""
    g = synth.rng(seed * 1_000_003 + index)
    t = np.arange(N_CAD, dtype=np.float64) * synth.KEPLER_CADENCE_DAYS
    sigma = float(math.exp(g.uniform(math.log(100e-6), math.log(400e-6))))
    y = np.ones(N_CAD)
    tr = None
    if g.uniform() < 0.7:
        period = float(math.exp(g.uniform(math.log(0.6), math.log(40.0))))
        depth = float(g.uniform(2.0, 8.0) * sigma)
        p = math.sqrt(depth)
        tr = dict(period=period, t0=float(g.uniform(0, period)), t14=synth.grazing_t14(period, 0.0, p),
                  depth=depth, u1=float(g.uniform(0.2, 0.6)), u2=float(g.uniform(0.1, 0.4)), b=0.0)
        y = y - synth.transit_deficit(t, **tr)
    y = y + sigma * g.standard_normal(N_CAD)
    return {"t": t, "y": y.astype(np.float32).astype(np.float64), "dy": np.full(N_CAD, sigma), "meta": tr}


def search_inputs():
    span = (N_CAD - 1) * synth.KEPLER_CADENCE_DAYS
    grid = gtls.gtls_period_grid_ofir(span, 3.0, pmin_days=PMIN, pmax_days=PMAX)
    durs = gtls.gtls_duration_grid(PMIN, PMAX, 12)
    tm = gtls.gtls_template_quadratic(0.4, 0.25, 0.01, 0.0, 1024)
    return grid, durs, tm


def batched_search(ctx, curves, grids, durs, tm, params=None, chunk=512, log=None):
    """Full search of many curves (each its own grid) through the batched
    path, in chunks; returns per-curve (best period, SDE max, chi2 array)."""
    best, sde, chi2 = [], [], []
    for c0 in range(0, len(curves), chunk):
        if log and c0 and c0 % (8 * chunk) == 0:
            log(f"searched {c0} of {len(curves)} curves")
        cs = curves[c0:c0 + chunk]
        gs = grids[c0:c0 + chunk]
        off = np.cumsum([0] + [len(c["t"]) for c in cs])
        poff = np.cumsum([0] + [len(g) for g in gs])
        r = gtls.tls_search_batch(ctx, off, np.concatenate([c["t"] for c in cs]),
                                  np.concatenate([c["y"] for c in cs]), np.concatenate([c["dy"] for c in cs]),
                                  poff, np.concatenate(gs), durs, tm, params)
        for k in range(len(cs)):
            best.append(gs[k][r.summaries[k]["best_period"]])
            sde.append(float(r.summaries[k]["sde_max"]))
            chi2.append(r.chi2[poff[k]:poff[k + 1]])
    return np.array(best), np.array(sde), chi2


def views_of(ctx, curves) -> np.ndarray:
    off = np.cumsum([0] + [len(c["t"]) for c in curves])
    return gtls.gtls_cnn_view(ctx, off, np.concatenate([c["t"] for c in curves]),
                              np.concatenate([c["y"] for c in curves]))


def train(ctx, views, labels, steps: int, batch: int = 64, lr: float = 1e-3, seed: int = 0, log=None, net=None):
    """Adam steps on random batches (warm-up over 100 steps, cosine decay);
    a new network from the seeded initialisation unless `net` is given."""
    if net is None:
        net = gtls.Cnn(ctx, synth.cnn_init(seed).astype(np.float32))
    g = synth.rng(seed + 1)
    losses = []
    for s in range(steps):
        idx = g.integers(0, len(views), batch)
        lr_s = lr * min(1.0, (s + 1) / 100) * (0.5 * (1 + math.cos(math.pi * s / steps)))
        losses.append(gtls.gtls_cnn_train_step(net, views[idx], labels[idx], lr=lr_s))
        if log and (s % max(1, steps // 10) == 0 or s == steps - 1):
            log(f"step {s}: loss {np.mean(losses[-50:]):.4f}")
    return net, losses


def recall_at_k(ranked_bins: np.ndarray, labels: np.ndarray) -> float:
    return float(np.mean([labels[i] in set(ranked_bins[i].tolist()) for i in range(len(labels))]))


def run(n_train: int, n_test: int, steps: int, k: int = 32, seed: int = 0, accept: float = 7.0,
        lr: float = 1e-3, batch: int = 64, log=print) -> dict:
    ctx = gtls.Context(0)
    grid, durs, tm = search_inputs()
    log(f"grid {len(grid)} periods, {len(durs)} durations")
    t0 = time.perf_counter()
    train_c = []
    for i in range(n_train):
        train_c.append(training_curve(i, seed))
        if (i + 1) % 8192 == 0:
            log(f"generated {i + 1} training curves")
    test_c = [training_curve(10_000_000 + i, seed) for i in range(n_test)]
    log(f"curves generated in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    tr_best, tr_sde, _ = batched_search(ctx, train_c, [grid] * n_train, durs, tm, log=log)
    log(f"training labels (full-grid searches) in {time.perf_counter() - t0:.1f} s")
    tr_lab = period_bin(tr_best)
    v_tr = views_of(ctx, train_c)
    t0 = time.perf_counter()
    net, losses = train(ctx, v_tr, tr_lab, steps, batch=batch, lr=lr, seed=seed, log=log)
    t_train = time.perf_counter() - t0
    log(f"trained {steps} steps in {t_train:.1f} s")

    # held-out: full search (timed), then view + network + pruned search (timed)
    gtls.gtls_sync(ctx)
    t0 = time.perf_counter()
    te_best, te_sde, _ = batched_search(ctx, test_c, [grid] * n_test, durs, tm)
    t_full = time.perf_counter() - t0
    te_lab = period_bin(te_best)
    # learned: view + network + search of the top-k bins' periods; curves whose
    # pruned search finds no peak of SDE >= accept fall back to the full grid
    t0 = time.perf_counter()
    v_te = views_of(ctx, test_c)
    top = gtls.gtls_cnn_topk(net, v_te, k)
    gbin = period_bin(grid)
    sub = [grid[np.isin(gbin, top[i])] for i in range(n_test)]
    sub = [s if len(s) else grid[:1] for s in sub]
    pr_best, pr_sde, _ = batched_search(ctx, test_c, sub, durs, tm)
    t_pruned = time.perf_counter() - t0
    fall = np.nonzero(pr_sde < accept)[0]
    t0 = time.perf_counter()
    final = pr_best.copy()
    if len(fall):
        fb_best, _, _ = batched_search(ctx, [test_c[i] for i in fall], [grid] * len(fall), durs, tm)
        final[fall] = fb_best
    t_fallback = time.perf_counter() - t0
    # Recall / speed-up trade-off.  A curve that falls back gets exactly the
    # full-grid result, so for any threshold the final best period is known
    # from the two searches already run; the fallback time is the measured
    # full-grid time scaled by the fraction of curves (all test curves have
    # the same length).  Larger k re-runs only the pruned search.
    tradeoff = []
    for kk in sorted({k, 2 * k, 3 * k}):
        if kk == k:
            pb, ps, tp = pr_best, pr_sde, t_pruned
        else:
            t1 = time.perf_counter()
            topk = gtls.gtls_cnn_topk(net, views_of(ctx, test_c), kk)
            subk = [grid[np.isin(gbin, topk[i])] for i in range(n_test)]
            subk = [q if len(q) else grid[:1] for q in subk]
            pb, ps, _ = batched_search(ctx, test_c, subk, durs, tm)
            tp = time.perf_counter() - t1
        for thr in (7.0, 8.0, 9.0, 10.0, 12.0, 15.0, 20.0):
            fb = ps < thr
            fin = np.where(fb, te_best, pb)
            tradeoff.append({"k": kk, "accept_sde": thr, "fallback_fraction": float(fb.mean()),
                             "recall_best_period": float(np.mean(fin == te_best)),
                             "speedup_est": t_full / (tp + fb.mean() * t_full)})
    prior = np.argsort(-np.bincount(tr_lab, minlength=N_BINS), kind="stable")[:k]
    strong = te_sde >= 7.0
    out = {
        "n_train": n_train, "n_test": n_test, "steps": steps, "batch": batch, "lr": lr, "k": k,
        "grid_periods": int(len(grid)),
        "final_loss": float(np.mean(losses[-50:])), "train_seconds": t_train,
        "recall_at_k_net": recall_at_k(top, te_lab),
        "recall_at_k_net_sde7": recall_at_k(top[strong], te_lab[strong]) if strong.any() else None,
        "recall_at_k_prior": recall_at_k(np.tile(prior, (n_test, 1)), te_lab),
        "recall_at_k_prior_sde7": (recall_at_k(np.tile(prior, (int(strong.sum()), 1)), te_lab[strong])
                                   if strong.any() else None),
        "frac_sde7": float(strong.mean()),
        "pruned_grid_fraction": float(np.mean([len(s) for s in sub]) / len(grid)),
        "accept_sde": accept, "fallback_fraction": float(len(fall) / n_test),
        "recall_best_period": float(np.mean(final == te_best)),
        "recall_best_period_sde7": float(np.mean(final[strong] == te_best[strong])) if strong.any() else None,
        "t_full_s": t_full, "t_pruned_s": t_pruned, "t_fallback_s": t_fallback,
        "curves_per_hour_full": 3600.0 * n_test / t_full,
        "curves_per_hour_learned": 3600.0 * n_test / (t_pruned + t_fallback),
        "speedup": t_full / (t_pruned + t_fallback),
        "tradeoff": tradeoff,
    }
    net.close()
    ctx.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--train", type=int, default=8192)
    ap.add_argument("--test", type=int, default=1024)
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--k", type=int, default=32)
    ap.add_argument("--accept", type=float, default=7.0, help="pruned SDE below this falls back to the full grid")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    res = run(a.train, a.test, a.steps, a.k, accept=a.accept, lr=a.lr, batch=a.batch, log=lambda m: print(f"[learned] {m}", file=sys.stderr, flush=True))
    s = json.dumps(res)
    print(s, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(s + "\n")




# --------------------------------------------------------------------------
# The learned proposal on its configured workload: 3000-day curves with the
# 3000-day curve's gaps and noise (synth.proposal_curve), the full Ofir grid
# 0.5-1500 d (418,590 periods), 20 durations, T0 step 0.1, FP64.  Labels are
# the full-grid best periods; the pruned search is compared with the plain
# search and with two proposers that use no network: the prior ranking of the
# training labels' bins, and the coarse first pass of the two-stage search
# (Sect. 2.5: T0 step 0.5 over the grid, then the T0 step 0.1 on the periods
# with the largest coarse SDE).

C4_PMIN, C4_PMAX, C4_DT0 = 0.5, 1500.0, 0.1     # 3000-day curves: period range and T0 step


def c4_inputs():
    span = (int(round(3000.0 / synth.KEPLER_CADENCE_DAYS)) - 1) * synth.KEPLER_CADENCE_DAYS
    grid = gtls.gtls_period_grid_ofir(span, 3.0, pmin_days=C4_PMIN, pmax_days=C4_PMAX)
    durs = gtls.gtls_duration_grid(C4_PMIN, C4_PMAX, 20)
    tm = gtls.gtls_template_quadratic(0.4, 0.25, 0.01, 0.0, 1024)
    return grid, durs, tm


def c4_bin(p) -> np.ndarray:
    """Geometric bin over [0.5, 1500] d, as tls_search_pruned assigns it."""
    b = np.floor(np.log(np.asarray(p) / C4_PMIN) / math.log(C4_PMAX / C4_PMIN) * N_BINS)
    return np.clip(b, 0, N_BINS - 1).astype(np.int32)


def _gen(i):
    return synth.proposal_curve(int(i))


def _curves(indices, workers=8):
    from multiprocessing import get_context
    with get_context("spawn").Pool(workers) as pool:
        return pool.map(_gen, list(indices), chunksize=4)


def _injected_views(ctx, i0: int, count: int, workers: int = 16, chunk: int = 256, log=print):
    """Views and injected-period bins of the curves among [i0, i0 + count)
    that carry a transit (no search: the label is the bin of the injected
    period)."""
    from multiprocessing import get_context
    views, labels = [], []
    with get_context("spawn").Pool(workers) as pool:
        for c0 in range(i0, i0 + count, chunk):
            cs = pool.map(_gen, list(range(c0, min(i0 + count, c0 + chunk))), chunksize=8)
            cs = [c for c in cs if c["meta"]["transit"] is not None]
            if cs:
                views.append(views_of(ctx, cs))
                labels.append(c4_bin([c["meta"]["transit"]["period"] for c in cs]))
            if ((c0 - i0) // chunk) % 8 == 7:
                log(f"pretraining views: {sum(len(v) for v in views)} from {c0 + chunk - i0} curves")
    return np.concatenate(views), np.concatenate(labels)


def c4_label(i0: int, i1: int, out: str, log=print):
    """Full-grid searches of proposal curves [i0, i1): best period index and
    SDE per curve, saved to `out` (npz) as they come."""
    ctx = gtls.Context(0)
    grid, durs, tm = c4_inputs()
    prm = gtls.gtls_params_default(dt0=C4_DT0)
    idx, best, sde = [], [], []
    t0 = time.perf_counter()
    for c0 in range(i0, i1, 32):
        cs = _curves(range(c0, min(i1, c0 + 32)))
        for k, c in enumerate(cs):
            r = gtls.tls_search(ctx, c["t"], c["y"], c["dy"], grid, durs, tm, prm)
            idx.append(c0 + k)
            best.append(r.best_period)
            sde.append(r.sde_max)
        np.savez(out, index=np.array(idx), best=np.array(best), sde=np.array(sde), n_periods=len(grid))
        log(f"labelled {len(idx)} curves in {time.perf_counter() - t0:.0f} s")
    ctx.close()


def c4_eval(label_files, n_test: int, steps: int, batch: int = 64, lr: float = 1e-3, seed: int = 0,
            ks=(32, 64, 128), accepts=(7.0, 10.0, 15.0), refines=(200, 2000, 20000), log=print,
            pretrain: int = 0, pre_steps: int = 0, baselines: bool = True) -> dict:
    """Train on the search labels of `label_files` (after pretraining, when
    `pretrain` > 0, for `pre_steps` steps on the injected-period bins of that
    many further curves, indices from 20,000,000), then score the pruned
    search (and, with `baselines`, the prior-only ranking and the two-stage
    coarse pass) on n_test held-out curves against the full grid."""
    grid, durs, tm = c4_inputs()
    gbin = c4_bin(grid)
    idx, best = [], []
    for f in label_files:
        d = np.load(f)
        assert int(d["n_periods"]) == len(grid)
        idx.extend(d["index"].tolist())
        best.extend(d["best"].tolist())
    order = np.argsort(idx)
    idx, best = np.array(idx)[order], np.array(best)[order]
    labels = gbin[best]
    ctx = gtls.Context(0)
    t0 = time.perf_counter()
    train_views = []
    for c0 in range(0, len(idx), 64):
        cs = _curves(idx[c0:c0 + 64])
        train_views.append(views_of(ctx, cs))
    v_tr = np.concatenate(train_views)
    log(f"{len(idx)} training views in {time.perf_counter() - t0:.0f} s")
    net, n_pre, t_pre = None, 0, 0.0
    if pretrain > 0:
        t0 = time.perf_counter()
        v_pre, l_pre = _injected_views(ctx, 20_000_000, pretrain, log=log)
        n_pre = len(v_pre)
        net, _ = train(ctx, v_pre, l_pre, pre_steps, batch=batch, lr=lr, seed=seed, log=log)
        t_pre = time.perf_counter() - t0
        log(f"pretrained on {n_pre} injected-period views in {t_pre:.0f} s")
    t0 = time.perf_counter()
    net, losses = train(ctx, v_tr, labels, steps, batch=batch, lr=lr, seed=seed, log=log, net=net)
    t_train = time.perf_counter() - t0
    prior = np.argsort(-np.bincount(labels, minlength=N_BINS), kind="stable")
    prm = gtls.gtls_params_default(dt0=C4_DT0)
    coarse_prm = gtls.gtls_params_default(dt0=0.5)
    rec = []
    test = _curves(range(10_000_000, 10_000_000 + n_test))
    for i, c in enumerate(test):
        r = {}
        t1 = time.perf_counter()
        full = gtls.tls_search(ctx, c["t"], c["y"], c["dy"], grid, durs, tm, prm)
        r["t_full"] = time.perf_counter() - t1
        r["best"] = int(full.best_period)
        r["sde"] = float(full.sde_max)
        for k in ks:
            t1 = time.perf_counter()
            res, searched, fell = gtls.tls_search_pruned(ctx, net, c["t"], c["y"], c["dy"], grid, durs, tm, C4_PMIN,
                                                         C4_PMAX, k, -1e300, prm)
            r[f"net{k}"] = (int(res.best_period), float(res.sde_max), time.perf_counter() - t1,
                            float(searched.mean()), bool(searched[r["best"]]))
            if not baselines:
                continue
            sub = np.nonzero(np.isin(gbin, prior[:k]))[0]
            t1 = time.perf_counter()
            pr = gtls.tls_search(ctx, c["t"], c["y"], c["dy"], grid[sub], durs, tm, prm)
            r[f"prior{k}"] = (int(sub[pr.best_period]), float(pr.sde_max), time.perf_counter() - t1,
                              len(sub) / len(grid), bool(np.isin(r["best"], sub)))
        t1 = time.perf_counter()
        co = gtls.tls_search(ctx, c["t"], c["y"], c["dy"], grid, durs, tm, coarse_prm) if baselines else None
        t_coarse = time.perf_counter() - t1
        for nref in (refines if baselines else ()):
            t1 = time.perf_counter()
            top = np.sort(np.argsort(-co.sde, kind="stable")[:nref])
            fine = gtls.tls_search(ctx, c["t"], c["y"], c["dy"], grid[top], durs, tm, prm)
            chi2 = co.chi2.copy()
            chi2[top] = fine.chi2
            _, _, _, b2 = gtls.tls_sde(ctx, chi2, 91)
            r[f"two{nref}"] = (int(b2), t_coarse + time.perf_counter() - t1, bool(np.isin(r["best"], top)))
        rec.append(r)
        if (i + 1) % 16 == 0:
            log(f"evaluated {i + 1} of {n_test} test curves")
    t_full = float(np.mean([r["t_full"] for r in rec]))
    best_full = np.array([r["best"] for r in rec])
    strong = np.array([r["sde"] >= 7.0 for r in rec])
    rows = []
    for name in [f"net{k}" for k in ks] + ([f"prior{k}" for k in ks] if baselines else []):
        b = np.array([r[name][0] for r in rec])
        s = np.array([r[name][1] for r in rec])
        tt = np.array([r[name][2] for r in rec])
        frac = float(np.mean([r[name][3] for r in rec]))
        inside = float(np.mean([r[name][4] for r in rec]))
        for thr in accepts:
            fb = s < thr
            fin = np.where(fb, best_full, b)
            t = float(np.mean(tt + fb * np.array([r["t_full"] for r in rec])))
            rows.append({"method": name, "accept_sde": thr, "grid_fraction": frac, "best_inside": inside,
                         "fallback": float(fb.mean()), "recall": float(np.mean(fin == best_full)),
                         "recall_sde7": float(np.mean((fin == best_full)[strong])) if strong.any() else None,
                         "s_per_curve": t, "speedup": t_full / t})
    for nref in (refines if baselines else ()):
        b = np.array([r[f"two{nref}"][0] for r in rec])
        t = float(np.mean([r[f"two{nref}"][1] for r in rec]))
        rows.append({"method": f"two_stage_top{nref}", "accept_sde": None, "grid_fraction": nref / len(grid),
                     "best_inside": float(np.mean([r[f"two{nref}"][2] for r in rec])), "fallback": 0.0,
                     "recall": float(np.mean(b == best_full)),
                     "recall_sde7": float(np.mean((b == best_full)[strong])) if strong.any() else None,
                     "s_per_curve": t, "speedup": t_full / t})
    out = {"workload": "proposal_3000d", "n_train": int(len(idx)), "n_test": n_test, "steps": steps, "batch": batch,
           "lr": lr, "grid_periods": int(len(grid)), "final_loss": float(np.mean(losses[-50:])),
           "train_seconds": t_train, "t_full_s_per_curve": t_full, "frac_test_sde7": float(strong.mean()),
           "pretrain_views": n_pre, "pretrain_steps": pre_steps if pretrain > 0 else 0, "pretrain_seconds": t_pre,
           "rows": rows}
    net.close()
    ctx.close()
    return out


def c4_main(argv=None):
    ap = argparse.ArgumentParser(description="learned proposal on 3000-day curves")
    ap.add_argument("mode", choices=["label", "eval"])
    ap.add_argument("--start", type=int, default=0)
    ap.add_argument("--stop", type=int, default=64)
    ap.add_argument("--out", required=True)
    ap.add_argument("--labels", nargs="*", default=[])
    ap.add_argument("--test", type=int, default=64)
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--pretrain", type=int, default=0, help="eval: curves for injected-period pretraining")
    ap.add_argument("--pre-steps", type=int, default=2000)
    ap.add_argument("--no-baselines", action="store_true", help="eval: score the network only")
    a = ap.parse_args(argv)
    log = lambda m: print(f"[learned-c4] {m}", file=sys.stderr, flush=True)
    if a.mode == "label":
        c4_label(a.start, a.stop, a.out, log)
    else:
        res = c4_eval(a.labels, a.test, a.steps, a.batch, a.lr, log=log, pretrain=a.pretrain,
                      pre_steps=a.pre_steps, baselines=not a.no_baselines)
        s = json.dumps(res)
        print(s, flush=True)
        with open(a.out, "w") as f:
            f.write(s + "\n")


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] in ("label", "eval"):
        c4_main()
    else:
        main()
