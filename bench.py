#!/usr/bin/env python
"""TLS search throughput on one MI355X: (period x duration x phase) evals/s.

One step = one complete search of one light curve (fold, sort, padding,
template slide with per-window depth fit and chi2, per-period minimum, SDE
periodogram) with all inputs already in device memory.  The default workload
is the 3000-day Kepler-like curve (29.4-min cadence, ~132k points after 10 %
gaps, 100 ppm white + 30 ppm red noise, one Earth-like transit) searched over
its Ofir period grid 0.5-1500 d at oversampling 3 with 20 durations.

Prints one JSON line (rank 0).  Per-stage kernel times come from HIP events
the library records on its launch stream around each kernel during the timed
steps; the roofline object reports the stage that takes the most time.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E
METRIC = "TLS (period×duration×phase) evals/s"


def workload(name: str):
    from paper_2607_00348_amd import gtls, synth
    if name == "kepler_3000d":
        c = synth.curve_3000d()
        span = c["t"][-1] - c["t"][0]
        periods = gtls.gtls_period_grid_ofir(span, 3.0, pmin_days=0.5, pmax_days=1500.0)
        durs = gtls.gtls_duration_grid(0.5, 1500.0, 20)
    elif name == "kepler_90d":
        c = synth.curve_90d()
        span = c["t"][-1] - c["t"][0]
        periods = gtls.gtls_period_grid_ofir(span, 3.0, pmin_days=0.5, pmax_days=45.0)
        durs = gtls.gtls_duration_grid(0.5, 45.0, 12)
    elif name == "tess_13sector":
        c = synth.curve_tess()
        span = c["t"][-1] - c["t"][0]
        periods = gtls.gtls_period_grid_ofir(span, 3.0, pmax_days=175.0)
        durs = gtls.gtls_duration_grid(periods[0], periods[-1], 20)
    else:
        raise SystemExit(f"unknown workload {name}")
    tm = gtls.gtls_template_quadratic(0.4, 0.25, 0.01, 0.0, 1024)
    return c, periods, durs, tm


def host_threads():
    """Threads the oracle baseline uses: every core this process may run on
    (its CPU affinity), capped by OMP_NUM_THREADS when that is set (the GPU
    hosts give one GPU's job a fixed share of their cores that way)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        avail = min(avail, int(cap))
    return max(1, avail)


def cpu_baseline(c, periods, durs, tm, prm, n_sample: int, seed: int = 0):
    """The oracle, as it stands, on a seeded sample of the workload's periods."""
    from oracle import oracle as O
    threads = host_threads()
    g = np.random.Generator(np.random.PCG64(seed))
    idx = np.sort(g.choice(len(periods), size=min(n_sample, len(periods)), replace=False))
    t0 = time.perf_counter()
    r = O.tls_search(c["t"], c["y"], c["dy"], periods[idx], durs, tm, dt0=prm.dt0, envelope=prm.envelope,
                     k_min=prm.k_min, k_max=prm.k_max, q_cap=prm.q_cap, depth_mode=prm.depth_mode,
                     threads=threads)
    el = time.perf_counter() - t0
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return {"value": r.n_evals / el, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "nproc": os.cpu_count(), "affinity_cores": affinity,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS"),
            "sample": f"{len(idx)} of {len(periods)} periods (seeded uniform sample), same curve, durations "
                      f"and dt0; {r.n_evals} windows in {el:.1f} s on {threads} threads (all cores this "
                      f"process may use, capped by OMP_NUM_THREADS)"}


def survey_bench(args):
    """Batched survey: a seeded sample of the 4096-curve Kepler-like survey
    (lengths 4k-147k cadences, sigma 50-2000 ppm, 10 % injected), each curve
    on its own default grid (Roche limit to half the baseline, oversampling
    3), 20 shared durations, searched by one persistent launch per batch."""
    import torch

    from paper_2607_00348_amd import gtls, synth
    g = np.random.Generator(np.random.PCG64(17))
    idx = np.sort(g.choice(4096, size=args.curves, replace=False))
    curves = [synth.survey_curve(int(i)) for i in idx]
    grids = []
    for c in curves:
        span = c["t"][-1] - c["t"][0]
        grids.append(gtls.gtls_period_grid_ofir(span, 3.0))
    durs = gtls.gtls_duration_grid(float(min(gr[0] for gr in grids)), 1500.0, 20)
    tm = gtls.gtls_template_quadratic(0.4, 0.25, 0.01, 0.0, 1024)
    route = {} if args.route_min is None else {"batch_route_min": args.route_min}
    prm = gtls.gtls_params_default(dt0=args.dt0,
                                   precision=(gtls.GTLS_FP32C if args.precision == "fp32c" else gtls.GTLS_FP64),
                                   **route)
    off = np.cumsum([0] + [len(c["t"]) for c in curves])
    poff = np.cumsum([0] + [len(gr) for gr in grids])
    dev = torch.device("cuda:0")
    f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    cat = lambda k: np.concatenate([c[k] for c in curves])
    t_d, y_d, dy_d = f64(cat("t")), f64(cat("y")), f64(cat("dy"))
    p_d, d_d, tm_d = f64(np.concatenate(grids)), f64(durs), f64(tm)
    npd = int(poff[-1])
    outs = {k: torch.empty(npd, dtype=torch.float64, device=dev) for k in ("chi2", "depth", "t0", "sr", "raw", "sde")}
    bd = torch.empty(npd, dtype=torch.int32, device=dev)
    bs = torch.empty(npd, dtype=torch.int32, device=dev)
    summ = torch.zeros(len(curves) * 5, dtype=torch.int64, device=dev)
    ctx = gtls.Context(0, torch.cuda.current_stream().cuda_stream)

    # curves per batched call: all by default; with --chunk, consecutive chunks (each a batched call of its own,
    # a progress line after each)
    chunk = args.chunk if args.chunk > 0 else len(curves)

    def step():
        for c0 in range(0, len(curves), chunk):
            c1 = min(len(curves), c0 + chunk)
            o = off[c0:c1 + 1] - off[c0]
            po = poff[c0:c1 + 1] - poff[c0]
            pt = lambda x, k: x.data_ptr() + int(k) * x.element_size()
            gtls.tls_search_batch_dev(ctx, o, pt(t_d, off[c0]), pt(y_d, off[c0]), pt(dy_d, off[c0]), po,
                                      pt(p_d, poff[c0]), d_d.data_ptr(), len(durs), tm_d.data_ptr(), len(tm), prm,
                                      pt(outs["chi2"], poff[c0]), pt(bd, poff[c0]), pt(bs, poff[c0]),
                                      pt(outs["depth"], poff[c0]), pt(outs["t0"], poff[c0]), pt(outs["sr"], poff[c0]),
                                      pt(outs["raw"], poff[c0]), pt(outs["sde"], poff[c0]), pt(summ, 5 * c0))
            if chunk < len(curves):
                torch.cuda.synchronize()
                print(f"[bench] survey: {c1} of {len(curves)} curves searched", file=sys.stderr, flush=True)

    print(f"[bench] survey sample: {len(curves)} curves, {off[-1]} points, {npd} (curve, period) items",
          file=sys.stderr, flush=True)
    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    sm = summ.cpu().numpy().reshape(len(curves), 5)
    n_evals = int(sm[:, 2].sum())
    line = {"metric": "light curves/hr (batched survey)", "value": len(curves) / el * 3600.0,
            "unit": "light curves/hr", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": el * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if args.precision == "fp64" else "f32", "data": "synthetic",
            "config": {"workload": "kepler_survey_sample", "curves": len(curves), "points": int(off[-1]),
                       "items": npd, "durations": len(durs), "dt0": args.dt0, "precision": args.precision,
                       "route_min": int(prm.batch_route_min), "curves_per_call": chunk},
            "evals_per_s": n_evals / el}
    ctx.close()
    print(json.dumps(line), flush=True)


def cnn_bench(args):
    """Training throughput of the period-proposal network: Adam steps of batch
    256 on seeded 4096-bin views (the BF16 MFMA forward and backward kernels,
    the head, the loss and the update), then top-k inference."""
    from paper_2607_00348_amd import gtls, synth
    batch = 256
    g = np.random.Generator(np.random.PCG64(23))
    views = g.normal(0.0, 1.0, (batch, gtls.CNN_VIEW)).astype(np.float32)
    labels = g.integers(0, gtls.CNN_BINS, batch).astype(np.int32)
    ctx = gtls.Context(0)
    net = gtls.Cnn(ctx, synth.cnn_init(0).astype(np.float32))
    for w in range(args.warmup):
        gtls.gtls_cnn_train_step(net, views, labels, lr=1e-3)
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gtls.gtls_cnn_train_step(net, views, labels, lr=1e-3)
    el = (time.perf_counter() - t0) / args.steps
    t1 = time.perf_counter()
    gtls.gtls_cnn_topk(net, views, 32)
    inf = time.perf_counter() - t1
    # forward + backward flops of the convolutions: 2 * B * L * 32 * (C_in * 7) per layer, x3 with backward
    conv_flops = sum(2.0 * batch * gtls.CNN_VIEW * 32 * (cin * 7) for cin in (1, 32, 32, 32, 32))
    line = {"metric": "CNN training samples/s", "value": batch / el, "unit": "samples/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": el * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
            "config": {"workload": "cnn_train", "batch": batch, "view": gtls.CNN_VIEW, "bins": gtls.CNN_BINS},
            "inference_ms_per_batch": inf * 1e3, "conv_tflops_fwd_bwd": 3.0 * conv_flops / el / 1e12}
    net.close()
    ctx.close()
    print(json.dumps(line), flush=True)


def sort_bytes(n: int, periods, durs, prm) -> float:
    """Algorithmic HBM bytes of the fold + sort + pad stage for one search:
    per element-period 8 B of t, the packed 8-byte (key, index) word written
    by the top-digit pass and read and written again by the LDS-tile pass
    (24 B), and the padded residuals, 8 B (4 B in FP32C) per position over
    n + D_max(P) positions, plus the 16 B (8 B) prefix sums in MEAN mode
    (per-point weights, absent from these workloads, would add as much again
    as the residuals)."""
    dmax = _valid_d(n, periods, durs, prm).max(axis=1)
    es = 4.0 if prm.precision == 1 else 8.0
    per_pos = es + ((8.0 if prm.precision == 1 else 16.0) if prm.depth_mode == 1 else 0.0)
    return float(np.sum(8.0 * n + 24.0 * n + per_pos * (n + dmax)))


def _valid_d(n: int, periods, durs, prm):
    """Points per window D for every (period, duration), 0 where the
    duration is outside the period's envelope."""
    p = np.asarray(periods)[:, None]
    q = np.asarray(durs)[None, :] / p
    ps = p * 86400.0
    ok = q <= prm.q_cap
    if prm.envelope:
        ok &= (q ** 3 * ps ** 2 >= prm.k_min ** 3) & (q ** 3 * ps ** 2 <= prm.k_max ** 3)
    d = np.clip(np.floor(n * q + 0.5), 1, n)
    return np.where(ok, d, 0).astype(np.int64)


def strided_mac_count(n: int, periods, durs, prm) -> float:
    """Multiply-adds of the strided items (T0 stride >= 2): windows x D."""
    d = _valid_d(n, periods, durs, prm)
    s = np.maximum(1, np.floor(prm.dt0 * d)).astype(np.int64)
    use = (d > 0) & (s >= 2)
    nw = (n + s - 1) // np.maximum(s, 1)
    return float(np.sum(np.where(use, nw * d, 0)))


def measured_traffic(kernel: str, args):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload (FETCH_SIZE and WRITE_SIZE, each scaled by the
    factor a plain copy of known size gives), or None when there is none or
    the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        f"traffic_{args.workload}_dt0_{args.dt0:g}_{args.precision}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2607_00348_amd", "csrc", "kernels.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec.get("kernels_hip_sha256"):
        return None
    k = rec["kernels"].get(kernel)
    if not k:
        return None
    return k["fetch_kib_per_launch"] * 1024 * rec["fetch_factor"] + k["write_kib_per_launch"] * 1024 * rec["write_factor"]


def copy_probe(nbytes: int):
    """A plain device-to-device copy of a known size (calibrates the HBM
    byte counters of a profiler against an exactly known traffic)."""
    import torch
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "copies": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="kepler_3000d",
                    choices=["kepler_3000d", "kepler_90d", "tess_13sector", "survey", "cnn_train"])
    ap.add_argument("--curves", type=int, default=32, help="survey sample size (--workload survey)")
    ap.add_argument("--chunk", type=int, default=0,
                    help="survey: curves per batched call (default: the whole sample in one call)")
    ap.add_argument("--route-min", type=int, default=None,
                    help="survey: curves of at least this many points go through the single-curve kernels "
                         "(default: the library's, 3000; 0: all in the persistent launch)")
    ap.add_argument("--dt0", type=float, default=0.1)
    ap.add_argument("--depth-mode", choices=["wls", "mean"], default="wls")
    ap.add_argument("--precision", choices=["fp64", "fp32c"], default="fp64")
    ap.add_argument("--cpu-sample", type=int, default=12000, help="periods the oracle baseline runs on")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a device copy of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only (the single-GPU kernel path; sharding periods across GPUs is a "
              "design, not measured here); use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "survey":
        survey_bench(args)
        return
    if args.workload == "cnn_train":
        cnn_bench(args)
        return

    import torch

    from paper_2607_00348_amd import gtls

    c, periods, durs, tm = workload(args.workload)
    prm = gtls.gtls_params_default(dt0=args.dt0, depth_mode=(1 if args.depth_mode == "mean" else 0),
                                   precision=(gtls.GTLS_FP32C if args.precision == "fp32c" else gtls.GTLS_FP64))
    dev = torch.device("cuda:0")
    f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    t_d, y_d, dy_d = f64(c["t"]), f64(c["y"]), f64(c["dy"])
    p_d, d_d, tm_d = f64(periods), f64(durs), f64(tm)
    npd = len(periods)
    outs = {k: torch.empty(npd, dtype=torch.float64, device=dev) for k in ("chi2", "depth", "t0", "sr", "raw", "sde")}
    bdur = torch.empty(npd, dtype=torch.int32, device=dev)
    bst = torch.empty(npd, dtype=torch.int32, device=dev)
    summary = torch.zeros(5, dtype=torch.int64, device=dev)     # gtls_summary, 40 bytes
    stream = torch.cuda.current_stream()
    ctx = gtls.Context(0, stream.cuda_stream)

    def step():
        gtls.tls_search_dev(ctx, t_d.data_ptr(), y_d.data_ptr(), dy_d.data_ptr(), len(c["t"]), p_d.data_ptr(), npd,
                            d_d.data_ptr(), len(durs), tm_d.data_ptr(), len(tm), prm, outs["chi2"].data_ptr(),
                            bdur.data_ptr(), bst.data_ptr(), outs["depth"].data_ptr(), outs["t0"].data_ptr(),
                            outs["sr"].data_ptr(), outs["raw"].data_ptr(), outs["sde"].data_ptr(),
                            summary.data_ptr())

    print(f"[bench] workload {args.workload}: n={len(c['t'])} periods={npd} durations={len(durs)} "
          f"dt0={args.dt0}", file=sys.stderr, flush=True)
    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    gtls.gtls_profile_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = gtls.gtls_profile_read(ctx)
    gtls.gtls_profile_enable(ctx, False)
    summ = summary.cpu().numpy().view(np.uint8)
    chi2_null, sde_max = np.frombuffer(summ[:16].tobytes(), dtype=np.float64)
    n_evals, n_macs = np.frombuffer(summ[16:32].tobytes(), dtype=np.int64)
    best_period = int(np.frombuffer(summ[32:36].tobytes(), dtype=np.int32)[0])
    ms_per_step = el / args.steps * 1e3
    evals_per_s = float(n_evals) / (el / args.steps)
    print(f"[bench] {args.steps} steps in {el:.3f} s; best period {periods[best_period]:.6f} d "
          f"SDE {sde_max:.2f}; evals/step {n_evals}; macs/step {n_macs}", file=sys.stderr, flush=True)
    for k, (ms, nl) in prof.items():
        print(f"[bench] stage {k:10s} {ms / args.steps:10.3f} ms/step  {nl // args.steps} launches/step",
              file=sys.stderr, flush=True)

    # Roofline of the kernel stage with the largest share of kernel time.
    stage = max(prof, key=lambda k: prof[k][0])
    stage_ms = prof[stage][0] / args.steps
    launches = max(1, prof[stage][1] // args.steps)
    per_launch_ms = stage_ms / launches
    strided_macs = strided_mac_count(len(c["t"]), periods, durs, prm)
    if stage in ("slide", "slide_strided"):
        macs = strided_macs if stage == "slide_strided" else float(n_macs) - strided_macs
        flops = 2.0 * macs / launches                     # one multiply-add per template point per window
        achieved = flops / (per_launch_ms * 1e-3) / 1e12
        kernel = "k_slide_rows" if stage == "slide_strided" else "k_slide_unit"
        roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS, "traffic": measured_traffic(kernel, args),
                "kernel": kernel, "per_launch_ms": per_launch_ms, "flops_per_launch": flops}
    else:
        byts = sort_bytes(len(c["t"]), periods, durs, prm) / launches
        achieved = byts / (per_launch_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": measured_traffic("k_fold_sort", args),
                "kernel": "k_fold_sort", "per_launch_ms": per_launch_ms, "bytes_per_launch": byts}

    line = {"metric": METRIC, "value": evals_per_s, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32", "data": "synthetic",
            "config": {"workload": args.workload, "n_points": int(len(c["t"])), "n_periods": int(npd),
                       "n_durations": int(len(durs)), "dt0": args.dt0, "depth_mode": args.depth_mode,
                       "precision": args.precision},
            "light_curves_per_hour": 3600.0 / (ms_per_step * 1e-3),
            "stage_ms_per_step": {k: v[0] / args.steps for k, v in prof.items()},
            "roofline": roof}
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(c, periods, durs, tm, prm, args.cpu_sample)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
