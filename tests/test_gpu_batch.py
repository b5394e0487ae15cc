"""GPU tests of the batched survey path (one persistent launch over many
curves; optionally, curves above batch_route_min points through the
single-curve kernels): every curve's results must equal, bit for bit, the
single-curve search of that curve (itself bit-exact against the oracle),
including ragged lengths, per-point errors, strided T0 grids, the
moving-average depth and the FP32C mode; batches split between the two
routes match the oracle; the captured graph must give the same results on
every replay."""
import os

import numpy as np
import pytest

from paper_2607_00348_amd import gtls, synth

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def ctx():
    c = gtls.Context(0)
    yield c
    c.close()


def _curves(seed, count, n_lo, n_hi, varying_every=0):
    out = []
    for k in range(count):
        c = synth.curve_random(seed * 100 + k, n_min=n_lo, n_max=n_hi, inject=(k % 3 == 0),
                               varying_dy=bool(varying_every and k % varying_every == 1))
        out.append(c)
    return out


def _pack(oracle, curves, nper=120):
    offs, poffs, grids = [0], [0], []
    for c in curves:
        span = c["t"].max() - c["t"].min()
        g = oracle.period_grid_ofir(span, 2.0, pmin_days=0.5, pmax_days=max(0.6, span / 2))
        if len(g) > nper:
            g = g[np.linspace(0, len(g) - 1, nper).astype(int)]
        grids.append(g)
        offs.append(offs[-1] + len(c["t"]))
        poffs.append(poffs[-1] + len(g))
    cat = lambda k: np.concatenate([c[k] for c in curves])
    return (np.array(offs), cat("t"), cat("y"), cat("dy"), np.array(poffs), np.concatenate(grids), grids)


def _check_against_single(ctx, curves, packed, durs, tm, prm, res):
    offs, t, y, dy, poffs, periods, grids = packed
    for k, c in enumerate(curves):
        one = gtls.tls_search(ctx, c["t"], c["y"], c["dy"], grids[k], durs, tm, prm)
        sl = slice(poffs[k], poffs[k + 1])
        label = f"curve {k} n={len(c['t'])}"
        assert np.array_equal(res.chi2[sl], one.chi2), label
        assert np.array_equal(res.best_dur[sl], one.best_dur), label
        assert np.array_equal(res.best_start[sl], one.best_start), label
        assert np.array_equal(res.depth[sl], one.depth), label
        assert np.array_equal(np.isnan(res.t0[sl]), np.isnan(one.t0)), label
        ok = ~np.isnan(one.t0)
        assert np.array_equal(res.t0[sl][ok], one.t0[ok]), label
        assert np.array_equal(res.sde[sl], one.sde), label
        s = res.summaries[k]
        assert s["best_period"] == one.best_period and s["sde_max"] == one.sde_max, label
        assert s["chi2_null"] == one.chi2_null and s["n_evals"] == one.n_evals and s["n_macs"] == one.n_macs


@pytest.mark.parametrize("kw,varying", [(dict(), 0), (dict(dt0=0.1), 0), (dict(depth_mode=1), 4),
                                        (dict(dt0=0.05, depth_mode=1), 0), (dict(precision=1), 3),
                                        (dict(precision=1, dt0=0.2), 0)])
def test_batch_equals_single_curve(ctx, oracle, kw, varying):
    curves = _curves(7 + len(kw) + varying, 9, 300, 9000, varying)
    packed = _pack(oracle, curves)
    durs = oracle.duration_grid(0.5, 100.0, 12)
    tm = oracle.template_quadratic(0.4, 0.25, 0.02, 0.0, 256)
    prm = gtls.gtls_params_default(batch_route_min=0, **kw)
    offs, t, y, dy, poffs, periods, grids = packed
    print("batch", kw, [len(c["t"]) for c in curves], flush=True)
    res = gtls.tls_search_batch(ctx, offs, t, y, dy, poffs, periods, durs, tm, prm)
    _check_against_single(ctx, curves, packed, durs, tm, prm, res)
    # replay: same arguments, the cached graph runs again
    again = gtls.tls_search_batch(ctx, offs, t, y, dy, poffs, periods, durs, tm, prm)
    assert np.array_equal(again.chi2, res.chi2) and np.array_equal(again.best_start, res.best_start)


def test_batch_matches_oracle(ctx, oracle):
    curves = _curves(31, 4, 500, 3000)
    packed = _pack(oracle, curves, nper=60)
    durs = oracle.duration_grid(0.5, 100.0, 10)
    tm = oracle.template_quadratic(0.4, 0.25, 0.02, 0.0, 128)
    offs, t, y, dy, poffs, periods, grids = packed
    print("batch vs oracle", flush=True)
    res = gtls.tls_search_batch(ctx, offs, t, y, dy, poffs, periods, durs, tm, gtls.gtls_params_default(batch_route_min=0))
    for k, c in enumerate(curves):
        ref = oracle.tls_search(c["t"], c["y"], c["dy"], grids[k], durs, tm, threads=THREADS)
        sl = slice(poffs[k], poffs[k + 1])
        assert np.allclose(res.chi2[sl], ref.chi2, rtol=1e-9, atol=0)
        assert np.array_equal(res.best_dur[sl], ref.best_dur)
        assert np.array_equal(res.best_start[sl], ref.best_start)
        assert res.summaries[k]["best_period"] == oracle.sde(ref.chi2)[3]


@pytest.mark.parametrize("dt0", [0.0, 0.1])
def test_routed_batch_matches_oracle(ctx, oracle, dt0):
    """batch_route_min = 6000: short curves (persistent launch) and long ones
    (single-curve kernels) in one call, interleaved, against the oracle curve
    by curve; the same call without routing gives identical results."""
    lengths = [700, 7000, 1500, 6000, 5999, 9000]
    curves = [synth.curve_random(900 + k, n=n, inject=(k % 2 == 0)) for k, n in enumerate(lengths)]
    packed = _pack(oracle, curves, nper=40)
    durs = oracle.duration_grid(0.5, 100.0, 10)
    tm = oracle.template_quadratic(0.4, 0.25, 0.02, 0.0, 128)
    offs, t, y, dy, poffs, periods, grids = packed
    print("mixed batch vs oracle", lengths, dt0, flush=True)
    prm = gtls.gtls_params_default(dt0=dt0, batch_route_min=6000)
    res = gtls.tls_search_batch(ctx, offs, t, y, dy, poffs, periods, durs, tm, prm)
    for k, c in enumerate(curves):
        ref = oracle.tls_search(c["t"], c["y"], c["dy"], grids[k], durs, tm, dt0=dt0, threads=THREADS)
        sl = slice(poffs[k], poffs[k + 1])
        label = f"curve {k} n={len(c['t'])}"
        assert np.allclose(res.chi2[sl], ref.chi2, rtol=1e-9, atol=0), label
        assert np.array_equal(res.best_dur[sl], ref.best_dur), label
        assert np.array_equal(res.best_start[sl], ref.best_start), label
        _, _, sde, best = oracle.sde(ref.chi2)
        assert np.allclose(res.sde[sl], sde, rtol=1e-9, atol=1e-12), label
        assert res.summaries[k]["best_period"] == best and res.summaries[k]["n_evals"] == ref.n_evals, label
    again = gtls.tls_search_batch(ctx, offs, t, y, dy, poffs, periods, durs, tm, prm)
    assert np.array_equal(again.chi2, res.chi2) and np.array_equal(again.sde, res.sde)
    whole = gtls.tls_search_batch(ctx, offs, t, y, dy, poffs, periods, durs, tm,
                                  gtls.gtls_params_default(dt0=dt0, batch_route_min=0))
    for k in ("chi2", "best_dur", "best_start", "depth", "sde"):
        assert np.array_equal(getattr(whole, k), getattr(res, k)), k
    for k in ("chi2_null", "sde_max", "n_evals", "n_macs", "best_period"):
        assert np.array_equal(whole.summaries[k], res.summaries[k]), k


def test_batch_graph_replays_on_device_buffers(ctx, oracle):
    """Device-pointer variant: the graph is captured on the first call and
    replayed on later ones; eager GPU work and synchronisations run between
    replays and every replay must equal the first result."""
    import torch
    curves = _curves(41, 6, 1000, 6000)
    packed = _pack(oracle, curves, nper=80)
    offs, t, y, dy, poffs, periods, grids = packed
    durs = oracle.duration_grid(0.5, 100.0, 10)
    tm = oracle.template_quadratic(0.4, 0.25, 0.02, 0.0, 128)
    dev = torch.device("cuda:0")
    f = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    t_d, y_d, dy_d, p_d, d_d, tm_d = f(t), f(y), f(dy), f(periods), f(durs), f(tm)
    npd = len(periods)
    outs = {k: torch.empty(npd, dtype=torch.float64, device=dev) for k in ("chi2", "depth", "t0", "sr", "raw", "sde")}
    bd = torch.empty(npd, dtype=torch.int32, device=dev)
    bs = torch.empty(npd, dtype=torch.int32, device=dev)
    summ = torch.zeros(len(curves) * 5, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    dctx = gtls.Context(0, stream.cuda_stream)
    prm = gtls.gtls_params_default(batch_route_min=0)      # every curve in the captured persistent launch
    first = None
    for rep in range(4):
        print("graph replay", rep, flush=True)
        gtls.tls_search_batch_dev(dctx, offs, t_d.data_ptr(), y_d.data_ptr(), dy_d.data_ptr(), poffs,
                                  p_d.data_ptr(), d_d.data_ptr(), len(durs), tm_d.data_ptr(), len(tm), prm,
                                  outs["chi2"].data_ptr(), bd.data_ptr(), bs.data_ptr(), outs["depth"].data_ptr(),
                                  outs["t0"].data_ptr(), outs["sr"].data_ptr(), outs["raw"].data_ptr(),
                                  outs["sde"].data_ptr(), summ.data_ptr())
        torch.cuda.synchronize()
        got = (outs["chi2"].cpu().numpy().copy(), bs.cpu().numpy().copy(), outs["sde"].cpu().numpy().copy())
        if first is None:
            first = got
            ref = gtls.tls_search_batch(ctx, offs, t, y, dy, poffs, periods, durs, tm, prm)
            assert np.array_equal(first[0], ref.chi2) and np.array_equal(first[1], ref.best_start)
        else:
            for a, b in zip(first, got):
                assert np.array_equal(a, b)
        # eager work between replays, overwriting the outputs
        outs["chi2"].fill_(-1.0)
        bs.zero_()
        (torch.randn(1000, device=dev) * 2).sum().item()
    dctx.close()


def test_batch_graph_key_covers_params_and_outputs(ctx, oracle):
    """A second device-pointer call on the same context that changes only
    the duration envelope (q_cap, k_max) and writes into freshly allocated
    outputs (the first call's outputs kept alive) must capture a new graph:
    its results equal a fresh context's search with the new parameters, and
    the first call's outputs stay untouched."""
    import torch
    curves = _curves(43, 5, 800, 5000)
    packed = _pack(oracle, curves, nper=60)
    offs, t, y, dy, poffs, periods, grids = packed
    durs = oracle.duration_grid(0.5, 100.0, 10)
    tm = oracle.template_quadratic(0.4, 0.25, 0.02, 0.0, 128)
    dev = torch.device("cuda:0")
    f = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    t_d, y_d, dy_d, p_d, d_d, tm_d = f(t), f(y), f(dy), f(periods), f(durs), f(tm)
    npd = len(periods)

    def outputs():
        o = {k: torch.empty(npd, dtype=torch.float64, device=dev) for k in ("chi2", "depth", "t0", "sr", "raw", "sde")}
        o["bd"] = torch.empty(npd, dtype=torch.int32, device=dev)
        o["bs"] = torch.empty(npd, dtype=torch.int32, device=dev)
        o["summ"] = torch.zeros(len(curves) * 5, dtype=torch.int64, device=dev)
        return o

    def run(dctx, prm, o):
        gtls.tls_search_batch_dev(dctx, offs, t_d.data_ptr(), y_d.data_ptr(), dy_d.data_ptr(), poffs,
                                  p_d.data_ptr(), d_d.data_ptr(), len(durs), tm_d.data_ptr(), len(tm), prm,
                                  o["chi2"].data_ptr(), o["bd"].data_ptr(), o["bs"].data_ptr(),
                                  o["depth"].data_ptr(), o["t0"].data_ptr(), o["sr"].data_ptr(),
                                  o["raw"].data_ptr(), o["sde"].data_ptr(), o["summ"].data_ptr())
        torch.cuda.synchronize()
        return o["chi2"].cpu().numpy().copy(), o["bd"].cpu().numpy().copy(), o["bs"].cpu().numpy().copy()

    stream = torch.cuda.current_stream()
    dctx = gtls.Context(0, stream.cuda_stream)
    p1 = gtls.gtls_params_default(dt0=0.1, batch_route_min=0)
    p2 = gtls.gtls_params_default(dt0=0.1, q_cap=0.05, k_max=300.0, batch_route_min=0)
    o1 = outputs()
    print("graph key: first call", flush=True)
    first = run(dctx, p1, o1)
    o2 = outputs()
    print("graph key: second call, new envelope and outputs", flush=True)
    second = run(dctx, p2, o2)
    dctx.close()
    ref1 = gtls.tls_search_batch(ctx, offs, t, y, dy, poffs, periods, durs, tm, p1)
    fresh = gtls.Context(0)
    ref2 = gtls.tls_search_batch(fresh, offs, t, y, dy, poffs, periods, durs, tm, p2)
    fresh.close()
    assert not np.array_equal(ref1.best_dur, ref2.best_dur)       # the envelope change matters
    assert np.array_equal(second[0], ref2.chi2)
    assert np.array_equal(second[1], ref2.best_dur)
    assert np.array_equal(second[2], ref2.best_start)
    assert np.array_equal(o1["chi2"].cpu().numpy(), first[0])    # first outputs untouched
    assert np.array_equal(first[0], ref1.chi2) and np.array_equal(first[1], ref1.best_dur)


def test_batch_validation(ctx):
    c = synth.curve_random(5, n=100)
    tm = np.linspace(0.5, 1.0, 16)
    with pytest.raises(gtls.GtlsError):
        gtls.tls_search_batch(ctx, np.array([0, 2]), c["t"][:2], c["y"][:2], c["dy"][:2], np.array([0, 1]),
                              np.array([1.0]), np.array([0.05]), tm)
    with pytest.raises(gtls.GtlsError):
        gtls.tls_search_batch(ctx, np.array([0, 100]), c["t"], c["y"], c["dy"], np.array([0, 0]),
                              np.array([1.0]), np.array([0.05]), tm)
