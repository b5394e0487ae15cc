"""GPU test of the allocation-free search entry point: its outputs must
equal tls_search_dev's, bit for bit, on two calls in a row on one context
(the second with a smaller curve and grid, so the static scratch holds the
first call's contents when the second starts), through the C ABI."""
import numpy as np
import pytest

from paper_2607_00348_amd import gtls, synth

pytestmark = pytest.mark.gpu

KEYS = ("chi2", "depth", "t0", "sr", "raw", "sde")


def _case(seed, n, nper, dt0):
    c = synth.curve_random(seed, n=n, inject=True)
    span = c["t"].max() - c["t"].min()
    periods = gtls.gtls_period_grid_ofir(span, 2.0, pmin_days=0.5, pmax_days=max(0.6, span / 2))
    if len(periods) > nper:
        periods = periods[np.linspace(0, len(periods) - 1, nper).astype(int)]
    durs = gtls.gtls_duration_grid(periods[0], periods[-1], 12)
    tm = gtls.gtls_template_quadratic(0.4, 0.25, 0.02, 0.0, 256)
    return c, periods, durs, tm, gtls.gtls_params_default(dt0=dt0)


def _run(fn, dctx, case):
    import torch
    c, periods, durs, tm, prm = case
    dev = torch.device("cuda:0")
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    t_d, y_d, dy_d, p_d, d_d, tm_d = f(c["t"]), f(c["y"]), f(c["dy"]), f(periods), f(durs), f(tm)
    npd = len(periods)
    o = {k: torch.full((npd,), -7.0, dtype=torch.float64, device=dev) for k in KEYS}
    bd = torch.full((npd,), -7, dtype=torch.int32, device=dev)
    bs = torch.full((npd,), -7, dtype=torch.int32, device=dev)
    summ = torch.zeros(5, dtype=torch.int64, device=dev)
    fn(dctx, t_d.data_ptr(), y_d.data_ptr(), dy_d.data_ptr(), len(c["t"]), p_d.data_ptr(), npd, d_d.data_ptr(),
       len(durs), tm_d.data_ptr(), len(tm), prm, o["chi2"].data_ptr(), bd.data_ptr(), bs.data_ptr(),
       o["depth"].data_ptr(), o["t0"].data_ptr(), o["sr"].data_ptr(), o["raw"].data_ptr(), o["sde"].data_ptr(),
       summ.data_ptr())
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in o.items()}
    out["best_dur"], out["best_start"], out["summary"] = bd.cpu().numpy(), bs.cpu().numpy(), summ.cpu().numpy()
    return out


def _same(a, b, label):
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), (label, k)


def test_noalloc_equals_dev_search():
    import torch
    stream = torch.cuda.current_stream()
    dctx = gtls.Context(0, stream.cuda_stream)
    big = _case(61, 9000, 900, 0.1)
    small = _case(62, 2500, 300, 0.0)
    for label, case in (("first call, 9000 points", big), ("second call, 2500 points", small)):
        print("no-alloc:", label, flush=True)
        ref = _run(gtls.tls_search_dev, dctx, case)
        got = _run(gtls.tls_search_dev_noalloc, dctx, case)
        _same(got, ref, label)
        assert np.all(got["best_dur"] >= -1) and got["summary"][2] > 0
    dctx.close()


def test_noalloc_rejects_oversized_curve():
    """A curve whose template rows alone exceed the static scratch is refused
    before anything runs."""
    import torch
    stream = torch.cuda.current_stream()
    dctx = gtls.Context(0, stream.cuda_stream)
    n = 200000
    dev = torch.device("cuda:0")
    t = torch.arange(n, dtype=torch.float64, device=dev) * 0.02
    y = torch.ones(n, dtype=torch.float64, device=dev)
    dy = torch.full((n,), 1e-3, dtype=torch.float64, device=dev)
    per = torch.tensor([1.0, 2.0], dtype=torch.float64, device=dev)
    dur = torch.tensor([0.1], dtype=torch.float64, device=dev)
    tm = torch.tensor([0.5, 1.0, 0.5], dtype=torch.float64, device=dev)
    outs = [torch.empty(2, dtype=torch.float64, device=dev) for _ in range(6)]
    ints = [torch.empty(2, dtype=torch.int32, device=dev) for _ in range(2)]
    summ = torch.zeros(5, dtype=torch.int64, device=dev)
    with pytest.raises(gtls.GtlsError) as ei:
        gtls.tls_search_dev_noalloc(dctx, t.data_ptr(), y.data_ptr(), dy.data_ptr(), n, per.data_ptr(), 2,
                                    dur.data_ptr(), 1, tm.data_ptr(), 3, None, outs[0].data_ptr(),
                                    ints[0].data_ptr(), ints[1].data_ptr(), outs[1].data_ptr(), outs[2].data_ptr(),
                                    outs[3].data_ptr(), outs[4].data_ptr(), outs[5].data_ptr(), summ.data_ptr())
    assert ei.value.code == gtls.GTLS_ENOMEM
    dctx.close()
