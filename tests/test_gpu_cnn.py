"""GPU tests of the learned period proposal's hand-written kernels against the
FP64 CPU reference (oracle/cnn.py).

The GPU multiplies BF16 operands with FP32 accumulation: the input view, the
conv weights, the GELU outputs that feed the next convolution and the
back-propagated pre-activation gradients are stored as BF16.  The reference
is evaluated on the same BF16-rounded weights and inputs with the same
storage roundings (the oracle's ``rnd`` hook, each value rounded from FP32 to
BF16 with round-to-nearest-even), so what is left is FP32 against FP64
accumulation and FP32 transcendental functions, plus the rare BF16 rounding
that an FP32 and an FP64 value near a rounding boundary take differently.
Element-wise bars: logits |gpu - ref| <= 1e-3 |ref| + 1e-5 max|ref|; each
gradient tensor |gpu - ref| <= 1e-2 |ref| + 1e-3 max|ref| (the absolute term
covers elements near zero whose sums of B x 4096 products cancel: FP32
accumulation leaves about sqrt(n) 2^-24 of the sum of magnitudes, a flipped
BF16 rounding moves one product by 2^-8).  The Adam update is compared with
the reference update from the same gradients.  The view is compared exactly."""
import numpy as np
import pytest

from oracle import cnn
from paper_2607_00348_amd import gtls, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = gtls.Context(0)
    yield c
    c.close()


def _bf16(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16            # round to nearest even
    return u.astype(np.uint32).view(np.float32)


def _effective_params(p):
    q = np.asarray(p, dtype=np.float32).astype(np.float64)
    for l in range(cnn.NL):
        o = 0
        for k in range(l):
            ws, bs = cnn.SHAPES[k]
            o += int(np.prod(ws)) + int(np.prod(bs))
        nw = int(np.prod(cnn.SHAPES[l][0]))
        q[o:o + nw] = _bf16(q[o:o + nw]).astype(np.float64)
    return q


def test_view_matches_oracle(ctx):
    curves = [synth.curve_90d(), synth.curve_random(3, n=20000, inject=True), synth.curve_random(4, n=500)]
    off = np.cumsum([0] + [len(c["t"]) for c in curves])
    t = np.concatenate([c["t"] for c in curves])
    y = np.concatenate([c["y"] for c in curves])
    v = gtls.gtls_cnn_view(ctx, off, t, y)
    for k, c in enumerate(curves):
        ref = cnn.view(c["t"], c["y"]).astype(np.float32)
        assert np.array_equal(v[k], ref), k


def _bf16_store(a):
    """BF16 storage of a value computed in FP32 (round to nearest even)."""
    return _bf16(np.asarray(a, dtype=np.float64).astype(np.float32)).astype(np.float64)


def _tensors(flat):
    o = 0
    for l, (ws, bs) in enumerate(cnn.SHAPES):
        for n_el, name in ((int(np.prod(ws)), "W"), (int(np.prod(bs)), "b")):
            yield l, name, slice(o, o + n_el)
            o += n_el


def test_forward_and_gradients_match_oracle(ctx):
    p = synth.cnn_init(11).astype(np.float32)
    p[-512:] = synth.rng(12).normal(0, 0.05, 512)
    g = synth.rng(13)
    views = _bf16(g.normal(0, 1, (4, cnn.L)))
    labels = g.integers(0, cnn.NB, 4).astype(np.int32)
    net = gtls.Cnn(ctx, p)
    lg = gtls.gtls_cnn_forward(net, views)
    loss, gr = gtls.gtls_cnn_gradients(net, views, labels)
    q = _effective_params(p)
    ref_lg, _ = cnn.forward(q, views.astype(np.float64), rnd=_bf16_store)
    ref_loss, ref_gr = cnn.loss_and_grad(q, views.astype(np.float64), labels, rnd=_bf16_store)
    lim = 1e-3 * np.abs(ref_lg) + 1e-5 * np.abs(ref_lg).max()
    worst = float(np.max(np.abs(lg - ref_lg) / lim))
    print(f"logits: worst |err| / bound {worst:.3f}; loss {loss:.7f} vs {ref_loss:.7f}", flush=True)
    assert worst <= 1.0
    assert abs(loss - ref_loss) <= 1e-4 * abs(ref_loss)
    for l, name, sl in _tensors(gr):
        a, b = gr[sl].astype(np.float64), ref_gr[sl]
        lim = 1e-2 * np.abs(b) + 1e-3 * np.abs(b).max()
        ratio = np.abs(a - b) / lim
        print(f"layer {l} {name}: worst |err| / bound {ratio.max():.3f}, "
              f"max rel err {np.max(np.abs(a - b)) / np.abs(b).max():.2e}", flush=True)
        assert ratio.max() <= 1.0, (l, name, int(np.argmax(ratio)))
    net.close()


def test_adam_matches_oracle(ctx):
    """Three Adam steps on the GPU against the reference update (FP64) fed
    with the GPU's own gradients at each step's parameters."""
    p = synth.cnn_init(31).astype(np.float32)
    g = synth.rng(32)
    views = g.normal(0, 1, (4, cnn.L)).astype(np.float32)
    labels = g.integers(0, cnn.NB, 4).astype(np.int32)
    net = gtls.Cnn(ctx, p)
    q = p.astype(np.float64)
    m = np.zeros(cnn.N_PARAMS)
    v = np.zeros(cnn.N_PARAMS)
    lr = 2e-3
    for step in (1, 2, 3):
        cur = gtls.gtls_cnn_get_params(net)
        _, gr = gtls.gtls_cnn_gradients(net, views, labels)
        q, m, v = cnn.adam(q, gr.astype(np.float64), m, v, step, lr=lr)
        gtls.gtls_cnn_train_step(net, views, labels, lr=lr)
        got = gtls.gtls_cnn_get_params(net).astype(np.float64)
        moved = got - cur
        want = q - cur
        err = np.max(np.abs(moved - want)) / lr
        print(f"adam step {step}: max |update error| / lr {err:.2e}", flush=True)
        assert np.allclose(got, q, rtol=1e-6, atol=1e-3 * lr)
        q = got                               # continue from the GPU's FP32 parameters
    net.close()


def test_training_reduces_loss_and_topk(ctx):
    p = synth.cnn_init(21).astype(np.float32)
    g = synth.rng(22)
    views = g.normal(0, 1, (16, cnn.L)).astype(np.float32)
    labels = g.integers(0, cnn.NB, 16).astype(np.int32)
    net = gtls.Cnn(ctx, p)
    losses = [gtls.gtls_cnn_train_step(net, views, labels, lr=3e-3) for _ in range(30)]
    print("losses", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.7 * losses[0]
    lg = gtls.gtls_cnn_forward(net, views)
    top = gtls.gtls_cnn_topk(net, views, 32)
    assert np.array_equal(top, cnn.topk_bins(lg.astype(np.float64), 32))
    q = gtls.gtls_cnn_get_params(net)
    assert np.all(np.isfinite(q)) and not np.array_equal(q, p)
    net.close()


def test_checkpoint_resume_is_bit_exact(ctx, tmp_path):
    """Train 5 steps, save, train 4 more; a new network loaded from the
    checkpoint and trained the same 4 steps ends with the same parameters,
    bit for bit (parameters, Adam moments and step count are restored)."""
    p = synth.cnn_init(41).astype(np.float32)
    g = synth.rng(42)
    batches = [(g.normal(0, 1, (4, cnn.L)).astype(np.float32), g.integers(0, cnn.NB, 4).astype(np.int32))
               for _ in range(9)]
    net = gtls.Cnn(ctx, p)
    for v, lab in batches[:5]:
        gtls.gtls_cnn_train_step(net, v, lab, lr=2e-3)
    path = str(tmp_path / "net.ckpt")
    gtls.gtls_cnn_save(net, path)
    saved = gtls.gtls_cnn_get_params(net)
    for v, lab in batches[5:]:
        gtls.gtls_cnn_train_step(net, v, lab, lr=2e-3)
    a = gtls.gtls_cnn_get_params(net)
    net.close()
    other = gtls.Cnn(ctx, synth.cnn_init(99).astype(np.float32))
    gtls.gtls_cnn_load(other, path)
    assert np.array_equal(gtls.gtls_cnn_get_params(other), saved)
    for v, lab in batches[5:]:
        gtls.gtls_cnn_train_step(other, v, lab, lr=2e-3)
    b = gtls.gtls_cnn_get_params(other)
    assert np.array_equal(a, b)
    with open(path, "r+b") as f:                       # a damaged header is refused
        f.write(b"XXXX")
    with pytest.raises(gtls.GtlsError):
        gtls.gtls_cnn_load(other, path)
    other.close()


def test_pruned_search_subset_and_fallback(ctx, oracle):
    """tls_search_pruned: the periods it searches are exactly the grid
    periods inside the network's top-k bins; their chi2, windows and depths
    equal the plain search's at those periods (periods are independent), the
    SR/SDE equal the oracle's periodogram of that subset; with an accept
    threshold no subset can reach, the result is the whole-grid search."""
    c = synth.curve_random(71, n=3000, inject=True)
    span = c["t"].max() - c["t"].min()
    grid = gtls.gtls_period_grid_ofir(span, 2.0, pmin_days=0.5, pmax_days=span / 2)
    durs = gtls.gtls_duration_grid(grid[0], grid[-1], 10)
    tm = gtls.gtls_template_quadratic(0.4, 0.25, 0.02, 0.0, 256)
    net = gtls.Cnn(ctx, synth.cnn_init(5).astype(np.float32))
    full = gtls.tls_search(ctx, c["t"], c["y"], c["dy"], grid, durs, tm)
    k = 48
    res, searched, fell = gtls.tls_search_pruned(ctx, net, c["t"], c["y"], c["dy"], grid, durs, tm, grid[0],
                                                 grid[-1], k, -1e300)
    assert not fell
    view = gtls.gtls_cnn_view(ctx, np.array([0, len(c["t"])]), c["t"], c["y"])
    top = gtls.gtls_cnn_topk(net, view, k)[0]
    b = np.clip(np.floor(np.log(grid / grid[0]) / np.log(grid[-1] / grid[0]) * 512), 0, 511).astype(int)
    assert np.array_equal(searched, np.isin(b, top))
    sel = np.nonzero(searched)[0]
    assert len(sel) > 0
    assert np.array_equal(res.chi2[sel], full.chi2[sel])
    assert np.array_equal(res.best_start[sel], full.best_start[sel])
    assert np.array_equal(res.depth[sel], full.depth[sel])
    assert np.all(np.isnan(res.chi2[~searched])) and np.all(res.best_dur[~searched] == -1)
    sr, raw, sde, best = oracle.sde(full.chi2[sel], 91)
    assert np.allclose(res.sde[sel], sde, rtol=0, atol=1e-9 * np.max(np.abs(sde)))
    assert res.best_period == sel[best]
    assert res.n_evals > 0
    res2, searched2, fell2 = gtls.tls_search_pruned(ctx, net, c["t"], c["y"], c["dy"], grid, durs, tm, grid[0],
                                                    grid[-1], k, 1e300)
    assert fell2 and np.all(searched2)
    assert np.array_equal(res2.chi2, full.chi2) and res2.best_period == full.best_period
    assert res2.n_evals == res.n_evals + full.n_evals
    net.close()
