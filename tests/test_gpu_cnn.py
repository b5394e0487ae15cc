"""GPU tests of the learned period proposal's hand-written kernels against the
FP64 CPU reference (oracle/cnn.py).

The GPU multiplies BF16 operands with FP32 accumulation and keeps layer
activations in BF16, so the reference is evaluated on the same BF16-rounded
conv weights and inputs and the bar follows from BF16 rounding (8 bits of
mantissa, relative 2^-9 per rounding, compounded over five layers): logits
within 3 % of their range, gradients with cosine similarity >= 0.995 and
relative L2 error <= 5 % per tensor.  The view is compared exactly."""
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
    ref_lg, _ = cnn.forward(q, views.astype(np.float64))
    ref_loss, ref_gr = cnn.loss_and_grad(q, views.astype(np.float64), labels)
    span = ref_lg.max() - ref_lg.min()
    err = np.max(np.abs(lg - ref_lg)) / span
    print(f"logits rel err {err:.2e} (range {span:.3f}); loss {loss:.5f} vs {ref_loss:.5f}", flush=True)
    assert err <= 3e-2
    assert abs(loss - ref_loss) <= 3e-2 * abs(ref_loss)
    o = 0
    for l, (ws, bs) in enumerate(cnn.SHAPES):
        for n_el, name in ((int(np.prod(ws)), "W"), (int(np.prod(bs)), "b")):
            a, b = gr[o:o + n_el].astype(np.float64), ref_gr[o:o + n_el]
            o += n_el
            cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))
            rel = float(np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-300))
            print(f"layer {l} {name}: cosine {cos:.5f}, rel L2 {rel:.2e}", flush=True)
            assert cos >= 0.995 and rel <= 5e-2, (l, name, cos, rel)
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
