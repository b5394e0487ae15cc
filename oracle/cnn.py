"""Plain FP64 reference of the learned period proposal (numpy).

TEST INFRASTRUCTURE ONLY: only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP library.

What it computes:

* ``view`` -- the network input: the light curve's time span cut into 4096
  equal bins; per bin the median flux, standardised as (median - 1) /
  (1.4826 MAD) with MAD the median absolute deviation of the whole curve from
  its median; empty bins are 0.  Medians of an even count average the two
  middle values.
* ``forward`` / ``backward`` -- five conv1d layers (1 -> 32 -> 32 -> 32 ->
  32 -> 32 channels, kernel 7, zero padding 3, stride 1), each followed by
  GELU (the erf form), a global average over the 4096 positions, a 32 ->
  512 linear layer and the softmax cross-entropy against a period-bin label
  (mean over the batch).
* ``adam`` -- one Adam update (beta1 0.9, beta2 0.999, eps 1e-8).

Parameters travel as one flat vector in the order W0, b0, ..., W4, b4, Wf,
bf with W_l of shape (32, C_in, 7) and Wf of shape (512, 32).

Storage precision.  ``forward`` and ``loss_and_grad`` take an optional
``rnd`` function.  It models a precision scheme that multiplies reduced-
precision operands with a wider accumulation (the learned proposal is
specified with BF16 operands and FP32 accumulation): it is applied to every
tensor that such a scheme stores as a matrix operand -- the network input, the
GELU outputs that feed the next convolution, and the back-propagated
pre-activation gradients dz of every layer before they enter the weight,
bias and data gradients.  Weights are rounded by the caller.  The default
(None) keeps everything in FP64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

L = 4096
C = 32
KW = 7
NB = 512
NL = 5
SHAPES = ([((C, 1, KW), (C,))] + [((C, C, KW), (C,))] * (NL - 1) + [((NB, C), (NB,))])
N_PARAMS = sum(int(np.prod(w)) + int(np.prod(b)) for w, b in SHAPES)


def unflatten(p):
    out, o = [], 0
    for ws, bs in SHAPES:
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out.append((p[o:o + nw].reshape(ws), p[o + nw:o + nw + nb]))
        o += nw + nb
    return out


def flatten(layers):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in layers])


# --------------------------------------------------------------------------
# Input view

def view(t, y):
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    t0, t1 = t.min(), t.max()
    span = t1 - t0
    b = np.floor((t - t0) / span * float(L)).astype(np.int64) if span > 0 else np.zeros(len(t), np.int64)
    b = np.clip(b, 0, L - 1)
    med = np.median(y)
    scale = 1.4826 * np.median(np.abs(y - med))
    out = np.zeros(L)
    if not scale > 0:
        return out
    for k in range(L):
        sel = y[b == k]
        if sel.size:
            out[k] = (np.median(sel) - 1.0) / scale
    return out


def period_bins(pmin: float, pmax: float, nb: int = NB) -> np.ndarray:
    """nb + 1 geometric bin edges over [pmin, pmax]."""
    return pmin * (pmax / pmin) ** (np.arange(nb + 1) / nb)


# --------------------------------------------------------------------------
# Network

def _gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def _gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def _conv(h, w, b):
    """z[n, co, l] = sum_{ci, k} w[co, ci, k] h[n, ci, l + k - 3] + b[co]."""
    n, cin, ln = h.shape
    hp = np.zeros((n, cin, ln + KW - 1))
    hp[:, :, KW // 2:KW // 2 + ln] = h
    z = np.zeros((n, w.shape[0], ln))
    for k in range(KW):
        z += np.einsum("oc,ncl->nol", w[:, :, k], hp[:, :, k:k + ln])
    return z + b[None, :, None]


def _keep(a):
    return a


def forward(p, x, rnd=None):
    """x: (B, 4096) views -> (logits (B, 512), cache)."""
    rnd = rnd or _keep
    layers = unflatten(np.asarray(p, dtype=np.float64))
    h = rnd(np.asarray(x, dtype=np.float64))[:, None, :]
    cache = []
    for li, (w, b) in enumerate(layers[:NL]):
        z = _conv(h, w, b)
        cache.append((h, z))
        h = _gelu(z)
        if li < NL - 1:
            h = rnd(h)
    g = h.mean(axis=2)
    wf, bf = layers[NL]
    logits = g @ wf.T + bf
    return logits, (cache, h, g)


def loss_and_grad(p, x, labels, rnd=None):
    """Mean softmax cross-entropy and its gradient (flat, like p)."""
    rnd = rnd or _keep
    layers = unflatten(np.asarray(p, dtype=np.float64))
    logits, (cache, h_last, g) = forward(p, x, rnd)
    n = logits.shape[0]
    m = logits.max(axis=1, keepdims=True)
    e = np.exp(logits - m)
    s = e.sum(axis=1, keepdims=True)
    lse = (m + np.log(s))[:, 0]
    loss = float(np.mean(lse - logits[np.arange(n), labels]))
    d = e / s
    d[np.arange(n), labels] -= 1.0
    d /= n
    wf, bf = layers[NL]
    grads = [None] * (NL + 1)
    grads[NL] = (d.T @ g, d.sum(axis=0))
    dg = d @ wf
    dh = np.repeat(dg[:, :, None], L, axis=2) / L
    for li in range(NL - 1, -1, -1):
        h, z = cache[li]
        w, b = layers[li]
        dz = rnd(dh * _gelu_grad(z))
        hp = np.zeros((n, h.shape[1], L + KW - 1))
        hp[:, :, KW // 2:KW // 2 + L] = h
        dw = np.zeros_like(w)
        for k in range(KW):
            dw[:, :, k] = np.einsum("nol,ncl->oc", dz, hp[:, :, k:k + L])
        db = dz.sum(axis=(0, 2))
        grads[li] = (dw, db)
        if li > 0:
            dzp = np.zeros((n, dz.shape[1], L + KW - 1))
            dzp[:, :, KW // 2:KW // 2 + L] = dz
            dhp = np.zeros_like(h)
            for k in range(KW):
                # h[l'] feeds z[l' - k + 3] through w[:, :, k]
                dhp += np.einsum("oc,nol->ncl", w[:, :, k], dzp[:, :, KW - 1 - k:KW - 1 - k + L])
            dh = dhp
    return loss, flatten(grads)


def adam(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def topk_bins(logits, k):
    """Indices of the k largest logits per row, largest first (ties: lower index)."""
    order = np.argsort(-logits, axis=1, kind="stable")
    return order[:, :k]
