"""Plain CPU oracle for the learned embedding-dimension surrogate.

TEST INFRASTRUCTURE ONLY (never imported by the product path).  float64 numpy.

The network maps a z-scored series x[L] to a distribution over E = 1..20:
three 1-D convolutions (kernel width KW, zero "same" padding), each followed by
ReLU, then the mean over time (global average pool), then a linear layer to 20
logits; training minimises the mean softmax cross-entropy against the E* that
the simplex sweep selects (the method's own E selection, Section 2.1 step 1 /
Section 3.4 of the kEDM paper, used as the label).  Adam updates the
parameters.

Flat parameter layout (shared contract with the GPU kernels, documented in
include/edm.h):  w1[C][1][KW], b1[C], w2[C][C][KW], b2[C], w3[C][C][KW], b3[C],
wo[20][C], bo[20].

Pin: gradients of ``loss_and_grads`` are checked against central finite
differences of ``loss`` (tests/test_net_oracle.py), which shares none of the
backward code.
"""
from __future__ import annotations

import numpy as np

NCLASS = 20
KW = 7


def param_shapes(C: int, kw: int = KW):
    return [("w1", (C, 1, kw)), ("b1", (C,)), ("w2", (C, C, kw)), ("b2", (C,)),
            ("w3", (C, C, kw)), ("b3", (C,)), ("wo", (NCLASS, C)), ("bo", (NCLASS,))]


def param_count(C: int, kw: int = KW) -> int:
    return int(sum(np.prod(s) for _, s in param_shapes(C, kw)))


def unpack(theta, C: int, kw: int = KW):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shp in param_shapes(C, kw):
        n = int(np.prod(shp))
        out[name] = theta[o:o + n].reshape(shp)
        o += n
    assert o == theta.size
    return out


def pack(p, C: int, kw: int = KW):
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in param_shapes(C, kw)])


def conv_same(x, w, b):
    """y[n][o][t] = b[o] + sum_i sum_k w[o][i][k] x[n][i][t + k - kw//2] (zero padded)."""
    n, ci, L = x.shape
    co, ci2, kw = w.shape
    assert ci == ci2
    h = kw // 2
    xp = np.zeros((n, ci, L + 2 * h))
    xp[:, :, h:h + L] = x
    y = np.zeros((n, co, L))
    for k in range(kw):
        # contraction over input channels for lag k
        y += np.einsum("oi,nit->not", w[:, :, k], xp[:, :, k:k + L])
    return y + b[None, :, None]


def forward(theta, X, C: int, kw: int = KW):
    """Returns logits [B][20] and the activations needed by the backward pass."""
    p = unpack(theta, C, kw)
    x = np.asarray(X, np.float64)[:, None, :]
    a1 = np.maximum(conv_same(x, p["w1"], p["b1"]), 0.0)
    a2 = np.maximum(conv_same(a1, p["w2"], p["b2"]), 0.0)
    a3 = np.maximum(conv_same(a2, p["w3"], p["b3"]), 0.0)
    g = a3.mean(axis=2)
    logits = g @ p["wo"].T + p["bo"]
    return logits, (x, a1, a2, a3, g)


def bf16_round(a):
    """Round to the nearest BF16 value (8 significant bits, ties to even),
    through float32 first (the GPU holds these values in float32); returned
    as float64.  BF16 is the upper half of an IEEE float32."""
    f = np.asarray(a, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def forward_bf16(theta, X, C: int, kw: int = KW):
    """Inference forward pass of the BF16 form: layer 1 as in ``forward``;
    the inputs and weights of the two C -> C convolutions rounded to BF16
    (their products are exact), sums, bias, ReLU, pooling and the linear
    layer in float64.  Returns logits [B][20]."""
    p = unpack(theta, C, kw)
    x = np.asarray(X, np.float64)[:, None, :]
    a1 = np.maximum(conv_same(x, p["w1"], p["b1"]), 0.0)
    a2 = np.maximum(conv_same(bf16_round(a1), bf16_round(p["w2"]), p["b2"]), 0.0)
    a3 = np.maximum(conv_same(bf16_round(a2), bf16_round(p["w3"]), p["b3"]), 0.0)
    g = a3.mean(axis=2)
    return g @ p["wo"].T + p["bo"]


def softmax(logits):
    z = logits - logits.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def loss(theta, X, labels, C: int, kw: int = KW) -> float:
    """Mean cross-entropy; labels hold E in 1..20 (class E-1)."""
    logits, _ = forward(theta, X, C, kw)
    z = logits - logits.max(axis=1, keepdims=True)
    lse = np.log(np.exp(z).sum(axis=1))
    y = np.asarray(labels) - 1
    return float(np.mean(lse - z[np.arange(len(y)), y]))


def conv_same_grads(x, w, dy):
    """Gradients of y = conv_same(x, w, b) given dy: (dx, dw, db)."""
    n, ci, L = x.shape
    co, _, kw = w.shape
    h = kw // 2
    xp = np.zeros((n, ci, L + 2 * h))
    xp[:, :, h:h + L] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for k in range(kw):
        dw[:, :, k] = np.einsum("not,nit->oi", dy, xp[:, :, k:k + L])
        dxp[:, :, k:k + L] += np.einsum("oi,not->nit", w[:, :, k], dy)
    return dxp[:, :, h:h + L], dw, dy.sum(axis=(0, 2))


def loss_and_grads(theta, X, labels, C: int, kw: int = KW):
    """Mean cross-entropy and its gradient with respect to the flat parameters."""
    p = unpack(theta, C, kw)
    logits, (x, a1, a2, a3, g) = forward(theta, X, C, kw)
    B = logits.shape[0]
    y = np.asarray(labels) - 1
    P = softmax(logits)
    lval = float(np.mean(-np.log(P[np.arange(B), y])))
    dlog = P.copy()
    dlog[np.arange(B), y] -= 1.0
    dlog /= B
    grads = {}
    grads["wo"] = dlog.T @ g
    grads["bo"] = dlog.sum(axis=0)
    dg = dlog @ p["wo"]
    L = a3.shape[2]
    dz3 = np.repeat(dg[:, :, None] / L, L, axis=2) * (a3 > 0)
    da2, grads["w3"], grads["b3"] = conv_same_grads(a2, p["w3"], dz3)
    dz2 = da2 * (a2 > 0)
    da1, grads["w2"], grads["b2"] = conv_same_grads(a1, p["w2"], dz2)
    dz1 = da1 * (a1 > 0)
    _, grads["w1"], grads["b1"] = conv_same_grads(x, p["w1"], dz1)
    return lval, pack(grads, C, kw)


def adam_step(theta, grad, m, v, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; returns new arrays."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
