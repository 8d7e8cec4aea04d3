"""Float64 reference of the witness-cell scoring MLP (oracle; test infrastructure only).

The network scores a candidate witness cell c of a pair (x, y) from F
scale-free features (distances divided by d(x,y)):
    h = relu(f @ W1 + b1)          W1 [F, H], b1 [H]
    s = h @ w2 + b2                w2 [H],   b2 scalar
and is trained with the mean binary cross-entropy with logits against the
label "cell c holds a witness of (x, y)".  Parameters are packed as one
vector [W1 (row-major), b1, w2, b2] of length F*H + 2*H + 1.

This module is the definition written out (no fusion or reordering); it pins
the GPU forward and backward kernels.  The ranking only orders the exhaustive
scan of Stages V-VI (Section 2); it never decides an edge.
"""
from __future__ import annotations

import numpy as np


def unpack(theta: np.ndarray, F: int, H: int):
    theta = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = theta[o:o + F * H].reshape(F, H); o += F * H
    b1 = theta[o:o + H]; o += H
    w2 = theta[o:o + H]; o += H
    b2 = theta[o]
    return W1, b1, w2, b2


def forward(theta, feats, F: int, H: int):
    W1, b1, w2, b2 = unpack(theta, F, H)
    X = np.asarray(feats, dtype=np.float64)
    pre = X @ W1 + b1
    h = np.maximum(pre, 0.0)
    return h @ w2 + b2


def loss(theta, feats, labels, F: int, H: int) -> float:
    s = forward(theta, feats, F, H)
    y = np.asarray(labels, dtype=np.float64)
    # mean of log(1 + exp(s)) - y*s, computed stably
    return float(np.mean(np.logaddexp(0.0, s) - y * s))


def grad(theta, feats, labels, F: int, H: int) -> np.ndarray:
    """Gradient of ``loss`` by the chain rule (backpropagation)."""
    W1, b1, w2, b2 = unpack(theta, F, H)
    X = np.asarray(feats, dtype=np.float64)
    y = np.asarray(labels, dtype=np.float64)
    n = X.shape[0]
    pre = X @ W1 + b1
    h = np.maximum(pre, 0.0)
    s = h @ w2 + b2
    ds = (1.0 / (1.0 + np.exp(-s)) - y) / n          # d loss / d s
    gw2 = h.T @ ds
    gb2 = ds.sum()
    dh = np.outer(ds, w2) * (pre > 0.0)
    gW1 = X.T @ dh
    gb1 = dh.sum(axis=0)
    return np.concatenate([gW1.reshape(-1), gb1, gw2, [gb2]])


def finite_difference(theta, feats, labels, F: int, H: int, eps: float = 1e-6) -> np.ndarray:
    theta = np.asarray(theta, dtype=np.float64)
    g = np.zeros_like(theta)
    for i in range(theta.size):
        tp = theta.copy(); tp[i] += eps
        tm = theta.copy(); tm[i] -= eps
        g[i] = (loss(tp, feats, labels, F, H) - loss(tm, feats, labels, F, H)) / (2 * eps)
    return g


def adam_step(theta, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(theta) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float64 values.

    bfloat16 keeps the top 16 bits of the float32 pattern (8 exponent bits,
    7 fraction bits); rounding adds half an ulp of the kept part, plus one
    when the kept part is odd and the dropped half is exactly half an ulp.
    """
    u = np.asarray(theta, dtype=np.float32).view(np.uint32).astype(np.uint64)
    keep_odd = (u >> 16) & 1
    r = ((u + 0x7FFF + keep_odd) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
