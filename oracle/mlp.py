"""CPU reference of the candidate-scoring network -- TEST INFRASTRUCTURE ONLY.

A plain float64 numpy transcription of the network's definition: two hidden
layers h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2) and the output
y = W3 . h2 + b3, with parameters in the flat layout W1[H][F], b1[H],
W2[H][H], b2[H], W3[H], b3.  Gradients are derived by hand (chain rule) and
pinned in the tests by central finite differences.  bf16 rounding
(round to nearest, ties to even, on the float32 bit pattern) is written out
here independently of the device code and pinned on hand-computed values.
"""
from __future__ import annotations

import numpy as np


def unpack(p: np.ndarray, F: int, H: int):
    p = np.asarray(p, np.float64).reshape(-1)
    o = 0
    W1 = p[o:o + H * F].reshape(H, F); o += H * F
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H]; o += H
    b3 = p[o]; o += 1
    assert o == p.size
    return W1, b1, W2, b2, W3, b3


def forward(p, x, F: int, H: int = 128):
    """Outputs y[B] and activations (h1, h2) of a batch x[B, F]."""
    W1, b1, W2, b2, W3, b3 = unpack(p, F, H)
    x = np.asarray(x, np.float64)
    h1 = np.maximum(x @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    y = h2 @ W3 + b3
    return y, h1, h2


def backward(p, x, dy, F: int, H: int = 128) -> np.ndarray:
    """d(sum_b dy[b] * y[b]) / d params, in the flat layout."""
    W1, b1, W2, b2, W3, b3 = unpack(p, F, H)
    x = np.asarray(x, np.float64)
    dy = np.asarray(dy, np.float64)
    y, h1, h2 = forward(p, x, F, H)
    d2 = dy[:, None] * W3[None, :] * (h2 > 0)        # dL/d(pre-activation 2)
    d1 = (d2 @ W2) * (h1 > 0)                         # dL/d(pre-activation 1)
    gW1 = d1.T @ x
    gb1 = d1.sum(0)
    gW2 = d2.T @ h1
    gb2 = d2.sum(0)
    gW3 = h2.T @ dy
    gb3 = dy.sum()
    return np.concatenate([gW1.reshape(-1), gb1, gW2.reshape(-1), gb2, gW3, [gb3]])


def bf16_round(a) -> np.ndarray:
    """float32 values rounded to the nearest bfloat16 (ties to even), as float32."""
    a = np.asarray(a, np.float32)
    bits = a.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32)


def forward_bf16(p, x, F: int, H: int = 128) -> np.ndarray:
    """Inference with bf16 weights, inputs and first-layer activations and
    float64 accumulation (a reference for the device's fp32 accumulation)."""
    q = bf16_round(np.asarray(p, np.float32)).astype(np.float64)
    W1, b1, W2, b2, W3, b3 = unpack(q, F, H)
    xq = bf16_round(np.asarray(x, np.float32)).astype(np.float64)
    h1 = np.maximum(xq @ W1.T + b1, 0.0)
    h1 = bf16_round(h1.astype(np.float32)).astype(np.float64)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    h2 = bf16_round(h2.astype(np.float32)).astype(np.float64)
    return h2 @ W3 + b3


def mse(y, t):
    """Mean squared error and its gradient with respect to y."""
    y = np.asarray(y, np.float64)
    t = np.asarray(t, np.float64)
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / y.size


def adam(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma and Ba, 2015, Algorithm 1) with bias-corrected
    moments; returns the new (p, m, v)."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
