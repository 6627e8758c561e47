"""Float64 reference of the learned-proposal network.

TEST INFRASTRUCTURE ONLY (see the oracle package docstring).

Network (the proposal model of the decoding path; not a method of the paper,
whose outlook only mentions learned pre-decoders):
    h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), delta = W3 h2 + b3
    z = -(Lambda + delta), loss = mean_b sum_j [max(z,0) - z y + log(1 + exp(-|z|))]
    (binary cross-entropy with logits; y = Relay-BP correction bits)
Parameters are one flat array laid out W1[h][in], b1[h], W2[h][h], b2[h],
W3[out][h], b3[out].  Adam: beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected.

``mirror=True`` rounds to bfloat16 (round to nearest even) where the GPU path
stores BF16 values: the weights used in products, the hidden activations and
the backward operands; everything else is float64.
"""
from __future__ import annotations

import numpy as np


def bf16(a: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even); returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    out = (r << 16).astype(np.uint32).view(np.float32)
    return out.astype(np.float64)


def split(params: np.ndarray, din: int, h: int, dout: int):
    o = 0
    W1 = params[o:o + h * din].reshape(h, din); o += h * din
    b1 = params[o:o + h]; o += h
    W2 = params[o:o + h * h].reshape(h, h); o += h * h
    b2 = params[o:o + h]; o += h
    W3 = params[o:o + dout * h].reshape(dout, h); o += dout * h
    b3 = params[o:o + dout]; o += dout
    assert o == params.size
    return W1, b1, W2, b2, W3, b3


def num_params(din: int, h: int, dout: int) -> int:
    return h * din + h + h * h + h + dout * h + dout


def _r(a, mirror):
    return bf16(a) if mirror else np.asarray(a, dtype=np.float64)


def forward(params, x, din, h, dout, mirror=True):
    """x: (B, din) 0/1.  Returns (delta, cache)."""
    W1, b1, W2, b2, W3, b3 = split(np.asarray(params, np.float64), din, h, dout)
    W1r, W2r, W3r = _r(W1, mirror), _r(W2, mirror), _r(W3, mirror)
    x = np.asarray(x, np.float64)
    h1 = _r(np.maximum(x @ W1r.T + b1, 0.0), mirror)
    h2 = _r(np.maximum(h1 @ W2r.T + b2, 0.0), mirror)
    delta = h2 @ W3r.T + b3
    return delta, (x, h1, h2, W1r, W2r, W3r)


def loss_and_grads(params, x, y, lam, din, h, dout, mirror=True):
    """Mean BCE-with-logits loss and its gradient (flat, parameter layout)."""
    delta, (x, h1, h2, W1r, W2r, W3r) = forward(params, x, din, h, dout, mirror)
    B = x.shape[0]
    z = -(np.asarray(lam, np.float64)[None, :] + delta)
    y = np.asarray(y, np.float64)
    loss = (np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))).sum() / B
    p = 1.0 / (1.0 + np.exp(-z))
    d3 = -(p - y) / B                     # dL/d(delta)
    d3r = _r(d3, mirror)
    gW3 = d3r.T @ h2
    gb3 = d3.sum(0)
    dh2 = (d3r @ W3r) * (h2 > 0)
    dh2r = _r(dh2, mirror)
    gW2 = dh2r.T @ h1
    gb2 = dh2.sum(0)
    dh1 = (dh2r @ W2r) * (h1 > 0)
    dh1r = _r(dh1, mirror)
    gW1 = dh1r.T @ x
    gb1 = dh1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam(params, grads, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grads
    v = b2 * v + (1 - b2) * grads * grads
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
