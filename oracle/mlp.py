"""FP64 reference of the growth-proposal MLP (test infrastructure only).

The network is 31 -> 256 -> 256 -> 256 -> 2 with ReLU.  The GPU kernels feed
the matrix cores BF16 operands: inputs and weights are rounded to BF16, and
each hidden activation is rounded to BF16 after bias and ReLU.  This reference
applies the same roundings (round to nearest even, written out on the float32
bit pattern) and computes everything else in FP64.

The backward treats the forward's roundings as the identity (straight-through:
the gradients of the unrounded network evaluated at the rounded values) and,
by default, rounds the operands it feeds to products as BF16 operands too:
the gradient with respect to each hidden activation, dL/dh_l, is rounded to
BF16 (before the ReLU mask, with which rounding commutes), and the output
gradient is rounded to BF16 where it multiplies h3 into the last layer's
weight gradient.  The output gradient itself stays unrounded where it is
back-propagated into dL/dh3 and summed into the last bias.  round_grads=False
gives the plain straight-through gradients.

Flat parameter layout (row-major [in][out] weights, then the bias):
W1 [32][256], b1, W2 [256][256], b2, W3 [256][256], b3, W4 [256][2], b4.
"""
from __future__ import annotations

import numpy as np

IN, HID, OUT = 31, 256, 2
SHAPES = [("W1", (32, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, HID)), ("b3", (HID,)), ("W4", (HID, OUT)), ("b4", (OUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out[nan] = np.nan
    return out


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(params, X):
    """Outputs [M][2] and the cache the backward pass needs."""
    P = unpack(params)
    X = np.asarray(X, dtype=np.float64)
    M = X.shape[0]
    x = np.zeros((M, 32))
    x[:, :IN] = bf16_round(X)
    W = {k: bf16_round(P[k]) for k in ("W1", "W2", "W3", "W4")}
    h1 = bf16_round(np.maximum(x @ W["W1"] + P["b1"], 0.0))
    h2 = bf16_round(np.maximum(h1 @ W["W2"] + P["b2"], 0.0))
    h3 = bf16_round(np.maximum(h2 @ W["W3"] + P["b3"], 0.0))
    out = h3 @ W["W4"] + P["b4"]
    return out, (x, h1, h2, h3, W)


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def loss(out, yg, yp, pos_weight):
    """Mean over rows of pos_weight*y*softplus(-z) + (1-y)*softplus(z) + y*(p - t)^2
    and its gradient with respect to the outputs."""
    z, p = out[:, 0], out[:, 1]
    y, t = np.asarray(yg, dtype=np.float64), np.asarray(yp, dtype=np.float64)
    M = out.shape[0]
    L = np.mean(pos_weight * y * softplus(-z) + (1 - y) * softplus(z) + y * (p - t) ** 2)
    sig = 1.0 / (1.0 + np.exp(-z))
    d = np.zeros_like(out)
    d[:, 0] = (pos_weight * y * (sig - 1.0) + (1 - y) * sig) / M
    d[:, 1] = 2.0 * y * (p - t) / M
    return float(L), d


def backward(cache, dout, round_grads=True):
    """Gradient of the loss with respect to the flat parameters."""
    x, h1, h2, h3, W = cache
    r = bf16_round if round_grads else (lambda v: v)
    dout = np.asarray(dout, dtype=np.float64)
    g = {}
    g["W4"] = h3.T @ r(dout)
    g["b4"] = dout.sum(0)
    d3 = r(dout @ W["W4"].T) * (h3 > 0)
    g["W3"] = h2.T @ d3
    g["b3"] = d3.sum(0)
    d2 = r(d3 @ W["W3"].T) * (h2 > 0)
    g["W2"] = h1.T @ d2
    g["b2"] = d2.sum(0)
    d1 = r(d2 @ W["W2"].T) * (h1 > 0)
    g["W1"] = x.T @ d1
    g["b1"] = d1.sum(0)
    return pack(g)
