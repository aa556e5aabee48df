"""FP64 CPU oracle of the learned line warm start -- TEST INFRASTRUCTURE ONLY.

A 20 -> 64 -> 64 -> 4 perceptron with SiLU activations, trained by mean squared
error with Adam.  Plain numpy in float64, written layer by layer.  With
``bf16=True`` the values the GPU kernels round to bfloat16 are rounded at the
same points (round to nearest even of the float32 value): the network input,
the three weight matrices, the two hidden activations, and in the backward pass
the output error and the two pre-activation errors before they enter a matrix
product.  Biases, pre-activations and bias gradients stay unrounded.

Parameter vector (float32 on the device, float64 here), in order:
W1 [64][20], b1 [64], W2 [64][64], b2 [64], W3 [4][64], b3 [4]   (5764 values).
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 20, 64, 4
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(vec):
    out, off = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(vec[off:off + n], dtype=np.float64).reshape(shape)
        off += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(x):
    """Round to bfloat16 (nearest even) through float32, returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(vec, X, rounding=True):
    """X: [n, 20].  Returns outputs [n, 4] and the cache for backward."""
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    P = unpack(vec)
    a0 = r(X)
    W1, W2, W3 = r(P["W1"]), r(P["W2"]), r(P["W3"])
    z1 = a0 @ W1.T + P["b1"]
    a1 = r(silu(z1))
    z2 = a1 @ W2.T + P["b2"]
    a2 = r(silu(z2))
    y = a2 @ W3.T + P["b3"]
    return y, (a0, z1, a1, z2, a2, W1, W2, W3)


def loss(vec, X, Y, rounding=True):
    y, _ = forward(vec, X, rounding)
    return float(np.mean((y - Y) ** 2))


def grad(vec, X, Y, rounding=True):
    """Gradient of the mean squared error over the batch and the four outputs."""
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    y, (a0, z1, a1, z2, a2, W1, W2, W3) = forward(vec, X, rounding)
    n = X.shape[0]
    dy = 2.0 * (y - Y) / (n * N_OUT)
    dyb = r(dy)
    g = {"W3": dyb.T @ a2, "b3": dy.sum(0)}
    da2 = dyb @ W3
    dz2 = da2 * dsilu(z2)
    dz2b = r(dz2)
    g["W2"] = dz2b.T @ a1
    g["b2"] = dz2.sum(0)
    da1 = dz2b @ W2
    dz1 = da1 * dsilu(z1)
    dz1b = r(dz1)
    g["W1"] = dz1b.T @ a0
    g["b1"] = dz1.sum(0)
    return pack(g), float(np.mean((y - Y) ** 2))


def init_params(seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            bound = 1.0 / np.sqrt(shape[1])
            d[name] = rng.uniform(-bound, bound, shape)
        else:
            d[name] = np.zeros(shape)
    return pack(d)


def adam(vec, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns the new (vec, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return vec - lr * mh / (np.sqrt(vh) + eps), m, v
