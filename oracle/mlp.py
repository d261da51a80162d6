"""Plain fp64 reference of the variant-cost network (test infrastructure only).

The network is not from the paper (whose variant choice is a fixed rule,
Section 2.2 galloping, Section 4); it is this project's learned dispatcher:
a multilayer perceptron that predicts, for one matched container pair, the
log2 cost of each count variant, so that the cheapest applicable one can be
chosen. Everything here is the definition written out in numpy, float64,
with no blocking or fusion: forward pass, masked mean-squared-error loss,
its gradient by the chain rule, one Adam step, and the 12 input features.

Parameter layout (one flat float vector of N_PARAMS values):
    W1[12][64], b1[64], W2[64][64], b2[64], W3[64][6], b3[6]   (row-major)
Forward:  z1 = x W1 + b1, h1 = relu(z1); z2 = h1 W2 + b2, h2 = relu(z2);
          y = h2 W3 + b3   (x: [n, 12], y: [n, 6])
Loss:     L = sum(m * (y - t)^2) / sum(m)   (0 when the mask is empty)
Adam:     m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
          p -= lr * (m / (1 - b1^s)) / (sqrt(v / (1 - b2^s)) + eps)   (step s >= 1)
Features of a pair (types 1 array, 2 bitset, 3 run; c cardinality; r run
count, 0 for non-run containers; op 0..3):
    onehot(type_a)[3], onehot(type_b)[3], log2(1+c_a)/16, log2(1+c_b)/16,
    log2(1+r_a)/16, log2(1+r_b)/16, log2(max(c)/max(1, min(c)))/16, op/3
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 12, 64, 6
SHAPES = [("W1", (N_IN, N_H)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("W3", (N_H, N_OUT)),
          ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(params) -> dict:
    p = np.asarray(params, dtype=np.float64)
    assert p.shape == (N_PARAMS,)
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def forward(params, x):
    """Returns (y, cache) for inputs x [n, 12]."""
    w = unpack(params)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ w["W1"] + w["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ w["W2"] + w["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w["W3"] + w["b3"]
    return y, (x, z1, h1, z2, h2)


def loss(params, x, t, m) -> float:
    y, _ = forward(params, x)
    m = np.asarray(m, dtype=np.float64)
    cnt = m.sum()
    if cnt == 0:
        return 0.0
    return float((m * (y - np.asarray(t, dtype=np.float64)) ** 2).sum() / cnt)


def grad(params, x, t, m) -> np.ndarray:
    """dL/dparams by the chain rule (same layout as params)."""
    w = unpack(params)
    y, (x, z1, h1, z2, h2) = forward(params, x)
    m = np.asarray(m, dtype=np.float64)
    cnt = m.sum()
    if cnt == 0:
        return np.zeros(N_PARAMS)
    dy = 2.0 * m * (y - np.asarray(t, dtype=np.float64)) / cnt
    g = {"W3": h2.T @ dy, "b3": dy.sum(axis=0)}
    dh2 = (dy @ w["W3"].T) * (z2 > 0)
    g["W2"] = h1.T @ dh2
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ w["W2"].T) * (z1 > 0)
    g["W1"] = x.T @ dh1
    g["b1"] = dh1.sum(axis=0)
    return pack(g)


def adam(params, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step; returns (params, m, v)."""
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return np.asarray(params, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


def features(type_a, type_b, c_a, c_b, r_a, r_b, op) -> np.ndarray:
    """The 12 inputs of one pair (see the module docstring)."""
    f = np.zeros(N_IN)
    f[int(type_a) - 1] = 1.0
    f[3 + int(type_b) - 1] = 1.0
    f[6] = np.log2(1.0 + c_a) / 16
    f[7] = np.log2(1.0 + c_b) / 16
    f[8] = np.log2(1.0 + r_a) / 16
    f[9] = np.log2(1.0 + r_b) / 16
    f[10] = np.log2(max(c_a, c_b) / max(1, min(c_a, c_b))) / 16
    f[11] = op / 3.0
    return f
