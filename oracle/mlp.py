"""FP64 reference for the mobility-correction network (TEST INFRASTRUCTURE ONLY).

Network: 4 inputs -> 64 tanh -> 64 tanh -> 1 linear output.  Parameters live
in one flat vector in this order: W1 [64, 4], b1 [64], W2 [64, 64], b2 [64],
W3 [1, 64], b3 [1]  (4545 values).  The forward pass uses the weights rounded
to bfloat16 (round to nearest, ties to even) and evaluates in FP64.  The loss
is the mean squared error; gradients are by plain backpropagation, with the
rounding treated as the identity (straight-through) so that the FP32 master
weights receive the gradient computed at the rounded weights.  Adam follows
Kingma & Ba (2015) with bias correction.
"""
from __future__ import annotations

import numpy as np

SIZES = [("W1", (64, 4)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (1, 64)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SIZES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SIZES])


def bf16_round(x):
    """float32 -> nearest bfloat16 (ties to even), returned as float64.  NaN/Inf not expected."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = (b + 0x7FFF + lsb) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed=0):
    """Glorot-uniform weights, zero biases, as float32 master values."""
    rng = np.random.default_rng(seed)
    parts = {}
    for name, shp in SIZES:
        if name.startswith("W"):
            fan_out, fan_in = shp
            lim = np.sqrt(6.0 / (fan_in + fan_out))
            parts[name] = rng.uniform(-lim, lim, size=shp)
        else:
            parts[name] = np.zeros(shp)
    return pack(parts).astype(np.float32)


def forward(theta_master, X, round_bf16=True):
    p = unpack(bf16_round(theta_master) if round_bf16 else theta_master)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    y = h2 @ p["W3"].T + p["b3"]
    return y[:, 0], (X, h1, h2, p)


def loss_and_grad(theta_master, X, y, round_bf16=True):
    """MSE loss = mean((yhat - y)^2) and its gradient (flat, FP64)."""
    yhat, (X, h1, h2, p) = forward(theta_master, X, round_bf16)
    n = len(y)
    r = yhat - np.asarray(y, dtype=np.float64)
    loss = float(np.mean(r * r))
    dy = (2.0 / n) * r[:, None]                      # [n, 1]
    g = {"W3": dy.T @ h2, "b3": dy.sum(0)}
    dh2 = dy @ p["W3"]
    dz2 = dh2 * (1 - h2 * h2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (1 - h1 * h1)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(0)
    return loss, pack(g)


def adam_step(theta, m, v, grad, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at iteration t (1-based); returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
