"""FP64 reference of the warm-start network (16 -> 128 -> 128 -> 1, ReLU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The warm start is not part of the paper: it predicts lambda/scale per node
from the node's 16 nearest-neighbour distances divided by the instance's
median neighbour distance, and the GDP then starts from that prediction.
This module is the plain reference the GPU kernels are checked against:
the forward pass, the mean-squared-error loss and its gradients, in float64,
with BF16 rounding applied at the points where the GPU kernels feed MFMA
operands (inputs, weights of layers 1 and 2, the layer-1 activations and the
back-propagated signals of layers 2 and 1).  With round_bf16=False it is the
exact float64 network (used for the finite-difference pin).

Parameter vector layout (float32/float64, 18817 entries):
  W1 [128,16], b1 [128], W2 [128,128], b2 [128], w3 [128], b3 [1].
"""
from __future__ import annotations

import numpy as np

D_IN, D_H = 16, 128
SIZES = (("W1", (D_H, D_IN)), ("b1", (D_H,)), ("W2", (D_H, D_H)), ("b2", (D_H,)), ("w3", (D_H,)), ("b3", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SIZES])


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    r = np.where(np.isnan(f), b, r)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(theta, X, round_bf16=True):
    """Returns y [N] and the intermediates."""
    p = unpack(theta)
    R = bf16 if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    x = R(X)
    z1 = x @ R(p["W1"]).T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    h1b = R(h1)
    z2 = h1b @ R(p["W2"]).T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["w3"] + p["b3"][0]
    return y, dict(x=x, z1=z1, h1b=h1b, z2=z2, h2=h2)


def loss_and_grad(theta, X, t, round_bf16=True):
    """MSE loss mean((y - t)^2) and its gradient with respect to theta."""
    p = unpack(theta)
    R = bf16 if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    y, c = forward(theta, X, round_bf16)
    n = y.shape[0]
    dy = 2.0 * (y - t) / n
    loss = float(np.mean((y - t) ** 2))
    g = {}
    g["w3"] = c["h2"].T @ dy
    g["b3"] = np.array([dy.sum()])
    g2 = np.outer(dy, p["w3"]) * (c["z2"] > 0)
    g2b = R(g2)
    g["W2"] = g2b.T @ c["h1b"]
    g["b2"] = g2.sum(0)
    g1 = (g2b @ R(p["W2"])) * (c["z1"] > 0)
    g1b = R(g1)
    g["W1"] = g1b.T @ c["x"]
    g["b1"] = g1.sum(0)
    return loss, pack(g)


def adamw(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, wd=0.0):
    """One AdamW update (decoupled weight decay); returns new theta, m, v."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    theta = theta - lr * (mh / (np.sqrt(vh) + eps) + wd * theta)
    return theta, m, v


def init(seed=0):
    """He-style initial parameters (float64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = {"W1": rng.normal(0, np.sqrt(2.0 / D_IN), (D_H, D_IN)), "b1": np.zeros(D_H),
         "W2": rng.normal(0, np.sqrt(2.0 / D_H), (D_H, D_H)), "b2": np.zeros(D_H),
         "w3": rng.normal(0, np.sqrt(1.0 / D_H), D_H), "b3": np.zeros(1)}
    return pack(p)
