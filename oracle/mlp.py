"""Float64 oracle of the engine-switch MLP -- TEST INFRASTRUCTURE ONLY.

The network maps 12 standardised per-level features to 3 engine logits:
h1 = relu(W1 x + b1) (64), h2 = relu(W2 h1 + b2) (64), z = W3 h2 + b3 (3).
Loss is the weighted mean softmax cross-entropy over a batch. Parameters are
one flat vector in the order W1, b1, W2, b2, W3, b3, each W row-major
[out][in]. Adam follows Kingma and Ba (ICLR 2015), bias-corrected.

The paper does not contain this network; it only names a more robust,
graph-adaptive switching criterion as future work (Conclusion). The shapes are
fixed by the workload description (12 -> 64 -> 64 -> 3).
"""
from __future__ import annotations

import numpy as np

D_IN, D_H, D_OUT = 12, 64, 3
SHAPES = [("W1", (D_H, D_IN)), ("b1", (D_H,)), ("W2", (D_H, D_H)), ("b2", (D_H,)),
          ("W3", (D_OUT, D_H)), ("b3", (D_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    if theta.size != N_PARAMS:
        raise ValueError(f"expected {N_PARAMS} parameters, got {theta.size}")
    out, off = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = theta[off:off + k].reshape(shp)
        off += k
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(theta, x):
    """Logits (B, 3) and the activations needed by backward."""
    p = unpack(theta)
    x = np.asarray(x, dtype=np.float64)
    a1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ p["W3"].T + p["b3"]
    return z, (x, a1, h1, a2, h2)


def loss_and_grad(theta, x, y, w=None):
    """Weighted mean cross-entropy and its gradient with respect to theta."""
    p = unpack(theta)
    z, (x, a1, h1, a2, h2) = forward(theta, x)
    y = np.asarray(y, dtype=np.int64)
    bsz = z.shape[0]
    w = np.ones(bsz) if w is None else np.asarray(w, dtype=np.float64)
    wsum = w.sum()
    zmax = z.max(axis=1, keepdims=True)
    ez = np.exp(z - zmax)
    lse = np.log(ez.sum(axis=1)) + zmax[:, 0]
    loss = float(np.sum(w * (lse - z[np.arange(bsz), y])) / wsum)
    prob = ez / ez.sum(axis=1, keepdims=True)
    dz = prob.copy()
    dz[np.arange(bsz), y] -= 1.0
    dz *= (w / wsum)[:, None]
    g = {"W3": dz.T @ h2, "b3": dz.sum(axis=0)}
    dh2 = dz @ p["W3"]
    da2 = dh2 * (a2 > 0)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ p["W2"]
    da1 = dh1 * (a1 > 0)
    g["W1"] = da1.T @ x
    g["b1"] = da1.sum(axis=0)
    return loss, pack(g)


def adam_step(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based). Returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
