"""fp64 reference of the threshold-selector network.  TEST INFRASTRUCTURE ONLY.

The selector is not part of the paper: it stands in for the search of
Algorithm 2 (Section 5).  This module is the plain definition of what the
library's selector kernels compute, written in numpy float64 with the
backward pass derived by hand, so that the GPU forward pass, loss gradient
and Adam step can be checked against it.  Its own correctness is pinned in
the tests by central finite differences of ``loss`` (gradient), by networks
whose output has a closed form (forward and parameter layout), and by the
closed form of Adam's first steps.

Network: x (16) -> relu(W1 x + b1) (64) -> relu(W2 h1 + b2) (64) -> W3 h2 + b3 (K).
Flat parameter layout: W1[64][16], b1[64], W2[64][64], b2[64], W3[K][64], b3[K].

Loss for targets t and weights m >= 0 (0 = no label), batch B:
    L = (1/B) sum_s [sum_k m[s,k] (y[s,k] - t[s,k])^2] / max(1, sum_k m[s,k])
"""
from __future__ import annotations

import numpy as np

N_IN = 16
N_HIDDEN = 64


def param_count(k: int) -> int:
    return N_HIDDEN * N_IN + N_HIDDEN + N_HIDDEN * N_HIDDEN + N_HIDDEN + k * N_HIDDEN + k


def unpack(params, k: int):
    """Views (W1, b1, W2, b2, W3, b3) of a flat parameter vector."""
    p = np.asarray(params, dtype=np.float64)
    if p.size != param_count(k):
        raise ValueError("parameter count does not match the layout")
    sizes = [(N_HIDDEN, N_IN), (N_HIDDEN,), (N_HIDDEN, N_HIDDEN), (N_HIDDEN,), (k, N_HIDDEN), (k,)]
    out, at = [], 0
    for shp in sizes:
        n = int(np.prod(shp))
        out.append(p[at:at + n].reshape(shp))
        at += n
    return out


def pack(W1, b1, W2, b2, W3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(a).astype(np.float64) for a in (W1, b1, W2, b2, W3, b3)])


def forward(params, k: int, x):
    """Outputs (B, K) and the intermediates (z1, h1, z2, h2)."""
    W1, b1, W2, b2, W3, b3 = unpack(params, k)
    x = np.asarray(x, dtype=np.float64).reshape(-1, N_IN)
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3.T + b3
    return y, (x, z1, h1, z2, h2)


def loss(params, k: int, x, target, weight) -> float:
    y, _ = forward(params, k, x)
    t = np.asarray(target, dtype=np.float64).reshape(y.shape)
    m = np.asarray(weight, dtype=np.float64).reshape(y.shape)
    b = y.shape[0]
    if b == 0:
        return 0.0
    per = (m * (y - t) ** 2).sum(axis=1) / np.maximum(m.sum(axis=1), 1.0)
    return float(per.sum() / b)


def loss_and_grad(params, k: int, x, target, weight):
    """Loss and its gradient with respect to the flat parameters (chain rule
    through the three layers; the ReLU derivative is taken as 0 at 0)."""
    y, (x, z1, h1, z2, h2) = forward(params, k, x)
    _, _, W2, _, W3, _ = unpack(params, k)
    t = np.asarray(target, dtype=np.float64).reshape(y.shape)
    m = np.asarray(weight, dtype=np.float64).reshape(y.shape)
    b = y.shape[0]
    if b == 0:
        return 0.0, np.zeros(param_count(k))
    norm = 1.0 / (np.maximum(m.sum(axis=1), 1.0) * b)  # (B,)
    e = y - t
    L = float((m * e * e * norm[:, None]).sum())
    dy = 2.0 * m * e * norm[:, None]  # dL/dy
    dW3 = dy.T @ h2
    db3 = dy.sum(axis=0)
    dh2 = dy @ W3
    dz2 = dh2 * (z2 > 0)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0)
    dW1 = dz1.T @ x
    db1 = dz1.sum(axis=0)
    return L, pack(dW1, db1, dW2, db2, dW3, db3)


def adam_step(params, m, v, grad, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """Adam (Kingma and Ba) with bias correction; returns new (params, m, v)."""
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    p = np.asarray(params, dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def init_params(k: int, seed: int) -> np.ndarray:
    """He-style random initial weights, zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, np.sqrt(2.0 / N_IN), (N_HIDDEN, N_IN))
    W2 = rng.normal(0, np.sqrt(2.0 / N_HIDDEN), (N_HIDDEN, N_HIDDEN))
    W3 = rng.normal(0, np.sqrt(1.0 / N_HIDDEN), (k, N_HIDDEN))
    return pack(W1, np.zeros(N_HIDDEN), W2, np.zeros(N_HIDDEN), W3, np.zeros(k))
