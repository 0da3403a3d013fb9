"""Pruner MLP in float64 numpy -- test infrastructure only (see the package
docstring for who may import it).

The network is 8 -> 32 -> 32 -> 1 with ReLU hidden layers and a sigmoid
output.  Flat parameter layout (1377 values): W1[32][8], b1[32], W2[32][32],
b2[32], w3[32], b3.  Training minimises the mean weighted binary
cross-entropy
    L = (1/N) sum_k c_k * (softplus(z_k) - y_k z_k),  c_k = pos_weight if y_k = 1 else 1,
whose derivative in the logit is c_k (sigmoid(z_k) - y_k) / N, with Adam
(Kingma and Ba, 2015; beta1 0.9, beta2 0.999, eps 1e-8).
"""
from __future__ import annotations

import numpy as np

IN, H = 8, 32
N_PARAMS = H * IN + H + H * H + H + H + 1
_SL = {
    "W1": (0, H * IN), "b1": (H * IN, H * IN + H), "W2": (H * IN + H, H * IN + H + H * H),
    "b2": (H * IN + H + H * H, H * IN + 2 * H + H * H), "w3": (H * IN + 2 * H + H * H, H * IN + 3 * H + H * H),
    "b3": (H * IN + 3 * H + H * H, N_PARAMS),
}
BETA1, BETA2, EPS = 0.9, 0.999, 1e-8
_M64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    g = {k: w[a:b] for k, (a, b) in _SL.items()}
    return g["W1"].reshape(H, IN), g["b1"], g["W2"].reshape(H, H), g["b2"], g["w3"], g["b3"][0]


def forward(w, X):
    """Logits z [N] and the activations needed by the backward pass."""
    W1, b1, W2, b2, w3, b3 = unpack(w)
    X = np.asarray(X, dtype=np.float64).reshape(-1, IN)
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ w3 + b3
    return z, (X, a1, h1, a2, h2)


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * np.asarray(z, dtype=np.float64)))


def loss(w, X, y, pos_weight: float) -> float:
    z, _ = forward(w, X)
    y = np.asarray(y, dtype=np.float64)
    c = np.where(y > 0.5, pos_weight, 1.0)
    return float(np.mean(c * (np.logaddexp(0.0, z) - y * z)))


def loss_grad(w, X, y, pos_weight: float):
    """(loss, gradient [N_PARAMS]) by explicit back-propagation."""
    z, (X, a1, h1, a2, h2) = forward(w, X)
    W1, b1, W2, b2, w3, b3 = unpack(w)
    y = np.asarray(y, dtype=np.float64)
    n = max(len(y), 1)
    c = np.where(y > 0.5, pos_weight, 1.0)
    L = float(np.sum(c * (np.logaddexp(0.0, z) - y * z)) / n)
    dz = c * (sigmoid(z) - y) / n
    g = np.zeros(N_PARAMS)
    g[_SL["w3"][0]:_SL["w3"][1]] = h2.T @ dz
    g[_SL["b3"][0]] = dz.sum()
    da2 = np.outer(dz, w3) * (a2 > 0)
    g[_SL["W2"][0]:_SL["W2"][1]] = (da2.T @ h1).ravel()
    g[_SL["b2"][0]:_SL["b2"][1]] = da2.sum(0)
    da1 = (da2 @ W2) * (a1 > 0)
    g[_SL["W1"][0]:_SL["W1"][1]] = (da1.T @ X).ravel()
    g[_SL["b1"][0]:_SL["b1"][1]] = da1.sum(0)
    return L, g


def adam_step(w, g, m, v, step: int, lr: float):
    """One Adam update (step counts from 1); returns new (w, m, v)."""
    m = BETA1 * m + (1 - BETA1) * g
    v = BETA2 * v + (1 - BETA2) * g * g
    mh = m / (1 - BETA1 ** step)
    vh = v / (1 - BETA2 ** step)
    return w - lr * mh / (np.sqrt(vh) + EPS), m, v


def splitmix64(x: int) -> int:
    """SplitMix64 output for counter value x (Steele, Lea and Flood, 2014)."""
    z = (x + _GAMMA) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def glorot_init(seed: int) -> np.ndarray:
    """Glorot-uniform weights, zero biases, in float32: parameter k of the flat
    layout draws u = (splitmix64(seed + k * gamma) >> 40) / 2^24 and becomes
    (2u - 1) * sqrt(6 / (fan_in + fan_out)), all in float32."""
    w = np.zeros(N_PARAMS, dtype=np.float32)
    for name, fi, fo in (("W1", IN, H), ("W2", H, H), ("w3", H, 1)):
        a, b = _SL[name]
        lim = np.sqrt(np.float32(6.0) / np.float32(fi + fo), dtype=np.float32)
        for k in range(a, b):
            u = np.float32((splitmix64((seed + k * _GAMMA) & _M64) >> 40) * 2.0 ** -24)
            w[k] = (np.float32(2.0) * u - np.float32(1.0)) * lim
    return w
