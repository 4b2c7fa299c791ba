"""The controller network 16 -> 64 -> 64 -> 3 (ReLU hidden layers, linear output),
its mean-squared-error loss, the gradient by backpropagation, and one Adam step,
in float64 NumPy -- the reference for the device kernels.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Parameter vector layout (shared as a document with the device code):
W1 [64][16], b1 [64], W2 [64][64], b2 [64], W3 [3][64], b3 [3]  (row-major).
Loss: L = (1 / (3 B)) sum_{b, o} (y_bo - t_bo)^2 over a batch of B samples.
Adam (Kingma & Ba, ICLR 2015): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 16, 64, 3
SHAPES = [(N_HID, N_IN), (N_HID,), (N_HID, N_HID), (N_HID,), (N_OUT, N_HID), (N_OUT,)]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)


def unpack(p: np.ndarray):
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(p[o:o + n].reshape(s))
        o += n
    return out


def forward(p: np.ndarray, X: np.ndarray):
    """Returns (Y, cache) for inputs X (B x 16)."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(p, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ W1.T + b1
    A1 = np.maximum(Z1, 0.0)
    Z2 = A1 @ W2.T + b2
    A2 = np.maximum(Z2, 0.0)
    Y = A2 @ W3.T + b3
    return Y, (X, Z1, A1, Z2, A2)


def loss(p, X, T) -> float:
    Y, _ = forward(p, X)
    return float(np.mean((Y - np.asarray(T, dtype=np.float64)) ** 2))


def loss_grad(p, X, T):
    """(loss, gradient) by backpropagation through the layers above."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(p, dtype=np.float64))
    Y, (X, Z1, A1, Z2, A2) = forward(p, X)
    T = np.asarray(T, dtype=np.float64)
    B = X.shape[0]
    dY = 2.0 * (Y - T) / (B * N_OUT)
    gW3 = dY.T @ A2
    gb3 = dY.sum(axis=0)
    dZ2 = (dY @ W3) * (Z2 > 0.0)
    gW2 = dZ2.T @ A1
    gb2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2) * (Z1 > 0.0)
    gW1 = dZ1.T @ X
    gb1 = dZ1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return float(np.mean((Y - T) ** 2)), g


def adam_step(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step number t >= 1); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            lim = np.sqrt(6.0 / s[1])
            parts.append(rng.uniform(-lim, lim, size=s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts)
