"""FP64 reference of the learned slope limiter's network and its training step.

TEST INFRASTRUCTURE ONLY.  A plain NumPy statement of the 4 -> 32 -> 32 -> 1
ReLU network that replaces the generalised-minmod limiter of eq. MinMod,
its hand-written backward pass (chain rule, checked against central finite
differences in the tests), the mean-squared-error loss and one Adam update.

Parameter layout (one flat vector of NPARAM values, the same order the GPU
library takes): W1[32][4], b1[32], W2[32][32], b2[32], w3[32], b3[1].
"""
from __future__ import annotations

import numpy as np

IN, H = 4, 32
NPARAM = H * IN + H + H * H + H + H + 1


def unpack(P):
    P = np.asarray(P, dtype=np.float64)
    o = 0
    W1 = P[o:o + H * IN].reshape(H, IN); o += H * IN
    b1 = P[o:o + H]; o += H
    W2 = P[o:o + H * H].reshape(H, H); o += H * H
    b2 = P[o:o + H]; o += H
    w3 = P[o:o + H]; o += H
    b3 = P[o:o + 1]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2),
                           np.ravel(w3), np.ravel(b3)]).astype(np.float64)


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even) through binary32."""
    f = np.asarray(a, dtype=np.float32).copy()
    b = f.view(np.uint32)
    finite = (b & 0x7F800000) != 0x7F800000
    r = (b + (0x7FFF + ((b >> 16) & 1))) & 0xFFFF0000
    b[...] = np.where(finite, r, b)
    return f.astype(np.float64)


def init_params(seed: int = 1207) -> np.ndarray:
    """He-style random initialisation (seeded)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = rng.normal(0, np.sqrt(2.0 / IN), size=(H, IN))
    b1 = np.zeros(H)
    W2 = rng.normal(0, np.sqrt(2.0 / H), size=(H, H))
    b2 = np.zeros(H)
    w3 = rng.normal(0, np.sqrt(1.0 / H), size=H)
    b3 = np.zeros(1)
    return pack(W1, b1, W2, b2, w3, b3)


def forward(P, X, bf16: bool = False):
    """X: (B, 4).  Returns y (B,) and the cache for backward."""
    W1, b1, W2, b2, w3, b3 = unpack(P)
    X = np.asarray(X, dtype=np.float64)
    if bf16:
        X, W1, W2 = bf16_round(X), bf16_round(W1), bf16_round(W2)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    if bf16:
        h1 = bf16_round(h1)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    if bf16:
        h2, w3 = bf16_round(h2), bf16_round(w3)
    y = h2 @ w3 + b3[0]
    return y, (X, W1, W2, w3, z1, h1, z2, h2)


def backward(P, cache, dy):
    """Gradient of sum(dy * y) with respect to every parameter (flat)."""
    X, W1, W2, w3, z1, h1, z2, h2 = cache
    dy = np.asarray(dy, dtype=np.float64)
    g_b3 = np.array([dy.sum()])
    g_w3 = h2.T @ dy
    dh2 = np.outer(dy, w3)
    dz2 = dh2 * (z2 > 0)
    g_W2 = dz2.T @ h1
    g_b2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0)
    g_W1 = dz1.T @ X
    g_b1 = dz1.sum(axis=0)
    return pack(g_W1, g_b1, g_W2, g_b2, g_w3, g_b3)


def loss_and_grad(P, X, T, bf16: bool = False):
    """Mean squared error 1/B sum (y - t)^2 and its gradient."""
    y, cache = forward(P, X, bf16)
    r = y - np.asarray(T, dtype=np.float64)
    B = len(r)
    loss = float(np.sum(r * r) / B)
    g = backward(P, cache, 2.0 * r / B)
    return loss, g


def adam(P, g, m, v, t: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One Adam update (Kingma & Ba); returns new (P, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return P - lr * mh / (np.sqrt(vh) + eps), m, v


def stencil_features(w5):
    """Normalised inputs of the learned limiter for stencils w5 (B, 5):
    the four one-sided differences divided by s = max|d| + 1e-12 (|w_2| + 1e-30).
    Returns (x (B, 4), s (B,), d (B, 4))."""
    w5 = np.asarray(w5, dtype=np.float64)
    d = np.diff(w5, axis=1)
    s = np.max(np.abs(d), axis=1) + 1e-12 * (np.abs(w5[:, 2]) + 1e-30)
    return d / s[:, None], s, d


def tvd_clamp(sigma, dm, dp):
    """0 <= sign(D) sigma <= 2 min(|D-|, |D+|), and 0 where D- D+ <= 0."""
    sigma = np.asarray(sigma, dtype=np.float64)
    sg = np.where(dp > 0, 1.0, -1.0)
    lim = 2.0 * np.minimum(np.abs(dm), np.abs(dp))
    out = sg * np.minimum(np.maximum(sg * sigma, 0.0), lim)
    return np.where(dm * dp <= 0.0, 0.0, out)
