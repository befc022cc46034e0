"""FP64 reference of the learned triplet scorer (TEST INFRASTRUCTURE ONLY).

Network: 12 -> 64 -> 64 -> 1, ReLU, ReLU, logistic output, binary cross-entropy loss, Adam.
Weights are used at BF16 precision (round-to-nearest-even of their FP32 master values);
everything else here is float64.

Parameter vector layout (5057 values): W1[12][64], b1[64], W2[64][64], b2[64], w3[64], b3.
"""
from __future__ import annotations

import numpy as np

N_PARAMS = 5057
SLICES = {"W1": (0, 768, (12, 64)), "b1": (768, 832, (64,)), "W2": (832, 4928, (64, 64)),
          "b2": (4928, 4992, (64,)), "w3": (4992, 5056, (64,)), "b3": (5056, 5057, (1,))}
WEIGHT_KEYS = ("W1", "W2", "w3")


def unpack(theta: np.ndarray) -> dict:
    return {k: theta[a:b].reshape(shape) for k, (a, b, shape) in SLICES.items()}


def pack(parts: dict) -> np.ndarray:
    out = np.zeros(N_PARAMS)
    for k, (a, b, _) in SLICES.items():
        out[a:b] = np.asarray(parts[k], dtype=np.float64).reshape(-1)
    return out


def bf16_round(x) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), via the float32 bit pattern."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def quantize(theta: np.ndarray) -> np.ndarray:
    """The parameters the scorer computes with: BF16 weights, FP32 biases."""
    parts = unpack(np.asarray(theta, dtype=np.float64))
    q = {}
    for k, v in parts.items():
        q[k] = bf16_round(v) if k in WEIGHT_KEYS else np.asarray(v, dtype=np.float32).astype(np.float64)
    return pack(q)


def forward(theta: np.ndarray, X: np.ndarray):
    """Logits for feature rows X [B, 12]; returns (logits, cache)."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ p["w3"] + p["b3"][0]
    return z3, (X, z1, h1, z2, h2)


def bce_loss(logits: np.ndarray, y: np.ndarray) -> float:
    """Mean binary cross-entropy of sigmoid(logits) against labels y, in the stable form
    softplus(z) - y z."""
    z = np.asarray(logits, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return float(np.mean(np.logaddexp(0.0, z) - y * z))


def backward(theta: np.ndarray, X: np.ndarray, y: np.ndarray) -> tuple[float, np.ndarray]:
    """Loss and its gradient with respect to all 5057 parameters (chain rule by hand)."""
    p = unpack(theta)
    z3, (X, z1, h1, z2, h2) = forward(theta, X)
    B = X.shape[0]
    y = np.asarray(y, dtype=np.float64)
    dz3 = (1.0 / (1.0 + np.exp(-z3)) - y) / B
    g = {"b3": np.array([dz3.sum()]), "w3": h2.T @ dz3}
    dz2 = np.outer(dz3, p["w3"]) * (z2 > 0)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"].T) * (z1 > 0)
    g["W1"] = X.T @ dz1
    g["b1"] = dz1.sum(0)
    return bce_loss(z3, y), pack(g)


def adam_step(theta, m, v, grad, step: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1); ``step`` counts from 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mhat = m / (1 - b1 ** step)
    vhat = v / (1 - b2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
