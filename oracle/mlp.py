"""Cost-model MLP oracle -- TEST INFRASTRUCTURE ONLY (numpy float64).

The learned cost model maps 32 expression-tree features to a predicted
(standardised) log-time for each of 64 launch configurations:

    Z1 = X W1 + b1          X: (B, 32)  W1: (32, 64)  b1: (64,)
    H  = max(Z1, 0)
    Y  = H W2 + b2          W2: (64, 64) b2: (64,)
    L  = sum(M * (Y - T)^2) / sum(M)     M: 0/1 mask of measured entries

trained with Adam (Kingma and Ba, "Adam: A Method for Stochastic
Optimization", ICLR 2015, Algorithm 1).  Everything is plain float64 numpy,
one matrix product per layer, no fusion.  Row-major weights, W[i, j] connects
input i to output j.
"""
from __future__ import annotations

from typing import Dict

import numpy as np

N_IN, N_HID, N_OUT = 32, 64, 64


def forward(p: Dict[str, np.ndarray], X: np.ndarray):
    Z1 = X @ p["W1"] + p["b1"]
    H = np.maximum(Z1, 0.0)
    Y = H @ p["W2"] + p["b2"]
    return Y, (X, Z1, H)


def loss(Y: np.ndarray, T: np.ndarray, M: np.ndarray) -> float:
    return float(np.sum(M * (Y - T) ** 2) / np.sum(M))


def backward(p: Dict[str, np.ndarray], cache, Y: np.ndarray, T: np.ndarray, M: np.ndarray):
    X, Z1, H = cache
    dY = 2.0 * M * (Y - T) / np.sum(M)
    g = {}
    g["W2"] = H.T @ dY
    g["b2"] = dY.sum(axis=0)
    dH = dY @ p["W2"].T
    dZ1 = dH * (Z1 > 0.0)
    g["W1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return g


def adam_step(w: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, t: int,
              lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update in place (t is the 1-based step count)."""
    m *= b1
    m += (1.0 - b1) * g
    v *= b2
    v += (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    w -= lr * mhat / (np.sqrt(vhat) + eps)


def init_params(g: np.random.Generator) -> Dict[str, np.ndarray]:
    """He-uniform first layer, Glorot-uniform second layer, zero biases."""
    l1 = np.sqrt(6.0 / N_IN)
    l2 = np.sqrt(6.0 / (N_HID + N_OUT))
    return {
        "W1": g.uniform(-l1, l1, (N_IN, N_HID)),
        "b1": np.zeros(N_HID),
        "W2": g.uniform(-l2, l2, (N_HID, N_OUT)),
        "b2": np.zeros(N_OUT),
    }
