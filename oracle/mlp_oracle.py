"""CPU float64 oracle of the learned block-rank predictor (TEST INFRASTRUCTURE ONLY:
imported by tests/, smoke() and the cpu_baseline leg of bench.py, never by the
product path).

The paper truncates every block with a tolerance rule (Section 3); the learned
variant predicts each block's rank from a cheap sketch so that the leaf only
computes the columns it needs, with the tolerance rule kept as fallback and
judge.  This module fixes what the GPU kernels must compute:

  features (16 per block, from the singular values s_1 >= ... >= s_16 of a
  16-column Gaussian sketch Y = A_b Omega and the block energy E = ||A_b||_F^2):
      f_j = max(log10(s_{j+1} / s_1), -16)        j = 1..15
      f_16 = log10(E * 16 / sum_j s_j^2)           (energy the sketch cannot see;
                                                    E[||Y||_F^2] = 16 E)
      (an all-zero block gives f = 0)
  network: h1 = relu(W1 x + b1) (64), h2 = relu(W2 h1 + b2) (64), y = w3 . h2 + b3,
      weights rounded to float16 where they are used (the stored format);
      y predicts log2 of the block's rank under the tolerance rule
  loss: mean over the batch of (y - t)^2 / 2
  training: Adam (beta1 0.9, beta2 0.999, eps 1e-8) on float32 master weights,
      gradients taken at the float16-rounded weights.

parity pinned: the gradients are pinned against central finite differences of the
loss (tests/test_oracle.py), independent of the analytic backward pass.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID = 16, 64
# parameter layout of the flat vector (float32 on the device): W1 (64 x 16, row-major),
# b1 (64), W2 (64 x 64, row-major), b2 (64), w3 (64), b3 (1)
SIZES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
         ("w3", (N_HID,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SIZES])


def fp16(theta: np.ndarray) -> np.ndarray:
    """The stored weight format: round to float16 (nearest even) and back."""
    return np.asarray(theta, dtype=np.float32).astype(np.float16).astype(np.float64)


def features(s: np.ndarray, energy: float) -> np.ndarray:
    """The 16 features of one block from its 16 sketch singular values (descending)."""
    s = np.asarray(s, dtype=np.float64)
    f = np.zeros(N_IN)
    if not (s[0] > 0.0) or not (energy > 0.0):
        return f
    with np.errstate(divide="ignore"):
        f[:15] = np.maximum(np.log10(s[1:16] / s[0]), -16.0)
    f[15] = np.log10(energy * 16.0 / np.sum(s * s))
    return f


def init_params(seed: int) -> np.ndarray:
    """He-style initialisation (seeded), as float32."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.standard_normal((N_HID, N_IN)) * np.sqrt(2.0 / N_IN), "b1": np.zeros(N_HID),
         "W2": rng.standard_normal((N_HID, N_HID)) * np.sqrt(2.0 / N_HID), "b2": np.zeros(N_HID),
         "w3": rng.standard_normal(N_HID) * np.sqrt(1.0 / N_HID), "b3": np.array([3.0])}
    return pack(p).astype(np.float32)


def forward(theta: np.ndarray, X: np.ndarray):
    """Predictions y (batch) and the activations the backward pass needs."""
    p = unpack(theta)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["w3"] + p["b3"][0]
    return y, (X, z1, h1, z2, h2)


def loss(theta: np.ndarray, X: np.ndarray, t: np.ndarray) -> float:
    y, _ = forward(theta, X)
    return float(np.mean((y - t) ** 2) / 2.0)


def grad(theta: np.ndarray, X: np.ndarray, t: np.ndarray):
    """(loss, gradient) of the mean squared error at the given weights (chain rule
    through the three layers)."""
    p = unpack(theta)
    y, (X, z1, h1, z2, h2) = forward(theta, X)
    B = X.shape[0]
    dy = (y - t) / B
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()])}
    dz2 = np.outer(dy, p["w3"]) * (z2 > 0.0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"]) * (z1 > 0.0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return float(np.mean((y - t) ** 2) / 2.0), pack(g)


def adam(master: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, step: int, lr: float,
         b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step counts from 1); returns new (master, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return master - lr * mh / (np.sqrt(vh) + eps), m, v


def train(master: np.ndarray, X: np.ndarray, t: np.ndarray, steps: int, lr: float, batch: int = 64):
    """Minibatch b of step s takes samples (s * batch + i) mod count, i < batch;
    gradients at the float16-rounded weights, updates on the float64 master copy."""
    master = np.asarray(master, dtype=np.float64).copy()
    m = np.zeros_like(master)
    v = np.zeros_like(master)
    n = X.shape[0]
    losses = []
    for s in range(steps):
        idx = (s * batch + np.arange(batch)) % n
        L, g = grad(fp16(master), X[idx], t[idx])
        master, m, v = adam(master, g, m, v, s + 1, lr)
        losses.append(L)
    return master, losses
