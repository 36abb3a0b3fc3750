"""Kernel functions K(x, y) on 3-D points (oracle; test infrastructure only).

Section 6 lists the Matern-3/2, Gaussian and inverse multiquadric kernels with
a multiplicative parameter l.  The workloads used here give them with a length
scale ell instead; this module follows the length-scale forms:

* gaussian:    exp(-r^2 / ell^2)
* matern32:    (1 + sqrt(3) r / ell) exp(-sqrt(3) r / ell)
* exponential: exp(-r / ell)
* imq:         1 / sqrt(r^2 + ell^2)          (ell plays the role of c)

The shifted matrix sigma*I + K(X, X) of Section 6.2 is formed by callers.
"""
from __future__ import annotations

import numpy as np

KINDS = ("gaussian", "matern32", "exponential", "imq")


def sqdist(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Squared Euclidean distances, summed per coordinate (no Gram trick)."""
    dx = X[:, 0][:, None] - Y[:, 0][None, :]
    dy = X[:, 1][:, None] - Y[:, 1][None, :]
    dz = X[:, 2][:, None] - Y[:, 2][None, :]
    return dx * dx + dy * dy + dz * dz


def evaluate(kind: str, ell: float, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Dense kernel block K(X, Y) of shape (len(X), len(Y))."""
    r2 = sqdist(np.asarray(X, dtype=np.float64), np.asarray(Y, dtype=np.float64))
    if kind == "gaussian":
        return np.exp(-r2 / (ell * ell))
    if kind == "matern32":
        t = np.sqrt(3.0) * np.sqrt(r2) / ell
        return (1.0 + t) * np.exp(-t)
    if kind == "exponential":
        return np.exp(-np.sqrt(r2) / ell)
    if kind == "imq":
        return 1.0 / np.sqrt(r2 + ell * ell)
    raise ValueError(f"unknown kernel {kind!r}")
