"""Kernel functions K(x, y) on 3-D points (oracle; test infrastructure only).

Section 6 lists the Matern-3/2, Gaussian and inverse multiquadric kernels with
a multiplicative parameter l.  The workloads used here give them with a length
scale ell instead; this module follows the length-scale forms:

* gaussian:    exp(-r^2 / ell^2)
* matern32:    (1 + sqrt(3) r / ell) exp(-sqrt(3) r / ell)
* exponential: exp(-r / ell)
* imq:         1 / sqrt(r^2 + ell^2)          (ell plays the role of c)
* rpy:         the Rotne-Prager-Yamakawa 3 x 3 tensor of Section 6 with particle
               radius a = ell, for r = x - y and rr = r r^T / |r|^2:
                 I / a                                          if r = 0
                 3/(4|r|) (I + rr) + 3a^2/(2|r|^3) (I/3 - rr)   if |r| >= 2a
                 (1/a)(1 - 9|r|/(32a)) I + 3|r|/(32a^2) rr      if |r| < 2a
               The printed overlapping form lacks the second 1/a; with it
               the two branches agree at |r| = 2a (both 7/(16a) I + 3/(16a) rr),
               as the tensor's physical form requires.

A tensor kernel acts on 3N rows, row 3p + c being component c of point p:
evaluate() takes the component of every row and column (cx, cy) and returns
the entries T(x - y)[cx, cy].

The shifted matrix sigma*I + K(X, X) of Section 6.2 is formed by callers.
"""
from __future__ import annotations

import numpy as np

KINDS = ("gaussian", "matern32", "exponential", "imq", "rpy")
TENSOR = ("rpy",)  # kernels whose value is a 3 x 3 tensor


def sqdist(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Squared Euclidean distances, summed per coordinate (no Gram trick)."""
    dx = X[:, 0][:, None] - Y[:, 0][None, :]
    dy = X[:, 1][:, None] - Y[:, 1][None, :]
    dz = X[:, 2][:, None] - Y[:, 2][None, :]
    return dx * dx + dy * dy + dz * dz


def rpy(a: float, X: np.ndarray, Y: np.ndarray, cx, cy) -> np.ndarray:
    """Entries T(x_i - y_j)[cx_i, cy_j] of the RPY tensor (radius a)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    cx = np.asarray(cx)
    cy = np.asarray(cy)
    d = [X[:, k][:, None] - Y[:, k][None, :] for k in range(3)]
    r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
    r = np.sqrt(r2)
    di = np.choose(cx[:, None] * np.ones_like(r, dtype=np.int64), d)
    dj = np.choose(cy[None, :] * np.ones_like(r, dtype=np.int64), d)
    eye = (cx[:, None] == cy[None, :]).astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        rr = np.where(r2 > 0.0, di * dj / r2, 0.0)
        far = 0.75 / r * (eye + rr) + 1.5 * a * a / (r2 * r) * (eye / 3.0 - rr)
        near = (1.0 - 9.0 * r / (32.0 * a)) / a * eye + 3.0 * r / (32.0 * a * a) * rr
    return np.where(r2 == 0.0, eye / a, np.where(r >= 2.0 * a, far, near))


def evaluate(kind: str, ell: float, X: np.ndarray, Y: np.ndarray, cx=None, cy=None) -> np.ndarray:
    """Dense kernel block K(X, Y) of shape (len(X), len(Y)); for a tensor
    kernel, X and Y are the points of the rows and columns and cx, cy their
    components."""
    if kind == "rpy":
        return rpy(ell, X, Y, cx, cy)
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
