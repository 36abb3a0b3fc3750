"""Preconditioned conjugate gradients and the matvec-error metric (oracle; test infrastructure only).

Section 6 solves the kernel systems with PCG preconditioned by the SPD HSS
approximation, random right-hand sides, and a relative-residual stopping
threshold.  Readings: x0 = 0; every right-hand-side column runs its own
(Hestenes-Stiefel) recurrence and stops once its recursively updated residual
satisfies ||r|| <= rtol * ||b||; the true residual ||b - A x|| / ||b|| is then
reported from one extra product.

Section 6.1 measures approximation accuracy as the mean relative 2-norm error
of products with Gaussian random vectors, the H^2 product being the reference.
"""
from __future__ import annotations

import numpy as np


def pcg(apply_A, apply_M, b: np.ndarray, rtol: float, maxit: int):
    """Returns (x, iterations per column, true relative residual per column)."""
    b = np.asarray(b, dtype=np.float64)
    vec = b.ndim == 1
    if vec:
        b = b[:, None]
    m = b.shape[1]
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.linalg.norm(b, axis=0)
    z = apply_M(r) if apply_M is not None else r.copy()
    p = z.copy()
    rz = np.einsum("ij,ij->j", r, z)
    iters = np.zeros(m, dtype=np.int64)
    active = np.linalg.norm(r, axis=0) > rtol * bn
    for _ in range(maxit):
        if not active.any():
            break
        q = apply_A(p)
        pq = np.einsum("ij,ij->j", p, q)
        alpha = np.where(active, rz / np.where(active, pq, 1.0), 0.0)
        x += alpha * p
        r -= alpha * q
        iters += active
        rn = np.linalg.norm(r, axis=0)
        active = active & (rn > rtol * bn)
        z = apply_M(r) if apply_M is not None else r.copy()
        rz_new = np.einsum("ij,ij->j", r, z)
        beta = np.where(active, rz_new / np.where(active, rz, 1.0), 0.0)
        p = np.where(active, z + beta * p, p)
        rz = np.where(active, rz_new, rz)
    res = np.linalg.norm(b - apply_A(x), axis=0) / np.where(bn > 0, bn, 1.0)
    if vec:
        return x[:, 0], iters, res
    return x, iters, res


def matvec_error(apply_ref, apply_approx, n: int, nvec: int = 10, seed: int = 0) -> float:
    """Mean relative 2-norm error of apply_approx against apply_ref over nvec
    Gaussian vectors (Section 6.1 accuracy metric)."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, nvec))
    Yr, Ya = apply_ref(X), apply_approx(X)
    return float(np.mean(np.linalg.norm(Yr - Ya, axis=0) / np.linalg.norm(Yr, axis=0)))
