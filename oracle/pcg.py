"""Preconditioned conjugate gradients and the matvec-error metric (oracle).

Section 6 solves the kernel systems with PCG preconditioned by the SPD HSS
approximation, random right-hand sides, and a relative-residual stopping
threshold.  Readings: x0 = 0; every right-hand-side column runs its own
(Hestenes-Stiefel) recurrence and stops once its recursively updated residual
satisfies ||r|| <= rtol * ||b||; the true residual ||b - A x|| / ||b|| is then
reported from one extra product.  A column whose curvature p^T A p or
r^T z is not positive (not a finite positive number) stops at that step
without updating x: in exact arithmetic both are positive whenever A and M are
SPD, which the method assumes of its input, so the column reports a breakdown
instead of iterating on an indefinite operator.

Section 6.1 measures approximation accuracy as the mean relative 2-norm error
of products with Gaussian random vectors, the H^2 product being the reference.
"""
from __future__ import annotations

import numpy as np


def pcg(apply_A, apply_M, b: np.ndarray, rtol: float, maxit: int, return_breakdown: bool = False):
    """Returns (x, iterations per column, true relative residual per column),
    and with return_breakdown a boolean per column: it stopped on
    non-positive curvature."""
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
    breakdown = np.zeros(m, dtype=bool)
    for _ in range(maxit):
        if not active.any():
            break
        q = apply_A(p)
        pq = np.einsum("ij,ij->j", p, q)
        with np.errstate(invalid="ignore"):
            bad = active & ~((pq > 0) & (rz > 0))
        breakdown |= bad
        active = active & ~bad
        alpha = np.where(active, rz / np.where(active, pq, 1.0), 0.0)
        x = np.where(active, x + alpha * p, x)
        r = np.where(active, r - alpha * q, r)
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
        out = (x[:, 0], iters, res)
    else:
        out = (x, iters, res)
    return out + (breakdown,) if return_breakdown else out


def matvec_error(apply_ref, apply_approx, n: int, nvec: int = 10, seed: int = 0) -> float:
    """Mean relative 2-norm error of apply_approx against apply_ref over nvec
    Gaussian vectors (Section 6.1 accuracy metric)."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, nvec))
    Yr, Ya = apply_ref(X), apply_approx(X)
    return float(np.mean(np.linalg.norm(Yr - Ya, axis=0) / np.linalg.norm(Yr, axis=0)))
