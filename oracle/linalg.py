"""Dense building blocks for the oracle (test infrastructure only).

Cholesky factors, triangular solves and symmetric eigen-decompositions are
unique results with plain definitions, so library routines serve for them.
Column-pivoted QR is written out here because its pivot choice is part of the
result (Algorithm 5.1, step 3) and library routines use their own norm-update
and tie rules.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def chol(A: np.ndarray) -> np.ndarray:
    """Lower Cholesky factor S with A = S S^T; raises LinAlgError if A is not SPD."""
    return np.linalg.cholesky(A)


def lsolve(L: np.ndarray, B: np.ndarray) -> np.ndarray:
    """L^{-1} B for lower-triangular L."""
    if B.shape[0] == 0:
        return B.copy()
    return sla.solve_triangular(L, B, lower=True)


def ltsolve(L: np.ndarray, B: np.ndarray) -> np.ndarray:
    """L^{-T} B for lower-triangular L."""
    if B.shape[0] == 0:
        return B.copy()
    return sla.solve_triangular(L, B, lower=True, trans="T")


def sym_sqrt_pair(M: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """(M^{1/2}, M^{-1/2}) of an SPD matrix by eigen-decomposition (eq. Si0)."""
    w, Q = np.linalg.eigh(M)
    if w.size and w.min() <= 0:
        raise np.linalg.LinAlgError("matrix is not positive definite")
    sq = np.sqrt(w)
    return (Q * sq) @ Q.T, (Q / sq) @ Q.T


class CPQR:
    """Householder QR with column pivoting, M[:, piv] = Q R.

    Step t picks, among the columns not yet chosen, the one whose trailing
    part (rows t..m-1) has the largest 2-norm, recomputed exactly from the
    current matrix (no norm down-dating); ties go to the lowest column
    index.  Columns are not moved: the pivot order is recorded instead.

    The factorization stops before step t when t reaches max_rank, min(m, n),
    or when the pivot norm |R_tt| is not larger than tol * |R_00|; the number
    of steps taken is the rank.  Diagonal entries of R are made non-negative
    by flipping the sign of the matching Q column and R row.
    """

    def __init__(self, M: np.ndarray, tol: float, max_rank: int):
        A = np.array(M, dtype=np.float64, copy=True)
        m, n = A.shape
        kmax = min(m, n, max(int(max_rank), 0))
        used = np.zeros(n, dtype=bool)
        piv, vs, betas, diag = [], [], [], []
        ref = None
        for t in range(kmax):
            sub = A[t:, :]
            norms2 = np.einsum("ij,ij->j", sub, sub)
            norms2[used] = -1.0
            j = int(np.argmax(norms2))  # first maximum: lowest index on ties
            nrm = float(np.sqrt(norms2[j]))
            if ref is None:
                ref = nrm
            if not (nrm > tol * ref) or nrm == 0.0:
                break
            x = A[t:, j].copy()
            alpha = -nrm if x[0] >= 0 else nrm     # H x = alpha e_1
            v = x
            v[0] -= alpha
            vnorm2 = float(v @ v)
            beta = 2.0 / vnorm2 if vnorm2 > 0 else 0.0
            # apply H = I - beta v v^T to rows t.. of every column
            w = v @ A[t:, :]
            A[t:, :] -= beta * np.outer(v, w)
            A[t:, j] = 0.0
            A[t, j] = alpha
            used[j] = True
            piv.append(j)
            vs.append(v)
            betas.append(beta)
            diag.append(alpha)
        self.m, self.n = m, n
        self.rank = len(piv)
        self.piv = np.array(piv, dtype=np.int64)
        rest = [j for j in range(n) if not used[j]]
        self.perm = np.concatenate([self.piv, np.array(rest, dtype=np.int64)])
        self._vs, self._betas = vs, betas
        sign = np.where(np.array(diag) < 0, -1.0, 1.0) if diag else np.zeros(0)
        self._sign = sign
        # R in pivot order: rows 0..rank-1, all n columns
        R = A[: self.rank, :][:, self.perm] if self.rank else np.zeros((0, n))
        self.R = sign[:, None] * R if self.rank else R
        self.diag = np.abs(np.array(diag))

    def q(self) -> np.ndarray:
        """First rank columns of Q (m x rank), orthonormal."""
        m, r = self.m, self.rank
        Q = np.zeros((m, r))
        Q[np.arange(r), np.arange(r)] = 1.0
        for t in range(r - 1, -1, -1):
            v, b = self._vs[t], self._betas[t]
            Q[t:, :] -= b * np.outer(v, v @ Q[t:, :])
        return Q * self._sign[None, :] if r else Q

    def interp(self) -> np.ndarray:
        """E = R11^{-1} R12 for the interpolative decomposition (rank x (n-rank))."""
        r = self.rank
        if r == 0:
            return np.zeros((0, self.n))
        return sla.solve_triangular(self.R[:, :r], self.R[:, r:], lower=False)
