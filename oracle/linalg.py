"""Dense building blocks for the oracle (test infrastructure only).

Cholesky factors, triangular solves and symmetric eigen-decompositions are
unique results with plain definitions, so library routines serve for them.
Column-pivoted QR is written out here because its pivot choice is part of the
result (Algorithm 5.1, step 3) and library routines use their own norm-update
and tie rules.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.linalg as sla

_HERE = os.path.dirname(os.path.abspath(__file__))
_CSRC = os.path.join(_HERE, "cpqr.c")
_CLIB = os.path.join(_HERE, "_cpqr.so")
_clib = None


def build_c() -> str:
    """Compile oracle/cpqr.c with gcc into oracle/_cpqr.so (plain IEEE
    arithmetic: no fast-math, no contraction)."""
    tmp = f"{_CLIB}.{os.getpid()}.tmp"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
                    "-o", tmp, _CSRC, "-lm"], check=True, capture_output=True)
    os.replace(tmp, _CLIB)
    return _CLIB


def _c_cpqr():
    """The C pivoted QR, built on first use; None where no compiler is found."""
    global _clib
    if _clib is None:
        try:
            if not os.path.exists(_CLIB) or os.path.getmtime(_CLIB) < os.path.getmtime(_CSRC):
                build_c()
            lib = ctypes.CDLL(_CLIB)
            P = ctypes.c_void_p
            lib.oracle_cpqr.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_double, ctypes.c_int,
                                        P, P, P, P]
            lib.oracle_cpqr.restype = ctypes.c_int
            _clib = lib
        except (OSError, subprocess.CalledProcessError):
            _clib = False
    return _clib or None


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

    def __init__(self, M: np.ndarray, tol: float, max_rank: int, use_c: bool = True):
        m, n = np.shape(M)
        kmax = min(m, n, max(int(max_rank), 0))
        lib = _c_cpqr() if use_c and m * n > 0 else None
        if lib is not None:
            self._factor_c(lib, M, tol, kmax)
            return
        A = np.array(M, dtype=np.float64, copy=True)
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

    def _factor_c(self, lib, M, tol, kmax):
        """The same factorization by oracle/cpqr.c (column-major copy of M)."""
        A = np.array(M, dtype=np.float64, order="F", copy=True)
        m, n = A.shape
        piv = np.zeros(max(kmax, 1), dtype=np.int32)
        alpha = np.zeros(max(kmax, 1))
        betas = np.zeros(max(kmax, 1))
        V = np.zeros((m, max(kmax, 1)), order="F")
        r = lib.oracle_cpqr(m, n, A.ctypes.data, float(tol), int(kmax), piv.ctypes.data,
                            alpha.ctypes.data, betas.ctypes.data, V.ctypes.data)
        used = np.zeros(n, dtype=bool)
        used[piv[:r]] = True
        self.m, self.n = m, n
        self.rank = r
        self.piv = piv[:r].astype(np.int64)
        self.perm = np.concatenate([self.piv, np.flatnonzero(~used).astype(np.int64)])
        self._vs = [V[t:, t].copy() for t in range(r)]
        self._betas = [float(b) for b in betas[:r]]
        sign = np.where(alpha[:r] < 0, -1.0, 1.0)
        self._sign = sign
        R = A[:r, :][:, self.perm] if r else np.zeros((0, n))
        self.R = sign[:, None] * R if r else R
        self.diag = np.abs(alpha[:r])

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
