"""Accelerated SPD HSS construction, Algorithm 5.3 (oracle; test infrastructure only).

Follows Algorithm 5.3 step by step on an H^2 matrix (oracle.h2.H2):

1. Sampling (eq. Yk): Y^(k) = (A - diag({A_ii}_{i in lvl(k)})) Omega for
   k = 1..L-1, each by one level-masked H^2 product.
2. Leaf level: A_ii = S_i S_i^T (Cholesky); Lambda Omega = S_i^{-1} Y_i^(1);
   V_i from the pivoted QR of it (Algorithm 5.1, step 3); Phi_i U_i^H2 =
   V_i^T S_i^{-1} U_i^H2; B_ij = V_i^T S_i^{-1} A_ij S_j^{-T} V_j for Type-1
   pairs (the algorithm's printed trailing transpose on V_j is a typo: the
   product must end with V_j) and B_ij = (Phi_i U_i)(B_ij^H2)(Phi_j U_j)^T for
   Type-3 pairs (eq. type3_Mij); U_i = S_i V_i.
3. Levels k = 2..L-1: bold B_ii from the children's sibling couplings
   (eq. Aii0); the factor F_i of I + bold B_ii; Lambda Omega =
   F_i^{-1} diag(Phi_c) Y_i^(k) through Algorithm 5.2; V-bar_i from its pivoted
   QR; Phi_i U_i^H2 by the nested recursion of Section 5.2.2 Case 1; Type-1
   B_ij = V-bar_i^T F_i^{-1} bold B_ij F_j^{-T} V-bar_j (eq. Mijk); Type-3 B_ij
   by eq. type3_Mij; R_i = F_i V-bar_i (eq. Rik).

Two forms of F_i are provided:

* variant="eig": F_i = (I + bold B_ii)^{1/2} from an eigen-decomposition, as
  printed (eq. Si0);
* variant="chol": F_i = the lower Cholesky factor of I + bold B_ii.  Any
  F F^T = I + bold B_ii gives a valid symmetric factor S_i = diag(S_c) S-bar_i
  with S-bar_i = I - V V^T + V F V^T, and F_chol = F_sqrt Q for an orthogonal
  Q.  The pivoted QR of Q^T Psi has the same pivots and R as that of Psi, so
  V-bar differs by Q^T while Phi_i, R_i, B_ij and U_i are unchanged.  The
  tests pin this equivalence.

Readings where the paper is silent: the rank rule r_i = min(max_rank,
#{t : |R_tt| > tol*|R_00|}, rows, columns) serves both the fixed-rank
(tol = 0) and the threshold forms (Section 5.2.3 mentions an error-threshold
form without details); and the root factor F_root of I + bold B_root is
computed for the solve (the algorithm stops at level L-1).
"""
from __future__ import annotations

import numpy as np

from .h2 import H2
from .linalg import CPQR, chol, lsolve, ltsolve, sym_sqrt_pair


class SPDHSS:
    def __init__(self, h2: H2, omega_tree: np.ndarray, tol: float, max_rank: int,
                 variant: str = "chol"):
        if variant not in ("chol", "eig"):
            raise ValueError(variant)
        self.h2, self.tree = h2, h2.tree
        self.tol, self.max_rank, self.variant = float(tol), int(max_rank), variant
        T = self.tree
        L = T.L
        self.Omega = np.asarray(omega_tree, dtype=np.float64)
        # step 1: sampling, one masked H^2 product per nonroot level (eq. Yk)
        self.Y = {k: h2.matvec(self.Omega, above=k) for k in range(1, L)}
        self.S, self.V, self.Z, self.PhiU = {}, {}, {}, {}
        self.F, self.Finv, self.Vbar, self.R = {}, {}, {}, {}
        self.Bc = {}      # HSS coefficient matrices, keyed (i, j)
        self.piv, self.rank, self.Rdiag = {}, {}, {}
        self.Psi = {}
        if L == 1:
            self.S[0] = chol(h2.near_blocks[(0, 0)])
            return
        self._leaf_level()
        for k in range(2, L):
            self._level(k)
        self._root()

    # -- helpers ---------------------------------------------------------------
    def _compress(self, v: int, Psi: np.ndarray) -> np.ndarray:
        f = CPQR(Psi, self.tol, self.max_rank)
        self.piv[v], self.rank[v], self.Rdiag[v] = f.piv, f.rank, f.diag
        self.Psi[v] = Psi
        return f.q()

    def _finv(self, v: int, X: np.ndarray) -> np.ndarray:
        if self.variant == "chol":
            return lsolve(self.F[v], X)
        return self.Finv[v] @ X

    def _finvT(self, v: int, X: np.ndarray) -> np.ndarray:
        if self.variant == "chol":
            return ltsolve(self.F[v], X)
        return self.Finv[v] @ X

    def _factor(self, v: int, M: np.ndarray):
        if self.variant == "chol":
            self.F[v] = chol(M)
        else:
            self.F[v], self.Finv[v] = sym_sqrt_pair(M)

    def bold_B(self, i: int, j: int) -> np.ndarray:
        """Concatenation [B_{c_a d_b}] of the children blocks of (i, j); the
        diagonal child blocks of bold B_ii are zero (eq. Aii0)."""
        T = self.tree
        ci, cj = T.children(i), T.children(j)
        rows = []
        for a in ci:
            row = []
            for b in cj:
                if a == b:
                    row.append(np.zeros((self.rank[a], self.rank[b])))
                else:
                    row.append(self.Bc[(a, b)])
            rows.append(row)
        return np.block(rows)

    def _couplings(self, k: int):
        T, h2 = self.tree, self.h2
        for i in T.nodes_at(k):
            for j in T.near[i]:
                if j == i:
                    continue
                if k == 1:
                    self.Bc[(i, j)] = self.Z[i].T @ h2.near_blocks[(i, j)] @ self.Z[j]
                else:
                    # eq. Mijk with Z-bar = F^{-T} V-bar
                    self.Bc[(i, j)] = self.Z[i].T @ self.bold_B(i, j) @ self.Z[j]
            for j in T.coup[i]:
                self.Bc[(i, j)] = self.PhiU[i] @ h2.B[(i, j)] @ self.PhiU[j].T

    # -- Algorithm 5.3, leaf level ---------------------------------------------
    def _leaf_level(self):
        T, h2 = self.tree, self.h2
        for i in T.leaves():
            S = chol(h2.near_blocks[(i, i)])
            self.S[i] = S
            Psi = lsolve(S, self.Y[1][T.rng(i)])          # Lambda_{ii^c} Omega_{i^c}
            V = self._compress(i, Psi)
            self.V[i] = V
            self.Z[i] = ltsolve(S, V)                      # Phi_i = Z_i^T = V_i^T S_i^{-1}
            self.PhiU[i] = self.Z[i].T @ h2.W[i]
        self._couplings(1)

    # -- Algorithm 5.2: T-blocks of Y^(k) up to level k-1 ------------------------
    def special_products(self, k: int) -> dict[int, np.ndarray]:
        T = self.tree
        Tb = {}
        for i in T.leaves():
            Tb[i] = self.V[i].T @ lsolve(self.S[i], self.Y[k][T.rng(i)])
        for l in range(2, k):
            for i in T.nodes_at(l):
                c1, c2 = T.children(i)
                Tb[i] = self.Vbar[i].T @ self._finv(i, np.vstack([Tb[c1], Tb[c2]]))
        return Tb

    # -- Algorithm 5.3, levels 2..L-1 --------------------------------------------
    def _level(self, k: int):
        T, h2 = self.tree, self.h2
        nodes = T.nodes_at(k)
        for i in nodes:
            self._factor(i, np.eye(self.rank[T.children(i)[0]] + self.rank[T.children(i)[1]])
                         + self.bold_B(i, i))
        Tb = self.special_products(k)
        for i in nodes:
            c1, c2 = T.children(i)
            Psi = self._finv(i, np.vstack([Tb[c1], Tb[c2]]))
            Vb = self._compress(i, Psi)
            self.Vbar[i] = Vb
            self.Z[i] = self._finvT(i, Vb)                 # Phi_i = Z_i^T diag(Phi_c)
            r1, r2 = self.rank[c1], self.rank[c2]
            k1, k2 = h2.rank(c1), h2.rank(c2)
            D = np.zeros((r1 + r2, k1 + k2))
            D[:r1, :k1] = self.PhiU[c1]
            D[r1:, k1:] = self.PhiU[c2]
            self.PhiU[i] = self.Z[i].T @ D @ h2.W[i]
            self.R[i] = self.F[i] @ Vb
        self._couplings(k)

    def _root(self):
        T = self.tree
        c1, c2 = T.children(0)
        self._factor(0, np.eye(self.rank[c1] + self.rank[c2]) + self.bold_B(0, 0))

    # -- dense forms for checks ----------------------------------------------------
    def U_full(self, v: int) -> np.ndarray:
        """Expanded HSS basis U_v = S_v V_v (|I_v| x r_v), nested by eq. nested."""
        T = self.tree
        if T.is_leaf(v):
            return self.S[v] @ self.V[v]
        c1, c2 = T.children(v)
        U1, U2 = self.U_full(c1), self.U_full(c2)
        Z = np.zeros((U1.shape[0] + U2.shape[0], U1.shape[1] + U2.shape[1]))
        Z[:U1.shape[0], :U1.shape[1]] = U1
        Z[U1.shape[0]:, U1.shape[1]:] = U2
        return Z @ self.R[v]

    def Phi_full(self, v: int) -> np.ndarray:
        """Dense Phi_v (r_v x |I_v|) by eq. phi."""
        T = self.tree
        if T.is_leaf(v):
            return self.Z[v].T
        c1, c2 = T.children(v)
        P1, P2 = self.Phi_full(c1), self.Phi_full(c2)
        Dg = np.zeros((P1.shape[0] + P2.shape[0], P1.shape[1] + P2.shape[1]))
        Dg[:P1.shape[0], :P1.shape[1]] = P1
        Dg[P1.shape[0]:, P1.shape[1]:] = P2
        return self.Z[v].T @ Dg

    def dense(self) -> np.ndarray:
        """The HSS approximation A^(L-1) assembled from its generators
        {A_ii, U_i, R_i, sibling B_ij} (tree order)."""
        T, h2 = self.tree, self.h2
        A = np.zeros((T.N, T.N))
        for i in T.leaves():
            A[T.rng(i), T.rng(i)] = h2.near_blocks[(i, i)]
        for k in range(1, T.L):
            for p in T.nodes_at(k + 1):
                c1, c2 = T.children(p)
                U1, U2 = self.U_full(c1), self.U_full(c2)
                blk = U1 @ self.Bc[(c1, c2)] @ U2.T
                A[T.rng(c1), T.rng(c2)] = blk
                A[T.rng(c2), T.rng(c1)] = blk.T
        return A

    # -- ULV-style solve with the nested factors ----------------------------------
    def solve(self, b: np.ndarray) -> np.ndarray:
        """x = A_hss^{-1} b (tree order) through the nested symmetric factors.

        At the leaf level A_hss = S (I + V M V^T) S^T with S = diag(S_i) and
        orthonormal V = diag(V_i) (eq. Aii0 applied to the whole matrix), so
        A_hss^{-1} = S^{-T} (I + V((I + M)^{-1} - I) V^T) S^{-1}; I + M has the
        same form one level up with F_i in place of S_i (eq. Si0/Si), down to
        I + bold B_root at the root.  Unfolding gives an upward sweep, a root
        solve and a downward sweep.
        """
        T = self.tree
        b = np.asarray(b, dtype=np.float64)
        vec = b.ndim == 1
        if vec:
            b = b[:, None]
        if T.L == 1:
            x = ltsolve(self.S[0], lsolve(self.S[0], b))
            return x[:, 0] if vec else x
        z, t, u = {}, {}, {}
        for i in T.leaves():
            z[i] = lsolve(self.S[i], b[T.rng(i)])
            t[i] = self.V[i].T @ z[i]
        for k in range(2, T.L):
            for i in T.nodes_at(k):
                c1, c2 = T.children(i)
                u[i] = self._finv(i, np.vstack([t[c1], t[c2]]))
                t[i] = self.Vbar[i].T @ u[i]
        w = {}
        c1, c2 = T.children(0)
        wr = self._finvT(0, self._finv(0, np.vstack([t[c1], t[c2]])))
        w[c1], w[c2] = wr[:self.rank[c1]], wr[self.rank[c1]:]
        for k in range(T.L - 1, 1, -1):
            for i in T.nodes_at(k):
                c1, c2 = T.children(i)
                ui = u[i] + self.Vbar[i] @ (w[i] - t[i])
                wc = self._finvT(i, ui)
                w[c1], w[c2] = wc[:self.rank[c1]], wc[self.rank[c1]:]
        x = np.zeros_like(b)
        for i in T.leaves():
            zi = z[i] + self.V[i] @ (w[i] - t[i])
            x[T.rng(i)] = ltsolve(self.S[i], zi)
        return x[:, 0] if vec else x

    def ranks_at(self, k: int) -> list[int]:
        return [self.rank[v] for v in self.tree.nodes_at(k)]
