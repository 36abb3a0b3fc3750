"""H^2 representation of sigma*I + K(X, X) (oracle; test infrastructure only).

Section 5.1 (eq. uniformbasis_h2): on every level, the blocks A_ij with j in
the far field of i are represented as U_i B_ij U_j^T with nested bases
U_i = diag(U_children) R_i (eq. nested); only Type-3 blocks (far, with
inadmissible parents) are stored, plus the dense near blocks of the leaf
level.

The paper builds this with H2Pack's proxy-point method and does not describe
it.  The construction here is this project's reading (an interpolative
decomposition against proxy points, bottom-up):

* candidates of a node: its points (leaf) or its children's skeletons,
  concatenated in child order (nonleaf);
* proxy points: Q spheres of P_v points each (Fibonacci lattice), centred at
  the node's box centre, at radii geometrically spaced from rho_in to rho_out,
  where rho_in is the smallest distance from the centre to a box of the node's
  far field (couplings of the node and all its ancestors) and rho_out the
  largest distance from the centre to a corner of the root box;
* the number of points per sphere resolves the kernel's length scale on the
  innermost sphere: P_v = density * (rho_in / ell)^2, rounded up to a multiple
  of 64 and clamped to [per_shell, per_shell_max] (density = 0 keeps
  P_v = per_shell).  A fixed count under-resolves the large boxes of the upper
  levels, whose far field then misses the tolerance by orders of magnitude;
* G = K(X_cand, proxies) (c x M).  When M exceeds l = max(2c, c + 16) it is
  first sketched, S = G Omega with an M x l standard normal Omega from the
  counter-based generator of oracle/rng.py (a randomized interpolative
  decomposition: Liberty, Woolfe, Martinsson, Rokhlin and Tygert, PNAS 2007;
  Halko, Martinsson and Tropp, SIAM Review 2011, Section 5.2); otherwise
  S = G.  A column-pivoted QR of S^T with relative truncation
  |R_tt| > eps * |R_00| selects the skeleton; E = R11^{-1} R12;
* the interpolation matrix W has identity rows at the skeleton and E^T rows
  elsewhere: U_i = W at a leaf, R_i = W at a nonleaf;
* B_ij = K(X_skel_i, X_skel_j) for coupling pairs;
* a node with no far field keeps no skeleton (rank 0).

The accuracy of this construction against the dense matrix is measured in the
tests; it is not a result fixed by the paper.
"""
from __future__ import annotations

import math
import numpy as np

from . import kernels, rng
from .linalg import CPQR
from .tree import Tree


def fibonacci_sphere(npts: int) -> np.ndarray:
    """npts points of the Fibonacci lattice on the unit sphere."""
    t = np.arange(npts, dtype=np.float64)
    z = 1.0 - (2.0 * t + 1.0) / npts
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = t * (math.pi * (3.0 - math.sqrt(5.0)))
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def proxy_count(rin: float, ell: float, per_shell: int, per_shell_max: int,
                density: float) -> int:
    """Points per proxy sphere of a node whose innermost sphere has radius rin."""
    if density <= 0.0:
        return int(per_shell)
    t = rin / ell
    n = 64 * int(math.ceil(density * (t * t) / 64.0))
    return int(min(max(n, per_shell), per_shell_max))


def sketch_rows(c: int) -> int:
    """Rows of the sketch of a proxy matrix with c candidate columns."""
    return max(2 * c, c + 16)


def box_distance(c: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> float:
    """Distance from point c to the axis-aligned box [lo, hi]."""
    d = np.maximum(np.maximum(lo - c, 0.0), c - hi)
    return float(math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]))


SKETCH_SEED = 0x5EEDF00D


class H2:
    def __init__(self, X, kind, ell, shift, leaf, tol, eta=1.0,
                 shells=8, per_shell=128, per_shell_max=2048, density=90.0,
                 sketch_seed=SKETCH_SEED, tree: Tree | None = None, tree_kind: str = "kd"):
        X = np.ascontiguousarray(X, dtype=np.float64)
        # a tensor kernel acts on 3 rows per point: row 3p + c is point p's
        # component c, and the tree partitions the rows (3 coincident entries a point)
        self.comp = np.tile(np.arange(3), X.shape[0]) if kind in kernels.TENSOR else None
        self.X = np.repeat(X, 3, axis=0) if self.comp is not None else X
        self.kind, self.ell, self.shift, self.tol = kind, float(ell), float(shift), float(tol)
        self.shells, self.per_shell = int(shells), int(per_shell)
        self.per_shell_max, self.density = max(int(per_shell_max), int(per_shell)), float(density)
        self.sketch_seed = int(sketch_seed)
        self.proxy_n: dict[int, int] = {}   # points per sphere of each node
        self.sketched: dict[int, bool] = {}
        self.tree = tree if tree is not None else Tree(self.X, leaf, eta, tree_kind)
        T = self.tree
        self.skel: dict[int, np.ndarray] = {}
        self.W: dict[int, np.ndarray] = {}   # U_i (leaf) or R_i (nonleaf)
        self._build_bases()
        self.B = {}
        for v in range(T.nnodes):
            for j in T.coup[v]:
                self.B[(v, j)] = self.K(self.skel[v], self.skel[j])
        self.near_blocks = {}
        for i in T.leaves():
            for j in T.near[i]:
                blk = self.K(T.perm[T.rng(i)], T.perm[T.rng(j)])
                if i == j:
                    blk = blk + self.shift * np.eye(blk.shape[0])
                self.near_blocks[(i, j)] = blk

    def K(self, ia, ib) -> np.ndarray:
        if self.comp is not None:
            return kernels.evaluate(self.kind, self.ell, self.X[ia], self.X[ib], self.comp[ia], self.comp[ib])
        return kernels.evaluate(self.kind, self.ell, self.X[ia], self.X[ib])

    # -- construction --------------------------------------------------------
    def proxies(self, v: int) -> np.ndarray | None:
        T = self.tree
        far = T.far_nodes(v)
        if not far:
            return None
        c = T.center[v]
        rin = min(box_distance(c, T.lo[j], T.hi[j]) for j in far)
        corners = np.array([[a, b, d] for a in (T.lo[0][0], T.hi[0][0])
                            for b in (T.lo[0][1], T.hi[0][1])
                            for d in (T.lo[0][2], T.hi[0][2])])
        dc = corners - c
        rout = float(np.sqrt(dc[:, 0] * dc[:, 0] + dc[:, 1] * dc[:, 1] + dc[:, 2] * dc[:, 2]).max())
        rout = max(rout, rin)
        Q = self.shells
        # a tensor kernel's ell is the particle radius, not a length scale of
        # its far field (which decays like 1/r): the per-sphere count is fixed
        # at twice per_shell (each proxy point then gives 3 columns)
        if self.comp is not None:
            P = min(2 * self.per_shell, self.per_shell_max)
        else:
            P = proxy_count(rin, self.ell, self.per_shell, self.per_shell_max, self.density)
        self.proxy_n[v] = P
        unit = fibonacci_sphere(P)
        pts = []
        for q in range(Q):
            rad = rin if Q == 1 else rin * (rout / rin) ** (q / (Q - 1))
            pts.append(c + rad * unit)
        return np.concatenate(pts, axis=0)

    def candidates(self, v: int) -> np.ndarray:
        T = self.tree
        if T.is_leaf(v):
            return T.perm[T.rng(v)]
        c1, c2 = T.children(v)
        return np.concatenate([self.skel[c1], self.skel[c2]])

    def _build_bases(self):
        T = self.tree
        for k in range(1, T.L):
            for v in T.nodes_at(k):
                cand = self.candidates(v)
                P = self.proxies(v)
                if P is None or len(cand) == 0:
                    self.skel[v] = cand[:0]
                    self.W[v] = np.zeros((len(cand), 0))
                    continue
                if self.comp is not None:
                    # every proxy point carries the 3 components: column 3q + c
                    G = kernels.evaluate(self.kind, self.ell, self.X[cand], np.repeat(P, 3, axis=0),
                                         self.comp[cand], np.tile(np.arange(3), len(P)))
                else:
                    G = kernels.evaluate(self.kind, self.ell, self.X[cand], P)
                c, M = G.shape
                l = sketch_rows(c)
                self.sketched[v] = M > l
                S = G @ rng.sketch(M, l, self.sketch_seed) if M > l else G
                f = CPQR(S.T, self.tol, min(S.shape))
                r = f.rank
                E = f.interp()
                W = np.zeros((len(cand), r))
                W[f.perm[:r], np.arange(r)] = 1.0
                W[f.perm[r:], :] = E.T
                self.skel[v] = cand[f.piv]
                self.W[v] = W
        self.skel[0] = np.zeros(0, dtype=np.int64)
        self.W[0] = np.zeros((sum(len(self.skel[c]) for c in T.children(0)) if T.L > 1 else T.N, 0))

    def rank(self, v: int) -> int:
        return len(self.skel[v])

    # -- products ------------------------------------------------------------
    def matvec(self, x: np.ndarray, above: int = 0) -> np.ndarray:
        """y = A x in tree order.  With above = k > 0 only blocks whose lowest
        common ancestor level exceeds k are applied, i.e. the product with
        A - diag({A_ii}, i in lvl(k)) of eq. (Yk)."""
        T = self.tree
        x = np.asarray(x, dtype=np.float64)
        if x.ndim == 1:
            return self.matvec(x[:, None], above)[:, 0]
        m = x.shape[1]
        y = np.zeros_like(x)
        if T.L == 1:
            if above < 1:
                y += self.near_blocks[(0, 0)] @ x
            return y
        xh = {}
        for k in range(1, T.L):
            for v in T.nodes_at(k):
                if T.is_leaf(v):
                    xh[v] = self.W[v].T @ x[T.rng(v)]
                else:
                    c1, c2 = T.children(v)
                    xh[v] = self.W[v].T @ np.vstack([xh[c1], xh[c2]])
        yh = {v: np.zeros((self.rank(v), m)) for v in range(1, T.nnodes)}
        for v in range(1, T.nnodes):
            for j in T.coup[v]:
                if T.lca_level(v, j) > above:
                    yh[v] += self.B[(v, j)] @ xh[j]
        for k in range(T.L - 1, 1, -1):
            for v in T.nodes_at(k):
                c1, c2 = T.children(v)
                t = self.W[v] @ yh[v]
                k1 = self.rank(c1)
                yh[c1] += t[:k1]
                yh[c2] += t[k1:]
        for v in T.leaves():
            y[T.rng(v)] += self.W[v] @ yh[v]
            for j in T.near[v]:
                if T.lca_level(v, j) > above:
                    y[T.rng(v)] += self.near_blocks[(v, j)] @ x[T.rng(j)]
        return y

    # -- dense forms for checks ---------------------------------------------
    def full_basis(self, v: int) -> np.ndarray:
        """Expanded nested basis of node v (|I_v| x k_v)."""
        T = self.tree
        if T.is_leaf(v):
            return self.W[v]
        c1, c2 = T.children(v)
        U1, U2 = self.full_basis(c1), self.full_basis(c2)
        Z = np.zeros((U1.shape[0] + U2.shape[0], U1.shape[1] + U2.shape[1]))
        Z[:U1.shape[0], :U1.shape[1]] = U1
        Z[U1.shape[0]:, U1.shape[1]:] = U2
        return Z @ self.W[v]

    def dense(self) -> np.ndarray:
        """The H^2 matrix assembled block by block (tree order)."""
        T = self.tree
        A = np.zeros((T.N, T.N))
        for (i, j), blk in self.near_blocks.items():
            A[T.rng(i), T.rng(j)] = blk
        Ufull = {}
        for (i, j), Bij in self.B.items():
            for v in (i, j):
                if v not in Ufull:
                    Ufull[v] = self.full_basis(v)
            A[T.rng(i), T.rng(j)] = Ufull[i] @ Bij @ Ufull[j].T
        return A

    def exact_dense(self) -> np.ndarray:
        """sigma*I + K(X, X) in tree order."""
        p = self.tree.perm
        return self.K(p, p) + self.shift * np.eye(len(p))
