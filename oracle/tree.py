"""Partition tree and admissibility lists (oracle; test infrastructure only).

Section 2 (notation): a perfect partition tree with levels numbered from the
leaves (level 1) to the root (level L); lvl(k) is the node set of level k.
Section 5.1 defines the far field F_i of a node as the same-level nodes whose
points are well separated from those of i; Section 5.2.2 classes blocks as
Type-1 (j not in F_i), Type-2 (inside a larger far block) and Type-3 (far, with
inadmissible parents).

Readings taken where the paper is silent (Section 6 uses a 2^d-ary box
bisection; the workloads ask for a binary kd-tree):

* depth D = smallest integer with N <= leaf * 2^D; L = D + 1 levels;
* a node is split on the axis of largest tight-bounding-box extent (lowest
  axis on ties), its points ordered by (coordinate, original index), and the
  left child takes the first floor(n/2) of them;
* admissible(i, j)  <=>  i != j and r_i + r_j <= eta * |c_i - c_j|, with c the
  bounding-box centre and r its half diagonal;
* near/coupling lists are built top-down: the children of every near node of
  par(i) are tested against i; admissible ones are Type-3 (coupling), the
  rest Type-1 (near).  Lists are sorted by node id.

Nodes are stored in heap order: the root is 0, children of v are 2v+1, 2v+2.
"""
from __future__ import annotations

import math
import numpy as np


def depth_for(n: int, leaf: int) -> int:
    d = 0
    while n > leaf * (1 << d):
        d += 1
    return d


class Tree:
    def __init__(self, X: np.ndarray, leaf: int, eta: float = 1.0):
        X = np.asarray(X, dtype=np.float64)
        N = X.shape[0]
        if N < 1:
            raise ValueError("empty point set")
        self.N, self.leaf, self.eta = N, int(leaf), float(eta)
        self.D = depth_for(N, leaf)
        self.L = self.D + 1
        nn = (1 << (self.D + 1)) - 1
        self.nnodes = nn
        perm = np.arange(N)
        start = np.zeros(nn, dtype=np.int64)
        end = np.zeros(nn, dtype=np.int64)
        start[0], end[0] = 0, N
        for v in range((1 << self.D) - 1):  # every internal node, top-down
            s, e = start[v], end[v]
            idx = perm[s:e]
            P = X[idx]
            ext = P.max(axis=0) - P.min(axis=0)
            axis = int(np.argmax(ext))  # first maximum -> lowest axis on ties
            order = np.lexsort((idx, P[:, axis]))  # primary: coordinate, then index
            perm[s:e] = idx[order]
            half = (e - s) // 2
            start[2 * v + 1], end[2 * v + 1] = s, s + half
            start[2 * v + 2], end[2 * v + 2] = s + half, e
        self.perm = perm                  # tree position -> original index
        self.iperm = np.empty(N, dtype=np.int64)
        self.iperm[perm] = np.arange(N)   # original index -> tree position
        self.start, self.end = start, end
        lo = np.zeros((nn, 3))
        hi = np.zeros((nn, 3))
        for v in range(nn):
            P = X[perm[start[v]:end[v]]]
            if len(P):
                lo[v], hi[v] = P.min(axis=0), P.max(axis=0)
        self.lo, self.hi = lo, hi
        d = hi - lo
        self.center = 0.5 * (lo + hi)
        self.radius = 0.5 * np.sqrt(d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2])
        self._build_lists()

    # -- structure ---------------------------------------------------------
    def depth(self, v: int) -> int:
        return int(math.floor(math.log2(v + 1)))

    def level(self, v: int) -> int:
        return self.L - self.depth(v)

    def nodes_at(self, k: int) -> list[int]:
        d = self.L - k
        return list(range((1 << d) - 1, (1 << (d + 1)) - 1))

    def parent(self, v: int) -> int:
        return (v - 1) // 2

    def children(self, v: int) -> tuple[int, int]:
        return 2 * v + 1, 2 * v + 2

    def is_leaf(self, v: int) -> bool:
        return self.depth(v) == self.D

    def leaves(self) -> list[int]:
        return self.nodes_at(1)

    def rng(self, v: int) -> slice:
        return slice(int(self.start[v]), int(self.end[v]))

    def size(self, v: int) -> int:
        return int(self.end[v] - self.start[v])

    def lca_level(self, i: int, j: int) -> int:
        """Level of the lowest common ancestor of two same-level nodes."""
        k = self.level(i)
        while i != j:
            i, j = self.parent(i), self.parent(j)
            k += 1
        return k

    # -- admissibility and lists -------------------------------------------
    def admissible(self, i: int, j: int) -> bool:
        if i == j:
            return False
        dc = self.center[i] - self.center[j]
        dist = math.sqrt(dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2])
        return bool(self.radius[i] + self.radius[j] <= self.eta * dist)

    def _build_lists(self):
        near = {0: [0]}
        coup = {0: []}
        for d in range(1, self.D + 1):
            for v in range((1 << d) - 1, (1 << (d + 1)) - 1):
                p = self.parent(v)
                nv, cv = [], []
                for q in near[p]:
                    for j in self.children(q):
                        (cv if self.admissible(v, j) else nv).append(j)
                near[v], coup[v] = sorted(nv), sorted(cv)
        self.near, self.coup = near, coup

    def far_nodes(self, v: int) -> list[int]:
        """All nodes whose points lie in the far field of v: couplings of v and
        of every ancestor of v."""
        out = []
        a = v
        while True:
            out.extend(self.coup[a])
            if a == 0:
                break
            a = self.parent(a)
        return out
