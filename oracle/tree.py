"""Partition tree and admissibility lists (oracle; test infrastructure only).

Section 2 (notation): a perfect partition tree with levels numbered from the
leaves (level 1) to the root (level L); lvl(k) is the node set of level k.
Section 5.1 defines the far field F_i of a node as the same-level nodes whose
points are well separated from those of i; Section 5.2.2 classes blocks as
Type-1 (j not in F_i), Type-2 (inside a larger far block) and Type-3 (far, with
inadmissible parents).

Two partition rules ("kind"):

* "kd" (the binary kd-tree of the workloads; the paper is silent on it):
  depth D = smallest integer with N <= leaf * 2^D; a node is split on the
  axis of largest tight-bounding-box extent (lowest axis on ties), its points
  ordered by (coordinate, original index), and the left child takes the first
  floor(n/2) of them;
* "box" (Section 6: the 2^d-ary tree that bisects every dimension of a box
  enclosing the points until the finest boxes are small enough), realised as
  a perfect binary tree with d = 3 binary levels per 2^d-ary level: a node at
  depth t is bisected along axis t mod 3 at the midpoint of its points' tight
  extent on that axis, points below the midpoint going left (ordered by
  (coordinate, original index) as above), and D is the smallest multiple of 3
  for which no node at depth D holds more than leaf points.  Readings: the
  box of a node is the tight box of its points (so that no box is empty and
  the tree stays perfect); the axes are taken in the order x, y, z; "small
  enough" is at most leaf points.  A node that cannot be bisected (no extent
  along the axis) is an error.

Shared by both:

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


def box_split(P: np.ndarray, axis: int) -> int:
    """Points of a node bisected at the midpoint of their extent along axis:
    the number below it (P already ordered along the axis)."""
    lo, hi = P[:, axis].min(), P[:, axis].max()
    mid = 0.5 * (lo + hi)
    m = int(np.count_nonzero(P[:, axis] < mid))
    if m == 0 or m == P.shape[0]:
        raise ValueError(f"box bisection: a node of {P.shape[0]} points has no extent along axis {axis}")
    return m


class Tree:
    def __init__(self, X: np.ndarray, leaf: int, eta: float = 1.0, kind: str = "kd"):
        X = np.asarray(X, dtype=np.float64)
        N = X.shape[0]
        if N < 1:
            raise ValueError("empty point set")
        if kind not in ("kd", "box"):
            raise ValueError(f"unknown tree kind {kind!r}")
        self.N, self.leaf, self.eta, self.kind = N, int(leaf), float(eta), kind
        perm = np.arange(N)
        start, end = [0], [N]

        def split(v: int, axis):
            s, e = start[v], end[v]
            idx = perm[s:e]
            P = X[idx]
            if axis is None:
                ext = P.max(axis=0) - P.min(axis=0)
                axis = int(np.argmax(ext))  # first maximum -> lowest axis on ties
            order = np.lexsort((idx, P[:, axis]))  # primary: coordinate, then index
            perm[s:e] = idx[order]
            m = (e - s) // 2 if kind == "kd" else box_split(P[order], axis)
            start.extend([s, s + m])
            end.extend([s + m, e])

        if kind == "kd":
            self.D = depth_for(N, leaf)
            for v in range((1 << self.D) - 1):  # every internal node, top-down
                split(v, None)
        else:
            self.D = 0
            while max(end[v] - start[v] for v in range((1 << self.D) - 1, (1 << (self.D + 1)) - 1)) > leaf:
                if self.D + 3 > 24:
                    raise ValueError("tree too deep")
                for t in range(self.D, self.D + 3):  # bisect x, then y, then z
                    for v in range((1 << t) - 1, (1 << (t + 1)) - 1):
                        split(v, t % 3)
                self.D += 3
        self.L = self.D + 1
        nn = (1 << (self.D + 1)) - 1
        self.nnodes = nn
        start = np.asarray(start, dtype=np.int64)
        end = np.asarray(end, dtype=np.int64)
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
