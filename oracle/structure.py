"""Cluster tree and block tree (Section 2: the H-matrix is a recursive
partition of the matrix into sub-blocks, most of them low-rank, a minor
number dense). The paper skips the partitioning rules; this module fixes the
readings used throughout:

Cluster tree
  * A node owns a contiguous range [lo, hi) of the permuted point order and
    the axis-aligned bounding box of those points.
  * A node with m = hi - lo > leaf_size is split: axis = the longest bounding
    box side (ties: lowest axis); its points are ordered by (coordinate on
    that axis, original index) and the first floor(m/2) go to the first
    child, the rest to the second. A node with m <= leaf_size is a leaf and
    keeps the order it inherited.
  * Nodes are numbered level by level (breadth first), children of a node
    consecutively, first child first.

Admissibility (eta > 0)
  * diam(t)^2 = sum_k (bmax_k - bmin_k)^2,
    dist(t,s)^2 = sum_k max(0, bmin_s,k - bmax_t,k, bmin_t,k - bmax_s,k)^2,
    the pair is admissible iff min(diam(t)^2, diam(s)^2) <= eta^2 dist(t,s)^2.
    A diagonal pair (t == s) is never admissible. Sums run over axes in
    increasing order, each term a product followed by an addition (no fused
    multiply-add), so that any implementation that follows the same order
    reaches the same decisions bit for bit.

Block tree (lower triangle only)
  * (t, t): a leaf t gives a dense diagonal block; otherwise recurse into
    (t1, t1), (t2, t1), (t2, t2).
  * (t, s), t after s: admissible -> low-rank block; else if t or s is a leaf
    -> dense block; else recurse into the four child pairs.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class ClusterTree:
    perm: np.ndarray      # int64[n]; perm[k] = original index of the k-th permuted point
    lo: np.ndarray        # int64[nn]
    hi: np.ndarray        # int64[nn]
    bmin: np.ndarray      # float64[nn, d]
    bmax: np.ndarray      # float64[nn, d]
    child: np.ndarray     # int64[nn, 2]; -1 for leaves
    level: np.ndarray     # int64[nn]

    @property
    def n_nodes(self) -> int:
        return int(self.lo.shape[0])

    def is_leaf(self, t: int) -> bool:
        return self.child[t, 0] < 0


def cluster_tree(pts, leaf_size: int) -> ClusterTree:
    pts = np.asarray(pts, dtype=np.float64)
    n, d = pts.shape
    perm = np.arange(n, dtype=np.int64)
    lo, hi, bmin, bmax, child, level = [], [], [], [], [], []

    frontier = [(0, n)]
    lev = 0
    while frontier:
        nxt = []
        base = len(lo) + len(frontier)   # id of the first node of the next level
        for (a, b) in frontier:
            p = pts[perm[a:b]]
            mn = p.min(axis=0)
            mx = p.max(axis=0)
            lo.append(a); hi.append(b); bmin.append(mn); bmax.append(mx); level.append(lev)
            m = b - a
            if m > leaf_size:
                ext = mx - mn
                axis = int(np.argmax(ext))   # first maximum -> lowest axis on ties
                idx = perm[a:b]
                order = np.lexsort((idx, pts[idx, axis]))   # primary: coordinate, then index
                perm[a:b] = idx[order]
                half = m // 2
                child.append([base + len(nxt), base + len(nxt) + 1])
                nxt.append((a, a + half))
                nxt.append((a + half, b))
            else:
                child.append([-1, -1])
        frontier = nxt
        lev += 1
    return ClusterTree(perm=perm, lo=np.array(lo, dtype=np.int64), hi=np.array(hi, dtype=np.int64),
                       bmin=np.array(bmin).reshape(-1, d), bmax=np.array(bmax).reshape(-1, d),
                       child=np.array(child, dtype=np.int64).reshape(-1, 2),
                       level=np.array(level, dtype=np.int64))


def _diam2(tree: ClusterTree, t: int) -> float:
    acc = 0.0
    for k in range(tree.bmin.shape[1]):
        e = float(tree.bmax[t, k]) - float(tree.bmin[t, k])
        acc = acc + e * e
    return acc


def _dist2(tree: ClusterTree, t: int, s: int) -> float:
    acc = 0.0
    for k in range(tree.bmin.shape[1]):
        g = max(0.0, float(tree.bmin[s, k]) - float(tree.bmax[t, k]),
                float(tree.bmin[t, k]) - float(tree.bmax[s, k]))
        acc = acc + g * g
    return acc


def admissible(tree: ClusterTree, t: int, s: int, eta: float) -> bool:
    if t == s:
        return False
    return min(_diam2(tree, t), _diam2(tree, s)) <= (eta * eta) * _dist2(tree, t, s)


@dataclass
class BlockTree:
    dense: np.ndarray     # int64[nd, 2] (row cluster, column cluster), sorted by (col lo, row lo)
    lowrank: np.ndarray   # int64[nl, 2]


def block_tree(tree: ClusterTree, eta: float) -> BlockTree:
    dense, lowrank = [], []
    stack = [(0, 0)]
    while stack:
        t, s = stack.pop()
        if t == s:
            if tree.is_leaf(t):
                dense.append((t, t))
            else:
                c1, c2 = tree.child[t]
                stack += [(int(c1), int(c1)), (int(c2), int(c1)), (int(c2), int(c2))]
        elif admissible(tree, t, s, eta):
            lowrank.append((t, s))
        elif tree.is_leaf(t) or tree.is_leaf(s):
            dense.append((t, s))
        else:
            for a in tree.child[t]:
                for b in tree.child[s]:
                    stack.append((int(a), int(b)))

    def canon(lst):
        if not lst:
            return np.zeros((0, 2), dtype=np.int64)
        arr = np.array(lst, dtype=np.int64)
        order = np.lexsort((tree.lo[arr[:, 0]], tree.lo[arr[:, 1]]))
        return arr[order]

    return BlockTree(dense=canon(dense), lowrank=canon(lowrank))


def covered_entries(tree: ClusterTree, bt: BlockTree) -> int:
    """Number of matrix entries the blocks cover, counting off-diagonal blocks
    twice (they stand for their transpose too)."""
    tot = 0
    for arr in (bt.dense, bt.lowrank):
        for t, s in arr:
            sz = int(tree.hi[t] - tree.lo[t]) * int(tree.hi[s] - tree.lo[s])
            tot += sz if t == s else 2 * sz
    return tot
