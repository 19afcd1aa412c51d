"""FP64 oracle -- cluster trees and block trees (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use anything under ``oracle/``.  The oracle shares no code
with the HIP path.

Follows Section 2 of the paper:
  * Definition 1 (cluster tree): a labelled tree whose children partition
    their parent's index set.
  * The admissibility condition (eq. admissibility):
        max(diam Omega_t, diam Omega_s) <= 2 * eta * dist(Omega_t, Omega_s).
  * Definition 2 (block tree) with the children rule (eq. block_children) and
    the recursive construction described after it: a block is kept as an
    admissible leaf if admissible, split if one of its clusters has children,
    kept as an inadmissible leaf otherwise.

Readings where the paper leaves the construction open ("a suitable algorithm"):
  * Omega_t is the axis-aligned bounding box of the cluster's points; diam is
    its diagonal, dist the Euclidean box-to-box distance (0 if they touch).
  * Geometric bisection: split along the longest box edge (lowest axis on
    ties) at the box midpoint; coordinate < midpoint goes to the first child,
    the rest to the second, both in their previous order.  If one side would
    be empty, the cluster is halved by a stable sort along that axis.  A
    cluster is a leaf iff it holds at most ``leaf_size`` indices.
"""
from __future__ import annotations

import math

import numpy as np


class ClusterTree:
    """Clusters are numbered in depth-first pre-order; each cluster owns the
    contiguous range [begin, end) of the permuted index order ``perm``
    (``perm[k]`` = original index of permuted position k)."""

    def __init__(self, points: np.ndarray, leaf_size: int):
        pts = np.asarray(points, dtype=np.float64)
        if pts.ndim != 2:
            raise ValueError("points must be n x dim")
        self.points = pts
        self.n, self.dim = pts.shape
        self.leaf_size = int(leaf_size)
        self.begin, self.end, self.parent, self.level = [], [], [], []
        self.children = []
        self.lo, self.hi = [], []
        perm = np.arange(self.n, dtype=np.int64)
        self._build(perm, 0, self.n, -1, 0)
        self.perm = perm
        self.begin = np.array(self.begin, dtype=np.int64)
        self.end = np.array(self.end, dtype=np.int64)
        self.parent = np.array(self.parent, dtype=np.int64)
        self.level = np.array(self.level, dtype=np.int64)
        self.lo = np.array(self.lo)
        self.hi = np.array(self.hi)
        self.ncl = len(self.begin)
        self.depth = int(self.level.max()) + 1

    def _build(self, perm, b, e, parent, lev):
        c = len(self.begin)
        idx = perm[b:e]
        P = self.points[idx]
        lo, hi = P.min(axis=0), P.max(axis=0)
        self.begin.append(b)
        self.end.append(e)
        self.parent.append(parent)
        self.level.append(lev)
        self.children.append([])
        self.lo.append(lo)
        self.hi.append(hi)
        if e - b <= self.leaf_size:
            return c
        ext = hi - lo
        ax = int(np.argmax(ext))  # first maximal axis
        mid = 0.5 * (lo[ax] + hi[ax])
        left = P[:, ax] < mid
        nl = int(left.sum())
        if nl == 0 or nl == e - b:
            order = np.argsort(P[:, ax], kind="stable")
            nl = (e - b) // 2
            newidx = idx[order]
        else:
            newidx = np.concatenate([idx[left], idx[~left]])
        perm[b:e] = newidx
        c0 = self._build(perm, b, b + nl, c, lev + 1)
        c1 = self._build(perm, b + nl, e, c, lev + 1)
        self.children[c] = [c0, c1]
        return c

    def size(self, t):
        return int(self.end[t] - self.begin[t])

    def is_leaf(self, t):
        return len(self.children[t]) == 0

    # Squared diameter and distance as plain sums of products in axis order
    # (Python floats: no fused multiply-add), the arithmetic the library's
    # host planner uses too, so exact ties of the admissibility condition on
    # regular point sets are decided alike.
    def diam2(self, t):
        acc = 0.0
        for d in self.hi[t] - self.lo[t]:
            acc += float(d) * float(d)
        return acc

    def dist2(self, t, s):
        gap = np.maximum(0.0, np.maximum(self.lo[t] - self.hi[s], self.lo[s] - self.hi[t]))
        acc = 0.0
        for g in gap:
            acc += float(g) * float(g)
        return acc

    def diam(self, t):
        return math.sqrt(self.diam2(t))

    def dist(self, t, s):
        return math.sqrt(self.dist2(t, s))

    def leaves(self):
        return [t for t in range(self.ncl) if self.is_leaf(t)]

    def chil_plus(self, t):
        """chil(t) if t has children, else {t} (children rule for blocks whose
        other cluster still has children)."""
        return self.children[t] if self.children[t] else [t]

    def ancestors_or_self(self, t):
        out = []
        while t >= 0:
            out.append(t)
            t = int(self.parent[t])
        return out


def dist2_between(tree_r: ClusterTree, t: int, tree_c: ClusterTree, s: int) -> float:
    """Squared distance of the boxes of cluster t of tree_r and cluster s of
    tree_c (the same arithmetic as ClusterTree.dist2)."""
    gap = np.maximum(0.0, np.maximum(tree_r.lo[t] - tree_c.hi[s], tree_c.lo[s] - tree_r.hi[t]))
    acc = 0.0
    for g in gap:
        acc += float(g) * float(g)
    return acc


def admissible(tree_r: ClusterTree, tree_c: ClusterTree, t: int, s: int, eta: float) -> bool:
    """eq. (admissibility): max(diam) <= 2*eta*dist, decided on the squares:
    max(diam^2) <= (2 eta)^2 dist^2.  Row and column clusters may come from
    different trees (the index sets I, J, K of the product)."""
    e2 = (2.0 * eta) * (2.0 * eta)
    return max(tree_r.diam2(t), tree_c.diam2(s)) <= e2 * dist2_between(tree_r, t, tree_c, s)


class BlockTree:
    """Block tree of Definition 2 built by the recursive procedure of Section 2.

    ``kind[(t,s)]`` is 'adm' (admissible leaf), 'inadm' (inadmissible leaf)
    or 'split' (has children), for every block of the tree."""

    def __init__(self, rows: ClusterTree, cols: ClusterTree, eta: float):
        self.rows, self.cols, self.eta = rows, cols, float(eta)
        self.kind = {}
        self.children = {}
        self._build(0, 0)
        self.adm = [b for b, k in self.kind.items() if k == "adm"]
        self.inadm = [b for b, k in self.kind.items() if k == "inadm"]

    def _build(self, t, s):
        R, C = self.rows, self.cols
        if admissible(R, C, t, s, self.eta):
            self.kind[(t, s)] = "adm"
            return
        if R.is_leaf(t) and C.is_leaf(s):
            self.kind[(t, s)] = "inadm"
            return
        self.kind[(t, s)] = "split"
        # eq. (block_children)
        if R.is_leaf(t):
            ch = [(t, s2) for s2 in C.children[s]]
        elif C.is_leaf(s):
            ch = [(t2, s) for t2 in R.children[t]]
        else:
            ch = [(t2, s2) for t2 in R.children[t] for s2 in C.children[s]]
        self.children[(t, s)] = ch
        for b in ch:
            self._build(*b)

    def is_adm(self, t, s):
        return self.kind.get((t, s)) == "adm"

    def is_inadm(self, t, s):
        return self.kind.get((t, s)) == "inadm"

    def is_split(self, t, s):
        return self.kind.get((t, s)) == "split"

    def contains(self, t, s):
        return (t, s) in self.kind
