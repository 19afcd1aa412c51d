"""Pins of the oracle's trees (Definitions 1 and 2, eq. admissibility)."""
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2403_01566_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden", "grid32_cluster_tree.txt")


def _golden():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        rows.append([float(x) for x in line.split()])
    return rows


def test_grid32_tree_closed_form():
    T = O.ClusterTree(W.grid2d(32), 32)
    assert T.ncl == 63 and T.depth == 6
    for lev, ncl, px, py, sx, sy, diam in _golden():
        cs = [c for c in range(T.ncl) if T.level[c] == lev]
        assert len(cs) == ncl
        for c in cs:
            X = T.points[T.perm[T.begin[c]:T.end[c]]]
            assert len(np.unique(X[:, 0])) == px and len(np.unique(X[:, 1])) == py
            side = (T.hi[c] - T.lo[c]) * 32
            assert np.allclose(side, [sx, sy])
            assert abs(T.diam(c) - diam) < 1e-9
            assert abs(T.diam(c) - math.hypot(sx, sy) / 32) < 1e-12


@pytest.mark.parametrize("gen", ["grid", "uniform", "sphere"])
def test_cluster_tree_partition(gen):
    if gen == "grid":
        P = W.grid2d(16)
    elif gen == "uniform":
        P = W.uniform2d(700, 5)
    else:
        P, _ = W.icosphere(2)
    T = O.ClusterTree(P, 20)
    assert sorted(T.perm.tolist()) == list(range(len(P)))
    for t in range(T.ncl):
        ch = T.children[t]
        if ch:
            assert len(ch) == 2
            assert T.begin[ch[0]] == T.begin[t] and T.end[ch[-1]] == T.end[t]
            assert T.end[ch[0]] == T.begin[ch[1]]
            for c in ch:
                assert T.level[c] == T.level[t] + 1 and T.parent[c] == t
                # child box inside parent box (Omega_t' subset Omega_t)
                assert np.all(T.lo[c] >= T.lo[t] - 1e-15) and np.all(T.hi[c] <= T.hi[t] + 1e-15)
        else:
            assert T.size(t) <= 20
        X = T.points[T.perm[T.begin[t]:T.end[t]]]
        assert np.allclose(X.min(0), T.lo[t]) and np.allclose(X.max(0), T.hi[t])


def test_box_distance_and_diameter():
    T = O.ClusterTree(np.array([[0.0, 0.0], [1.0, 0.0], [3.0, 4.0], [3.0, 5.0]]), 1)
    # leaves hold single points; the distance of two point-boxes is their distance
    leaves = T.leaves()
    pts = {l: T.points[T.perm[T.begin[l]]] for l in leaves}
    for a in leaves:
        for b in leaves:
            assert abs(T.dist(a, b) - np.linalg.norm(pts[a] - pts[b])) < 1e-12
    assert abs(T.diam(0) - math.hypot(3, 5)) < 1e-12


@pytest.mark.parametrize("eta", [0.5, 1.0])
def test_block_tree_invariants(eta):
    P, _ = W.icosphere(3)
    T = O.ClusterTree(P, 40)
    bt = O.BlockTree(T, T, eta)
    cover = np.zeros((T.n, T.n), dtype=np.int32)
    for (t, s), kind in bt.kind.items():
        if kind == "split":
            # the parent of every block is inadmissible, and children follow eq. block_children
            assert not O.admissible(T, T, t, s, eta)
            ch = bt.children[(t, s)]
            if T.is_leaf(t):
                assert ch == [(t, s2) for s2 in T.children[s]]
            elif T.is_leaf(s):
                assert ch == [(t2, s) for t2 in T.children[t]]
            else:
                assert len(ch) == 4
            continue
        cover[T.begin[t]:T.end[t], T.begin[s]:T.end[s]] += 1
        if kind == "adm":
            assert max(T.diam(t), T.diam(s)) <= 2 * eta * T.dist(t, s)
        else:
            assert T.is_leaf(t) and T.is_leaf(s)
            assert not O.admissible(T, T, t, s, eta)
    # leaves partition I x J exactly once
    assert cover.min() == 1 and cover.max() == 1


def test_grid32_admissibility_pattern():
    """With eta = 1/2 on the 32x32 grid no block at levels 1-2 is admissible, and
    at level 3 the admissible pairs are three columns of clusters apart."""
    T = O.ClusterTree(W.grid2d(32), 32)
    bt = O.BlockTree(T, T, 0.5)
    levels = {T.level[t] for (t, s) in bt.adm}
    assert min(levels) == 3
    for (t, s) in bt.adm:
        if T.level[t] == 3:
            dx = abs(T.lo[t][0] - T.lo[s][0]) * 32
            assert dx >= 24 - 1e-9
