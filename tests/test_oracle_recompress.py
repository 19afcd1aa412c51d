"""Pins of the oracle's H -> H2 recompression (Section 5 on its own: the
truncation of each block, the weighted row and column bases, the couplings)."""
import numpy as np
import pytest

import oracle as O
from paper_2403_01566_amd import workloads as W


def _h_matrix(P, leaf, eta, rank_tol=1e-13, kernel=O.KERNEL_NEG_LOG):
    """H-matrix of the kernel matrix on the block tree of (T, T, eta): every
    admissible block as the factors of its SVD truncated at rank_tol relative
    (its own low-rank form), every inadmissible block dense."""
    T = O.ClusterTree(P, leaf)
    K = O.kernel_matrix(kernel, P, P)
    Kp = K[np.ix_(T.perm, T.perm)]
    bt = O.BlockTree(T, T, eta)
    factors, near = {}, {}
    for (t, s) in bt.adm:
        G = Kp[T.begin[t]:T.end[t], T.begin[s]:T.end[s]]
        U, sv, Vt = np.linalg.svd(G, full_matrices=False)
        k = max(1, int(np.count_nonzero(sv > rank_tol * sv[0])))
        factors[(t, s)] = (U[:, :k] * sv[:k], Vt[:k].T)
    for (t, s) in bt.inadm:
        near[(t, s)] = Kp[T.begin[t]:T.end[t], T.begin[s]:T.end[s]].copy()
    return T, bt, factors, near


def _block_errors(C, factors):
    worst = 0.0
    for b, (U, Z) in factors.items():
        G = U @ Z.T
        nn = np.linalg.norm(G, 2)
        if nn > 0:
            worst = max(worst, np.linalg.norm(G - C.block_dense(*b), 2) / nn)
    return worst


@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-9])
def test_block_relative_bound(eps):
    T, bt, factors, near = _h_matrix(W.grid2d(16), 16, 0.5)
    C, info = O.recompress(T, T, 0.5, factors, near, eps)
    assert _block_errors(C, factors) <= eps
    for b in bt.inadm:
        assert np.array_equal(C.block_dense(*b), near[b])   # nearfield copied


def test_bases_orthonormal_and_nested():
    T, bt, factors, near = _h_matrix(W.uniform2d(300, 5), 20, 0.5)
    C, info = O.recompress(T, T, 0.5, factors, near, 1e-6)
    for basis in (C.V, C.W):
        for t in range(T.ncl):
            Vt = basis.full(t)
            if Vt.shape[1]:
                assert np.allclose(Vt.T @ Vt, np.eye(Vt.shape[1]), atol=1e-12)
            if not T.is_leaf(t):
                # V_t restricted to a child equals V_child E_child (eq. transfer)
                for c in T.children[t]:
                    r0 = T.begin[c] - T.begin[t]
                    part = Vt[r0:r0 + T.size(c)]
                    assert np.allclose(part, basis.full(c) @ basis.transfer[c], atol=1e-12)


def test_tiny_eps_reproduces_the_input():
    T, bt, factors, near = _h_matrix(W.grid2d(16), 16, 0.5, rank_tol=1e-6)
    C, info = O.recompress(T, T, 0.5, factors, near, 1e-12)
    assert _block_errors(C, factors) <= 1e-11


def test_h2_input_keeps_its_ranks():
    """An input that already is an H2-matrix with bases of rank k: every block
    lies in the span of V_t and W_s, so the adaptive bases need no more than k
    columns (the weighted stacks of a cluster have rank <= k)."""
    P = W.grid2d(16)
    T = O.ClusterTree(P, 16)
    A = O.build_interpolated(T, O.KERNEL_NEG_LOG, 3, 0.5)          # k = 9
    factors = {b: (A.V.full(b[0]) @ A.S[b], A.W.full(b[1])) for b in A.blocks.adm}
    near = {b: A.N[b] for b in A.blocks.inadm}
    C, info = O.recompress(T, T, 0.5, factors, near, 1e-10)
    assert max(C.V.rank.values()) <= 9 and max(C.W.rank.values()) <= 9
    assert _block_errors(C, factors) <= 1e-10


def test_homogeneity():
    T, bt, factors, near = _h_matrix(W.grid2d(16), 16, 0.5)
    C1, _ = O.recompress(T, T, 0.5, factors, near, 1e-5)
    f2 = {b: (3.0 * u, z) for b, (u, z) in factors.items()}
    n2 = {b: 3.0 * v for b, v in near.items()}
    C2, _ = O.recompress(T, T, 0.5, f2, n2, 1e-5)
    assert C1.V.rank == C2.V.rank and C1.W.rank == C2.W.rank
    D1, D2 = C1.to_dense(), C2.to_dense()
    assert np.allclose(D2, 3.0 * D1, rtol=0, atol=1e-12 * np.abs(D2).max())


def test_rejects_blocks_of_another_tree():
    T, bt, factors, near = _h_matrix(W.grid2d(16), 16, 0.5)
    with pytest.raises(ValueError):
        O.recompress(T, T, 1.0, factors, near, 1e-5)
