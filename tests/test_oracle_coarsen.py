"""Pins of the oracle's sequential agglomeration (Remark 13 of Section 5.1)."""
import numpy as np
import pytest

import oracle as O
from paper_2403_01566_amd import workloads as W


def _kernel_blocks(n, m, seed):
    """A smooth far-field block (-log|x-y| between two separated point sets),
    cut into n x m blocks, each given by exact factors (G_ij, I)."""
    rng = np.random.default_rng(seed)
    X = rng.random((40 * n, 2)) * 0.5
    Y = rng.random((30 * m, 2)) * 0.5 + np.array([2.0, 0.3])
    G = O.kernel_matrix(O.KERNEL_NEG_LOG, X, Y)
    rs = np.array_split(np.arange(G.shape[0]), n)
    cs = np.array_split(np.arange(G.shape[1]), m)
    blocks = [[(G[np.ix_(r, c)], np.eye(len(c))) for c in cs] for r in rs]
    return G, blocks


@pytest.mark.parametrize("n,m", [(1, 1), (1, 3), (2, 2), (3, 2)])
@pytest.mark.parametrize("eps_hat", [1e-2, 1e-5, 1e-9])
def test_remark13_bound(n, m, eps_hat):
    G, blocks = _kernel_blocks(n, m, 7 * n + m)
    U, Z, eps = O.agglomerate_sequential(blocks, eps_hat)
    assert eps == pytest.approx(eps_hat / (2 * m * n))
    err = np.linalg.norm(G - U @ Z.T, 2)
    assert err <= eps_hat * np.linalg.norm(G, 2)
    # any approximation within eps_hat ||G|| has at least the Eckart-Young rank
    sv = np.linalg.svd(G, compute_uv=False)
    assert U.shape[1] >= int(np.count_nonzero(sv > eps_hat * sv[0]))


def test_single_step_is_the_truncated_svd():
    """One agglomeration step [A B]: the best approximation keeping
    sigma_i > eps sigma_1, so the error is sigma_{k+1} exactly."""
    G, blocks = _kernel_blocks(1, 2, 3)
    U, Z, eps = O.agglomerate_sequential(blocks, 4e-6)    # one step, eps = 1e-6
    sv = np.linalg.svd(G, compute_uv=False)
    k = int(np.count_nonzero(sv > eps * sv[0]))
    assert U.shape[1] == k
    assert np.linalg.norm(G - U @ Z.T, 2) == pytest.approx(sv[k], rel=1e-6)


def test_tiny_tolerance_reproduces_the_matrix():
    G, blocks = _kernel_blocks(2, 3, 11)
    U, Z, _ = O.agglomerate_sequential(blocks, 1e-15)
    assert np.abs(G - U @ Z.T).max() <= 1e-12 * np.abs(G).max()
