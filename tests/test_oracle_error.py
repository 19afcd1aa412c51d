"""Pins of the oracle's matrix-vector products and of the power-iteration
estimate of the global error (Section 2; the error column of Section 6)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2403_01566_amd import workloads as W


def _small_h2():
    P = W.uniform2d(300, 3)
    T = O.ClusterTree(P, 24)
    return O.build_interpolated(T, O.KERNEL_NEG_LOG, 4, 0.5)


def test_matvec_and_adjoint_match_the_dense_matrix():
    A = _small_h2()
    D = A.to_dense()
    rng = np.random.default_rng(1)
    x = rng.standard_normal(D.shape[1])
    X = rng.standard_normal((D.shape[1], 3))
    assert np.allclose(A.matvec(x), D @ x, rtol=0, atol=1e-12 * np.abs(D).sum(axis=1).max())
    assert np.allclose(A.matvec(X), D @ X, rtol=0, atol=1e-12 * np.abs(D).sum(axis=1).max() * 3)
    assert np.allclose(A.rmatvec(x), D.T @ x, rtol=0, atol=1e-12 * np.abs(D).sum(axis=0).max())
    assert np.allclose(A.rmatvec(X), D.T @ X, rtol=0, atol=1e-12 * np.abs(D).sum(axis=0).max() * 3)


@pytest.mark.parametrize("iters", [1, 2, 5, 10])
def test_power_norm_closed_form_on_a_diagonal(iters):
    # E = diag(d), z0 = ones: after j steps z is d^(2j) / ||d^(2j)||, and the
    # last sigma is ||d * z|| for the z of that step (j = iters - 1)
    d = np.array([3.0, 2.0, 1.0, 0.5, 0.25])
    est = O.power_norm(lambda z: d * z, lambda w: d * w, np.ones(5), iters)
    j = iters - 1
    expect = math.sqrt(float(np.sum(d ** (4 * j + 2)))) / math.sqrt(float(np.sum(d ** (4 * j))))
    assert est == pytest.approx(expect, rel=1e-14)
    assert est <= 3.0


def test_power_norm_converges_to_the_spectral_norm_and_stays_below_it():
    rng = np.random.default_rng(7)
    A = rng.standard_normal((30, 20))
    s2 = np.linalg.norm(A, 2)
    z0 = rng.standard_normal(20)
    for it in range(1, 11):
        assert O.power_norm(lambda z: A @ z, lambda w: A.T @ w, z0, it) <= s2 * (1 + 1e-14)
    assert O.power_norm(lambda z: A @ z, lambda w: A.T @ w, z0, 400) == pytest.approx(s2, rel=1e-9)


def test_product_error_of_the_exact_product():
    A = _small_h2()
    D = A.to_dense()
    E = D @ D
    z0 = np.random.default_rng(3).standard_normal(D.shape[1])
    err, nxy = O.product_error(A, A, lambda z: E @ z, lambda w: E.T @ w, z0, 10)
    assert err <= 1e-12 * nxy
    assert nxy <= np.linalg.norm(E, 2) * (1 + 1e-14)
    assert nxy >= 0.99 * np.linalg.norm(E, 2)
    err0, nxy0 = O.product_error(A, A, None, None, z0, 10)
    assert err0 == 0.0 and nxy0 == nxy
