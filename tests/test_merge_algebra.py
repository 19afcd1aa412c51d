"""The algebra of the device's coarsening merges, checked in FP64 on the CPU.

A merge joins two truncated pieces W_a V_a^* and W_b V_b^* of a block
(W = U S with U, V orthonormal; Section 5.1 agglomerates such pieces and
truncates the result).  The device never factors the stacked [W_a, W_b] or
[V_a, V_b] with a wide QR.  It takes one Gram-Schmidt step against piece a:

- pieces side by side (same rows): G = [W_a, W_b] diag(V_a, V_b)^*, and with
  C = U_a^* W_b, P = W_b - U_a C = Q_P R_P the matrix
  R_G = [[S_a, C], [0, R_P]] has the singular values and right singular
  vectors of [W_a, W_b], hence of G;
- pieces on top of each other (same columns): G = diag(W_a, W_b) [V_a, V_b]^*,
  and with C = V_a^* V_b, P = V_b - V_a C = Q_P R_P the matrix
  M = [[S_a, 0], [S_b C^*, S_b R_P^*]] has the Gram matrix of
  G^ = U R_Z^*, R_Z = [[I, C], [0, R_P]].

These tests compare both constructions with an SVD of the merged block
itself, also where piece b lies almost in the span of piece a (a single
projection must still give the small singular values to absolute accuracy).
"""
import numpy as np
import pytest


def _orth(rng, m, k):
    q, _ = np.linalg.qr(rng.standard_normal((m, k)))
    return q


def _piece(rng, m, n, k, decay):
    """W V^* with W = U S (U, V orthonormal, S lower triangular as on the
    device, where S is the transposed R factor of a Cholesky step)."""
    U, V = _orth(rng, m, k), _orth(rng, n, k)
    S = np.tril(rng.standard_normal((k, k))) * decay ** np.arange(k)[None, :]
    return U, S, U @ S, V


def _gs(Ua, X):
    C = Ua.T @ X
    P = X - Ua @ C
    R_P = np.linalg.qr(P, mode="r")
    return C, R_P


def _sv(A):
    return np.linalg.svd(A, compute_uv=False)


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("ka,kb", [(7, 5), (12, 12), (1, 9), (9, 1)])
def test_side_by_side_merge(seed, ka, kb):
    rng = np.random.default_rng(seed)
    m, na, nb = 90, 40, 50
    Ua, Sa, Wa, Va = _piece(rng, m, na, ka, 0.7)
    Ub, Sb, Wb, Vb = _piece(rng, m, nb, kb, 0.5)
    G = np.hstack([Wa @ Va.T, Wb @ Vb.T])
    C, R_P = _gs(Ua, Wb)
    R_G = np.block([[Sa, C], [np.zeros((R_P.shape[0], ka)), R_P]])
    s_ref, s = _sv(G)[: ka + kb], _sv(R_G)
    assert np.allclose(s, s_ref, rtol=0, atol=1e-13 * s_ref[0])
    # right singular vectors of R_G, mapped through diag(V_a, V_b), are those of G
    _, _, Vt = np.linalg.svd(R_G)
    Z = np.zeros((na + nb, ka + kb))
    Z[:na, :ka], Z[na:, ka:] = Va, Vb
    r = 3
    P_ref = np.linalg.svd(G)[2][:r].T
    P_dev = Z @ Vt[:r].T
    assert np.allclose(np.abs(P_ref.T @ P_dev), np.eye(r), atol=1e-10)


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("ka,kb", [(7, 5), (12, 12), (1, 9), (9, 1)])
def test_stacked_merge(seed, ka, kb):
    rng = np.random.default_rng(seed)
    ma, mb, n = 45, 35, 80
    Ua, Sa, Wa, Va = _piece(rng, ma, n, ka, 0.7)
    Ub, Sb, Wb, Vb = _piece(rng, mb, n, kb, 0.5)
    G = np.vstack([Wa @ Va.T, Wb @ Vb.T])
    C, R_P = _gs(Va, Vb)
    # G^ = U R_Z^*: rows of a [W_a, 0], rows of b [W_b C^*, W_b R_P^*]
    Gh = np.block([[Wa, np.zeros((ma, kb))], [Wb @ C.T, Wb @ R_P.T]])
    M = np.block([[Sa, np.zeros((ka, kb))], [Sb @ C.T, Sb @ R_P.T]])
    assert np.allclose(M.T @ M, Gh.T @ Gh, atol=1e-12 * np.linalg.norm(Gh) ** 2)
    s_ref = _sv(G)[: ka + kb]
    assert np.allclose(_sv(M), s_ref, rtol=0, atol=1e-13 * s_ref[0])
    assert np.allclose(_sv(Gh), s_ref, rtol=0, atol=1e-13 * s_ref[0])


@pytest.mark.parametrize("tiny", [1e-6, 1e-10, 1e-14])
def test_nearly_dependent_pieces_keep_small_singular_values(tiny):
    """Piece b lies in the span of piece a up to `tiny`: the merged block has
    singular values near `tiny`, and one projection must resolve them to an
    absolute error of a few units of roundoff times the block's norm."""
    rng = np.random.default_rng(7)
    m, ka, kb = 120, 10, 6
    Ua = _orth(rng, m, ka)
    Sa = np.tril(rng.standard_normal((ka, ka))) + 3 * np.eye(ka)
    Wa = Ua @ Sa
    E = _orth(rng, m, kb)
    E -= Ua @ (Ua.T @ E)
    E = np.linalg.qr(E)[0]
    Wb = Ua @ rng.standard_normal((ka, kb)) + tiny * E @ np.diag(np.linspace(1.0, 0.5, kb))
    U = np.hstack([Wa, Wb])
    C, R_P = _gs(Ua, Wb)
    R_G = np.block([[Sa, C], [np.zeros((kb, ka)), R_P]])
    s_ref, s = _sv(U), _sv(R_G)
    assert np.max(np.abs(s - s_ref)) <= 50 * np.finfo(float).eps * s_ref[0]
    if tiny >= 1e-10:  # the small ones are resolved relative to the block norm
        assert np.allclose(s[-kb:], s_ref[-kb:], rtol=1e-3 if tiny < 1e-8 else 1e-7)
