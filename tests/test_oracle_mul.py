"""Pins of the oracle's product (Sections 3-5).  Brute force on small inputs:
the exact product of the dense operands, Eckart-Young, orthonormality and
nestedness of the new bases, the block-relative bound, Lemma 6, special cases."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2403_01566_amd import workloads as W


def _case(name):
    if name == "grid32":
        T = O.ClusterTree(W.grid2d(32), 32)
        A = O.build_interpolated(T, O.KERNEL_NEG_LOG, 3, 0.5)
        return T, A, A
    if name == "sphere":
        P, Nn = W.icosphere(3)
        T = O.ClusterTree(P, 64)
        A = O.build_interpolated(T, O.KERNEL_SLP, 3, 1.0, diag=O.DIAG_ROW_MEAN)
        return T, A, A
    if name == "slp_dlp":
        P, Nn = W.icosphere(2)
        T = O.ClusterTree(P, 20)
        A = O.build_interpolated(T, O.KERNEL_SLP, 2, 1.0, diag=O.DIAG_ROW_MEAN)
        B = O.build_interpolated(T, O.KERNEL_DLP, 2, 1.0, normals=Nn)
        return T, A, B
    if name == "random2d":
        T = O.ClusterTree(W.uniform2d(900, 11), 24)
        A = O.build_interpolated(T, O.KERNEL_NEG_LOG, 4, 0.5)
        return T, A, A
    raise KeyError(name)


_cache = {}


def _run(name, eps):
    key = (name, eps)
    if key not in _cache:
        T, A, B = _case(name)
        C, info = O.mul(A, B, eps)
        _cache[key] = (T, A, B, C, info)
    return _cache[key]


CASES = [("grid32", 1e-4), ("sphere", 1e-6), ("slp_dlp", 1e-4), ("random2d", 1e-5)]


@pytest.mark.parametrize("name,eps", CASES)
def test_basis_products_recursive_form(name, eps):
    """P_s = W_{X,s}^* V_{Y,s} also satisfies P_s = sum F_{s'}^* P_{s'} E_{s'} (Section 4.1)."""
    T, A, B, C, info = _run(name, eps)
    for s in range(T.ncl):
        if T.children[s]:
            rec = sum(A.W.transfer[c].T @ info.P[c] @ B.V.transfer[c] for c in T.children[s])
            assert np.allclose(rec, info.P[s], atol=1e-10 * max(1, np.abs(info.P[s]).max()))


@pytest.mark.parametrize("name,eps", CASES)
def test_exact_intermediate_equals_dense_product(name, eps):
    """The induced block structure represents XY exactly (end of Section 3)."""
    T, A, B, C, info = _run(name, eps)
    D = A.to_dense_permuted() @ B.to_dense_permuted()
    scale = np.abs(D).max()
    for b, (U, Z) in info.exact.items():
        t, r = b
        blk = D[T.begin[t]:T.end[t], T.begin[r]:T.end[r]]
        assert np.abs(U @ Z.T - blk).max() <= 1e-12 * scale
    for b, N in C.N.items():
        t, r = b
        blk = D[T.begin[t]:T.end[t], T.begin[r]:T.end[r]]
        assert np.abs(N - blk).max() <= 1e-12 * scale


@pytest.mark.parametrize("name,eps", CASES)
def test_block_relative_error_bound(name, eps):
    """Every leaf block: ||(XY)|_b - C|_b||_2 <= eps ||(XY)|_b||_2 (Section 5.3)."""
    T, A, B, C, info = _run(name, eps)
    errs = O.block_errors(A, B, C)
    assert len(errs) == len(C.blocks.adm) + len(C.blocks.inadm)
    worst = max(e / n for e, n in errs.values() if n > 0)
    assert worst <= eps, worst
    # the result is a genuine compression: ranks below the exact widths
    assert max(C.V.rank.values()) < T.size(0)


@pytest.mark.parametrize("name,eps", CASES)
def test_coarsening_eckart_young(name, eps):
    """||G_b - G~_b||_2 = sigma_{kappa+1}(G_b) <= delta_c ||G_b|| (Section 5.1)."""
    T, A, B, C, info = _run(name, eps)
    for b, (U, Z) in info.exact.items():
        G = U @ Z.T
        Uc, Zc, sk = info.coarse[b]
        sv = np.linalg.svd(G, compute_uv=False)
        err = np.linalg.norm(G - Uc @ Zc.T, 2)
        kap = info.kappa[b]
        nxt = sv[kap] if kap < len(sv) else 0.0
        assert abs(err - nxt) <= 1e-10 * sv[0] + 1e-300
        assert err <= info.delta_c * sv[0] * (1 + 1e-9)
        assert abs(info.nu[b] - sv[0]) <= 1e-10 * sv[0]
        # the column factor is isometric
        assert np.allclose(Zc.T @ Zc, np.eye(kap), atol=1e-10)


@pytest.mark.parametrize("name,eps", CASES)
def test_result_bases_isometric_and_nested(name, eps):
    """V_t^* V_t = I for every cluster (Section 5.2); nestedness holds by construction."""
    T, A, B, C, info = _run(name, eps)
    for basis in (C.V, C.W):
        for t in range(T.ncl):
            Vt = basis.full(t)
            k = basis.rank[t]
            assert Vt.shape == (T.size(t), k)
            assert np.allclose(Vt.T @ Vt, np.eye(k), atol=1e-10)
            if T.children[t]:
                for c in T.children[t]:
                    off = T.begin[c] - T.begin[t]
                    assert np.allclose(Vt[off:off + T.size(c)], basis.full(c) @ basis.transfer[c], atol=1e-12)


@pytest.mark.parametrize("name,eps", CASES)
def test_row_and_column_projection_errors(name, eps):
    """Each admissible block: ||G~ - V V^* G~|| <= delta_r nu_b and
    ||G~ - G~ W W^*|| <= delta_w nu_b (weighted construction, Section 5.3)."""
    T, A, B, C, info = _run(name, eps)
    for b in C.blocks.adm:
        t, r = b
        Uc, Zc, sk = info.coarse[b]
        Gt = Uc @ Zc.T
        Vt, Wr = C.V.full(t), C.W.full(r)
        nu = info.nu[b]
        if nu == 0:
            continue
        er = np.linalg.norm(Gt - Vt @ (Vt.T @ Gt), 2)
        ec = np.linalg.norm(Gt - (Gt @ Wr) @ Wr.T, 2)
        assert er <= eps / 4 * nu * (1 + 1e-8)
        assert ec <= eps / 4 * nu * (1 + 1e-8)


@pytest.mark.parametrize("name,eps", CASES)
def test_error_decomposition_sum(name, eps):
    """Section 5.3's error decomposition, formed per descendant.  For every
    admissible block b = (t, r) and every cluster s in desc(t) (t included)
    let e_{s,b} be the part of the unweighted piece G^_{s,b} dropped by the
    truncation at s (recorded by the oracle).  Then
      (a) e_{s,b} <= omega_{s,b} eps_r with omega_{s,b} = theta^{(level s -
          level t)/2} nu_b (the weighted SVD truncation keeps every dropped
          singular value of the weighted matrix below eps_r);
      (b) sum_{s in desc(t)} e_{s,b}^2 <= eps_r^2 nu_b^2 / (1 - sigma theta);
      (c) in the Frobenius norm the decomposition is exact: the projection
          error ||G~_b - V_t V_t^* G~_b||_F^2 equals sum_s ||.||_F^2 of the
          local errors (the nested isometric bases make the terms orthogonal);
      (d) in the spectral norm it is an upper bound of that projection error.
    Both sides, rows and (on the adjoint) columns."""
    T, A, B, C, info = _run(name, eps)
    th, sg = info.theta, info.sigma_br

    def desc(t):
        out, stack = [], [t]
        while stack:
            s = stack.pop()
            out.append(s)
            stack.extend(T.children[s])
        return out

    checked = 0
    for side in ("row", "col"):
        local = info.row_local if side == "row" else info.col_local
        tol = info.tol_r if side == "row" else info.tol_w
        for b in C.blocks.adm:
            nu = info.nu[b]
            if nu == 0.0 or info.kappa[b] == 0:
                continue
            t = b[0] if side == "row" else b[1]
            Uc, Zc, sk = info.coarse[b]
            G = Uc @ Zc.T if side == "row" else Zc @ Uc.T   # G~_b = U'_b Z'_b^*, or its adjoint
            V = C.V.full(t) if side == "row" else C.W.full(t)
            P = G - V @ (V.T @ G)
            s2 = f2 = 0.0
            for s in desc(t):
                e_spec, e_frob = local[(s, b)]
                w = th ** ((T.level[s] - T.level[t]) / 2.0) * nu
                assert e_spec <= w * tol * (1 + 1e-9) + 1e-14 * nu, (side, b, s)      # (a)
                s2 += e_spec ** 2
                f2 += e_frob ** 2
            assert s2 <= tol ** 2 * nu ** 2 / (1.0 - sg * th) * (1 + 1e-9)          # (b)
            pf = np.linalg.norm(P)
            # (rounding: P is a difference of terms of size nu)
            assert abs(pf - math.sqrt(f2)) <= 1e-6 * math.sqrt(f2) + 1e-12 * nu, (side, b)   # (c)
            assert np.linalg.norm(P, 2) <= math.sqrt(s2) * (1 + 1e-6) + 1e-12 * nu          # (d)
            checked += 1
    assert checked > 0


def test_lemma6_product_admissibility():
    """If P_tr is non-empty there is s with eta/(eta+1) dist(t,r) < max diam (Lemma 6),
    and the number of same-level partners stays bounded."""
    for name, eps in CASES:
        T, A, B, C, info = _run(name, eps)
        eta = A.blocks.eta
        per_t = {}
        for (t, r, ss) in info.induced_P:
            assert any(eta / (eta + 1) * T.dist(t, r) < max(T.diam(t), T.diam(s), T.diam(r)) for s in ss)
            if T.level[t] == T.level[r]:
                per_t.setdefault(t, set()).add(r)
        assert max(len(v) for v in per_t.values()) <= 40


def test_single_leaf_is_plain_product():
    """n <= leaf size: one inadmissible block, C = A B exactly (a textbook GEMM)."""
    P = W.uniform2d(30, 4)
    T = O.ClusterTree(P, 32)
    A = O.build_interpolated(T, O.KERNEL_NEG_LOG, 3, 0.5)
    C, info = O.mul(A, A, 1e-4)
    G = O.kernel_matrix(O.KERNEL_NEG_LOG, P, P)
    assert np.allclose(C.to_dense(), G @ G, rtol=0, atol=1e-12 * np.abs(G @ G).max())


def test_identity_right_factor():
    """B = I as an H2 matrix: C|_b approximates A|_b within eps per block."""
    T = O.ClusterTree(W.uniform2d(600, 9), 24)
    A = O.build_interpolated(T, O.KERNEL_NEG_LOG, 3, 0.5)
    I = O.identity_h2(T, 0.5, 9)
    eps = 1e-5
    C, info = O.mul(A, I, eps)
    Ad = A.to_dense_permuted()
    for b in list(C.blocks.adm) + list(C.blocks.inadm):
        t, r = b
        ex = Ad[T.begin[t]:T.end[t], T.begin[r]:T.end[r]]
        e = np.linalg.norm(ex - C.block_dense(t, r), 2)
        assert e <= eps * np.linalg.norm(ex, 2) + 1e-14


def test_scaling_keeps_ranks():
    T, A, B, C, info = _run("grid32", 1e-4)
    A2 = O.build_interpolated(T, O.KERNEL_NEG_LOG, 3, 0.5)
    for k in A2.S:
        A2.S[k] = 3.0 * A2.S[k]
    for k in A2.N:
        A2.N[k] = 3.0 * A2.N[k]
    C2, info2 = O.mul(A2, A, 1e-4)
    assert C2.V.rank == C.V.rank and C2.W.rank == C.W.rank
    assert np.allclose(C2.to_dense(), 3.0 * C.to_dense(), atol=1e-10 * np.abs(C.to_dense()).max())


def test_symmetric_square_gives_symmetric_result():
    T, A, B, C, info = _run("grid32", 1e-4)
    D = C.to_dense()
    ref = A.to_dense() @ A.to_dense()
    assert np.linalg.norm(D - D.T, 2) <= 2e-4 * np.linalg.norm(ref, 2)
    assert C.V.rank == C.W.rank


def test_tiny_eps_reproduces_product():
    T = O.ClusterTree(W.uniform2d(400, 2), 24)
    A = O.build_interpolated(T, O.KERNEL_NEG_LOG, 3, 0.5)
    C, info = O.mul(A, A, 1e-13)
    ref = A.to_dense() @ A.to_dense()
    assert np.linalg.norm(C.to_dense() - ref, 2) <= 1e-11 * np.linalg.norm(ref, 2)


def test_incompatible_and_invalid_arguments():
    T = O.ClusterTree(W.uniform2d(100, 2), 24)
    T2 = O.ClusterTree(W.uniform2d(100, 3), 24)
    A = O.build_interpolated(T, O.KERNEL_NEG_LOG, 3, 0.5)
    B = O.build_interpolated(T2, O.KERNEL_NEG_LOG, 3, 0.5)
    with pytest.raises(ValueError):
        O.mul(A, B, 1e-4)
    with pytest.raises(ValueError):
        O.mul(A, A, 0.0)
    with pytest.raises(ValueError):
        O.mul(A, A, 1.5)


def test_rectangular_product_three_trees():
    """X (I x J) times Y (J x K) on three different point sets (the index sets
    of Section 3): the cross-tree admissibility matches brute force, the
    block trees partition the index products, and every admissible block of
    the result meets the bound against the dense product."""
    P1, P2, P3 = W.uniform2d(300, 21), W.uniform2d(400, 22), W.uniform2d(250, 23)
    T1, T2, T3 = (O.ClusterTree(P, 20) for P in (P1, P2, P3))
    # admissibility across trees against a direct box computation
    for t in range(T1.ncl):
        for s in range(T2.ncl):
            gap = np.maximum(0.0, np.maximum(T1.lo[t] - T2.hi[s], T2.lo[s] - T1.hi[t]))
            d = float(np.sqrt((gap ** 2).sum()))
            dm = max(float(np.linalg.norm(T1.hi[t] - T1.lo[t])), float(np.linalg.norm(T2.hi[s] - T2.lo[s])))
            if abs(dm - d) > 1e-9 * max(dm, 1.0):  # away from exact ties
                assert O.admissible(T1, T2, t, s, 0.5) == (dm <= d)
    X = O.build_interpolated(T1, O.KERNEL_NEG_LOG, 4, 0.5, cols=T2)
    Y = O.build_interpolated(T2, O.KERNEL_NEG_LOG, 4, 0.5, cols=T3)
    for M, A, B in ((X, T1, T2), (Y, T2, T3)):
        cover = np.zeros((A.n, B.n), dtype=int)
        for (t, s) in M.blocks.adm + M.blocks.inadm:
            cover[A.begin[t]:A.end[t], B.begin[s]:B.end[s]] += 1
        assert (cover == 1).all()
    Xd, Yd = X.to_dense(), Y.to_dense()
    K = O.kernel_matrix(O.KERNEL_NEG_LOG, P1, P2)
    assert np.abs(Xd - K).max() <= 1e-3 * np.abs(K).max()   # interpolation, order 4
    C, info = O.mul(X, Y, 1e-5)
    assert C.rows is T1 and C.cols is T3
    errs = O.block_errors(X, Y, C)
    assert all(e <= 1e-5 * n for (b, (e, n)) in errs.items() if b in C.blocks.adm)
    D = C.to_dense()
    E = Xd @ Yd
    assert np.linalg.norm(D - E, 2) <= 1e-5 * np.linalg.norm(E, 2) * 10
