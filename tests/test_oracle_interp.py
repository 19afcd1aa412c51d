"""Pins of the oracle's operands (eq. interpolation, vsw, transfer; Definitions 3, 4)."""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from oracle.h2 import Interp, cheb_nodes_1d, lagrange_1d, dlagrange_1d
from paper_2403_01566_amd import workloads as W


def test_chebyshev_nodes_closed_form():
    # p = 3 on [-1, 1]: cos(pi/6), cos(pi/2), cos(5 pi/6)
    x = cheb_nodes_1d(-1.0, 1.0, 3)
    assert np.allclose(x, [math.sqrt(3) / 2, 0.0, -math.sqrt(3) / 2], atol=1e-15)


@pytest.mark.parametrize("p", [2, 3, 4, 6])
def test_lagrange_property_and_reproduction(p):
    nodes = cheb_nodes_1d(0.2, 1.7, p)
    assert np.allclose(lagrange_1d(nodes, nodes), np.eye(p), atol=1e-13)
    x = np.linspace(0.1, 1.8, 37)
    L = lagrange_1d(nodes, x)
    D = dlagrange_1d(nodes, x)
    for deg in range(p):
        f = nodes ** deg
        assert np.allclose(L @ f, x ** deg, atol=1e-11)
        df = deg * x ** (deg - 1) if deg > 0 else np.zeros_like(x)
        assert np.allclose(D @ f, df, atol=1e-9)


@pytest.mark.parametrize("dim,p", [(2, 3), (3, 2), (3, 4)])
def test_tensor_lagrange_reproduces_polynomials(dim, p):
    if dim == 2:
        P = W.uniform2d(300, 3)
    else:
        P, _ = W.icosphere(2)
    T = O.ClusterTree(P, 40)
    ip = Interp(T, p)
    rng = np.random.default_rng(0)
    for t in [0, 1, T.leaves()[0]]:
        X = T.points[T.perm[T.begin[t]:T.end[t]]]
        L = ip.lagrange(t, X)
        nodes = ip.nodes(t)
        assert np.allclose(ip.lagrange(t, nodes), np.eye(ip.k), atol=1e-11)
        for e in itertools.product(range(p), repeat=dim):
            c = rng.standard_normal()
            fX = c * np.prod(X ** np.array(e), axis=1)
            fN = c * np.prod(nodes ** np.array(e), axis=1)
            assert np.allclose(L @ fN, fX, atol=1e-9 * max(1, abs(c)))


@pytest.mark.parametrize("kernel", [O.KERNEL_NEG_LOG, O.KERNEL_SLP, O.KERNEL_DLP])
def test_nested_transfers_exact(kernel):
    if kernel == O.KERNEL_NEG_LOG:
        P, Nn = W.uniform2d(500, 1), None
        p = 3
    else:
        P, Nn = W.icosphere(2)
        p = 3
    T = O.ClusterTree(P, 30)
    M = O.build_interpolated(T, kernel, p, 0.5, normals=Nn)
    Pp = T.points[T.perm]
    ip = Interp(T, p)
    for t in range(T.ncl):
        # V_t as defined directly (Lagrange polynomials of t at its points) equals the nested form
        X = Pp[T.begin[t]:T.end[t]]
        direct = ip.lagrange(t, X)
        assert np.allclose(M.V.full(t), direct, atol=1e-11 * max(1, np.abs(direct).max()))
        if kernel == O.KERNEL_DLP:
            Nt = Nn[T.perm][T.begin[t]:T.end[t]]
            dW = ip.lagrange_normal_deriv(t, X, Nt)
            assert np.allclose(M.W.full(t), dW, atol=1e-9 * max(1, np.abs(dW).max()))


def test_kernel_matrix_definitions():
    X = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    Y = np.array([[0.0, 2.0, 0.0], [0.0, 0.0, 0.0]])
    ny = np.array([[0.0, 1.0, 0.0], [1.0, 0.0, 0.0]])
    K = O.kernel_matrix(O.KERNEL_SLP, X, Y)
    assert abs(K[0, 0] - 1 / (8 * math.pi)) < 1e-15 and K[0, 1] == 0.0
    D = O.kernel_matrix(O.KERNEL_DLP, X, Y, ny)
    # (x - y) . n_y / (4 pi |x-y|^3): x=(0,0,0), y=(0,2,0), n=(0,1,0) -> -2/(4 pi 8)
    assert abs(D[0, 0] + 2 / (32 * math.pi)) < 1e-15
    assert abs(D[1, 1] - 1 / (4 * math.pi)) < 1e-15
    L = O.kernel_matrix(O.KERNEL_NEG_LOG, X[:, :2], Y[:, :2])
    assert abs(L[0, 0] + math.log(2.0)) < 1e-15


def test_interpolation_error_decreases_with_order():
    P = W.uniform2d(400, 7)
    T = O.ClusterTree(P, 32)
    errs = []
    for p in (2, 4, 6):
        M = O.build_interpolated(T, O.KERNEL_NEG_LOG, p, 0.5)
        G = O.kernel_matrix(O.KERNEL_NEG_LOG, P, P)
        errs.append(np.linalg.norm(M.to_dense() - G) / np.linalg.norm(G))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-4


def test_slp_diagonal_rule_and_dense_exact_nearfield():
    P, Nn = W.icosphere(2)
    T = O.ClusterTree(P, 40)
    M = O.build_interpolated(T, O.KERNEL_SLP, 2, 1.0, diag=O.DIAG_ROW_MEAN)
    G = O.kernel_matrix(O.KERNEL_SLP, P, P)
    D = M.to_dense()
    for (t, s) in M.blocks.inadm:
        I = T.perm[T.begin[t]:T.end[t]]
        J = T.perm[T.begin[s]:T.end[s]]
        blk = D[np.ix_(I, J)]
        ref = G[np.ix_(I, J)]
        off = I[:, None] != J[None, :]
        assert np.allclose(blk[off], ref[off], rtol=1e-14)
    # row i diagonal = mean of the row's other nearfield entries
    i = 17
    js = []
    for (t, s) in M.blocks.inadm:
        I = T.perm[T.begin[t]:T.end[t]]
        if i in I:
            js.extend(j for j in T.perm[T.begin[s]:T.end[s]] if j != i)
    assert abs(D[i, i] - G[i, js].mean()) < 1e-12


def test_flat_clusters_keep_double_layer_bases_bounded():
    """Clusters inside one face of the cube surface have zero thickness along
    the normal; their boxes are widened to 1e-2 of the longest edge, so the
    normal derivatives of the Lagrange polynomials stay of size p^2 / width."""
    P, nrm = W.cube_surface(16)
    T = O.ClusterTree(P, 64)
    edges = T.hi - T.lo
    assert (edges.min(axis=1) == 0.0).any()  # the case exists
    A = O.build_interpolated(T, O.KERNEL_DLP, 4, 1.0, normals=nrm)
    assert max(np.abs(v).max() for v in A.W.leaf.values()) < 1e4
    # the factored and the dense form agree to rounding (no cancellation)
    x = np.random.default_rng(0).standard_normal(T.n)
    D = A.to_dense()
    assert np.abs(A.matvec(x) - D @ x).max() <= 1e-13 * np.abs(D).sum(axis=1).max() * np.abs(x).max()
