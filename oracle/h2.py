"""FP64 oracle -- H2-matrices and their construction by interpolation (test
infrastructure only; see oracle/tree.py for the usage rule).

Follows Section 2 of the paper:
  * eq. (interpolation)/(vsw): tensor interpolation of the kernel yields
    G|_{t x s} ~ V_t S_ts W_s^*, with v_{t,i nu} = l_{t,nu}(x_i) (point
    collocation stands in for the Galerkin integrals), s_{ts,nu mu} =
    g(xi_{t,nu}, xi_{s,mu}).
  * eq. (transfer): for equal order the transfer matrices are
    e_{t',nu' nu} = l_{t,nu}(xi_{t',nu'}), exact by the identity theorem.
  * Definition 3 (cluster basis) and Definition 4 (H2-matrix): leaf matrices,
    transfers, coupling matrices for admissible leaves, dense nearfield
    matrices for inadmissible leaves.

Readings: Chebyshev nodes of the first kind per axis on the cluster's bounding
box, xi_j = (a+b)/2 + (b-a)/2 cos((2j+1) pi / (2p)); the tensor index runs
with the first axis fastest; an edge shorter than max(1e-12 * root diameter,
1e-2 * the box's longest edge) is widened symmetrically to that length (a
flat cluster, e.g. inside one face of a polyhedral surface, would otherwise
give normal derivatives of the Lagrange polynomials of size 1/width).  Double layer: W_s[j, mu] =
n_j . grad l_{s,mu}(y_j), nearfield (x-y).n_y / (4 pi |x-y|^3), diagonal 0.
Single layer 1/(4 pi |x-y|): diagonal = mean of the kernel over the other
entries of the row's nearfield blocks.  -log|x-y|: diagonal 0.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from .tree import BlockTree, ClusterTree

KERNEL_NEG_LOG, KERNEL_SLP, KERNEL_DLP = 0, 1, 2
DIAG_ZERO, DIAG_ROW_MEAN = 0, 1


def kernel_matrix(kernel, X, Y, ny=None):
    """Kernel values g(x_i, y_j) for all pairs; entries with x_i == y_j are 0."""
    D = X[:, None, :] - Y[None, :, :]
    r = np.sqrt((D * D).sum(axis=2))
    same = r == 0.0
    rs = np.where(same, 1.0, r)
    if kernel == KERNEL_NEG_LOG:
        K = -np.log(rs)
    elif kernel == KERNEL_SLP:
        K = 1.0 / (4.0 * math.pi * rs)
    elif kernel == KERNEL_DLP:
        K = (D * ny[None, :, :]).sum(axis=2) / (4.0 * math.pi * rs ** 3)
    else:
        raise ValueError(kernel)
    K[same] = 0.0
    return K


def cheb_nodes_1d(a, b, p):
    j = np.arange(p)
    return 0.5 * (a + b) + 0.5 * (b - a) * np.cos((2 * j + 1) * math.pi / (2 * p))


def lagrange_1d(nodes, x):
    """L[i, j] = l_j(x_i) for the Lagrange polynomials of ``nodes``."""
    p = len(nodes)
    L = np.ones((len(x), p))
    for j in range(p):
        for m in range(p):
            if m != j:
                L[:, j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return L


def dlagrange_1d(nodes, x):
    """D[i, j] = l_j'(x_i)."""
    p = len(nodes)
    D = np.zeros((len(x), p))
    for j in range(p):
        for q in range(p):
            if q == j:
                continue
            term = np.full(len(x), 1.0 / (nodes[j] - nodes[q]))
            for m in range(p):
                if m != j and m != q:
                    term *= (x - nodes[m]) / (nodes[j] - nodes[m])
            D[:, j] += term
    return D


class Interp:
    """Per-cluster tensor Chebyshev nodes on (possibly widened) boxes."""

    def __init__(self, tree: ClusterTree, order: int):
        self.tree, self.p = tree, int(order)
        d = tree.dim
        self.k = self.p ** d
        root_diam = tree.diam(0)
        self.a = np.empty((tree.ncl, d))
        self.b = np.empty((tree.ncl, d))
        for t in range(tree.ncl):
            lo, hi = tree.lo[t].copy(), tree.hi[t].copy()
            minw = max(1e-12 * root_diam, 1e-2 * float(np.max(hi - lo)))
            for ax in range(d):
                if hi[ax] - lo[ax] < minw:
                    c = 0.5 * (lo[ax] + hi[ax])
                    lo[ax], hi[ax] = c - 0.5 * minw, c + 0.5 * minw
            self.a[t], self.b[t] = lo, hi
        # multi-index list, first axis fastest
        self.multi = [tuple(reversed(m)) for m in itertools.product(range(self.p), repeat=d)]

    def nodes1d(self, t, ax):
        return cheb_nodes_1d(self.a[t, ax], self.b[t, ax], self.p)

    def nodes(self, t):
        """k x d tensor nodes of cluster t."""
        d = self.tree.dim
        n1 = [self.nodes1d(t, ax) for ax in range(d)]
        return np.array([[n1[ax][m[ax]] for ax in range(d)] for m in self.multi])

    def lagrange(self, t, X):
        """|X| x k values l_{t,nu}(x)."""
        d = self.tree.dim
        L1 = [lagrange_1d(self.nodes1d(t, ax), X[:, ax]) for ax in range(d)]
        out = np.ones((len(X), self.k))
        for nu, m in enumerate(self.multi):
            for ax in range(d):
                out[:, nu] *= L1[ax][:, m[ax]]
        return out

    def lagrange_normal_deriv(self, t, X, N):
        """|X| x k values n . grad l_{t,nu}(x)."""
        d = self.tree.dim
        L1 = [lagrange_1d(self.nodes1d(t, ax), X[:, ax]) for ax in range(d)]
        D1 = [dlagrange_1d(self.nodes1d(t, ax), X[:, ax]) for ax in range(d)]
        out = np.zeros((len(X), self.k))
        for nu, m in enumerate(self.multi):
            for g in range(d):
                term = N[:, g].copy()
                for ax in range(d):
                    term *= D1[ax][:, m[ax]] if ax == g else L1[ax][:, m[ax]]
                out[:, nu] += term
        return out


class ClusterBasis:
    """Definition 3: leaf matrices V[t] (|t| x k_t) for leaves, transfer
    matrices E[t] (k_t x k_parent) for non-root clusters."""

    def __init__(self, tree, leaf, transfer, ranks):
        self.tree, self.leaf, self.transfer, self.rank = tree, leaf, transfer, ranks
        self._full = {}

    def full(self, t):
        """V_t for any cluster via eq. (transfer): V_t|_{t'} = V_{t'} E_{t'}."""
        if t in self._full:
            return self._full[t]
        T = self.tree
        if T.is_leaf(t):
            M = self.leaf[t]
        else:
            M = np.vstack([self.full(c) @ self.transfer[c] for c in T.children[t]])
        self._full[t] = M
        return M


class H2Matrix:
    """Definition 4: block tree, row basis V, column basis W, coupling matrices
    S[(t,s)] for admissible leaves, nearfield N[(t,s)] for inadmissible
    leaves.  Index sets are in the trees' permuted order."""

    def __init__(self, rows, cols, blocks: BlockTree, V: ClusterBasis, W: ClusterBasis, S, N):
        self.rows, self.cols, self.blocks = rows, cols, blocks
        self.V, self.W, self.S, self.N = V, W, S, N

    def block_dense(self, t, s):
        """X|_{t x s} for a block (t,s) of the block tree, permuted order."""
        bt = self.blocks
        k = bt.kind[(t, s)]
        if k == "adm":
            return self.V.full(t) @ self.S[(t, s)] @ self.W.full(s).T
        if k == "inadm":
            return self.N[(t, s)]
        R, C = self.rows, self.cols
        out = np.zeros((R.size(t), C.size(s)))
        for (t2, s2) in bt.children[(t, s)]:
            r0 = R.begin[t2] - R.begin[t]
            c0 = C.begin[s2] - C.begin[s]
            out[r0:r0 + R.size(t2), c0:c0 + C.size(s2)] = self.block_dense(t2, s2)
        return out

    def to_dense_permuted(self):
        return self.block_dense(0, 0)

    def to_dense(self):
        """Dense matrix in the original index order."""
        Dp = self.to_dense_permuted()
        out = np.empty_like(Dp)
        pr, pc = self.rows.perm, self.cols.perm
        out[np.ix_(pr, pc)] = Dp
        return out

    def apply_block(self, t, s, Z):
        """X|_{t x s} Z by recursion over the block tree below (t,s)
        (H2 matrix times k vectors, Section 2)."""
        bt = self.blocks
        k = bt.kind[(t, s)]
        if k == "adm":
            return self.V.full(t) @ (self.S[(t, s)] @ (self.W.full(s).T @ Z))
        if k == "inadm":
            return self.N[(t, s)] @ Z
        R, C = self.rows, self.cols
        out = np.zeros((R.size(t), Z.shape[1]))
        for (t2, s2) in bt.children[(t, s)]:
            r0 = R.begin[t2] - R.begin[t]
            c0 = C.begin[s2] - C.begin[s]
            out[r0:r0 + R.size(t2)] += self.apply_block(t2, s2, Z[c0:c0 + C.size(s2)])
        return out

    def apply_block_adjoint(self, t, s, Z):
        """(X|_{t x s})^* Z."""
        bt = self.blocks
        k = bt.kind[(t, s)]
        if k == "adm":
            return self.W.full(s) @ (self.S[(t, s)].T @ (self.V.full(t).T @ Z))
        if k == "inadm":
            return self.N[(t, s)].T @ Z
        R, C = self.rows, self.cols
        out = np.zeros((C.size(s), Z.shape[1]))
        for (t2, s2) in bt.children[(t, s)]:
            r0 = R.begin[t2] - R.begin[t]
            c0 = C.begin[s2] - C.begin[s]
            out[c0:c0 + C.size(s2)] += self.apply_block_adjoint(t2, s2, Z[r0:r0 + R.size(t2)])
        return out

    def matvec(self, x):
        """y = X x in the original index order."""
        xp = np.asarray(x)[self.cols.perm]
        yp = self.apply_block(0, 0, xp.reshape(len(xp), -1))
        y = np.empty_like(yp)
        y[self.rows.perm] = yp
        return y.reshape(np.shape(x)[:1] + np.shape(x)[1:])

    def rmatvec(self, x):
        """y = X^* x in the original index order (the adjoint recursion)."""
        xp = np.asarray(x)[self.rows.perm]
        yp = self.apply_block_adjoint(0, 0, xp.reshape(len(xp), -1))
        y = np.empty_like(yp)
        y[self.cols.perm] = yp
        return y.reshape((self.cols.n,) + np.shape(x)[1:])

    def storage_words(self):
        w = sum(v.size for v in self.V.leaf.values()) + sum(e.size for e in self.V.transfer.values())
        w += sum(v.size for v in self.W.leaf.values()) + sum(e.size for e in self.W.transfer.values())
        w += sum(s.size for s in self.S.values()) + sum(n.size for n in self.N.values())
        return w


def build_interpolated(tree: ClusterTree, kernel: int, order: int, eta: float,
                       diag: int = DIAG_ZERO, normals=None, cols: ClusterTree | None = None) -> H2Matrix:
    """Operand construction of Section 2 (eq. interpolation, vsw, transfer).
    Rows on `tree`, columns on `cols` (default: the same tree); normals belong
    to the column points; the diagonal rule needs rows and columns on one
    tree."""
    T = tree
    TC = T if cols is None else cols
    if kernel == KERNEL_DLP and normals is None:
        raise ValueError("double layer needs normals")
    if diag != DIAG_ZERO and TC is not T:
        raise ValueError("the diagonal rule needs one tree for rows and columns")
    blocks = BlockTree(T, TC, eta)
    ip = Interp(T, order)
    ipc = ip if TC is T else Interp(TC, order)
    Pp = T.points[T.perm]
    Pc = TC.points[TC.perm]
    Np = None if normals is None else np.asarray(normals, dtype=np.float64)[TC.perm]

    def basis(tr, itp, pts, deriv):
        leaf, E = {}, {}
        for t in range(tr.ncl):
            if tr.is_leaf(t):
                X = pts[tr.begin[t]:tr.end[t]]
                leaf[t] = itp.lagrange_normal_deriv(t, X, Np[tr.begin[t]:tr.end[t]]) if deriv else itp.lagrange(t, X)
            if tr.parent[t] >= 0:
                E[t] = itp.lagrange(int(tr.parent[t]), itp.nodes(t))
        return ClusterBasis(tr, leaf, E, {t: itp.k for t in range(tr.ncl)})

    V = basis(T, ip, Pp, False)
    W = basis(TC, ipc, Pc, kernel == KERNEL_DLP) if (kernel == KERNEL_DLP or TC is not T) else V
    gk = KERNEL_SLP if kernel == KERNEL_DLP else kernel
    S = {}
    for (t, s) in blocks.adm:
        S[(t, s)] = kernel_matrix(gk, ip.nodes(t), ipc.nodes(s))
    N = {}
    for (t, s) in blocks.inadm:
        X = Pp[T.begin[t]:T.end[t]]
        Y = Pc[TC.begin[s]:TC.end[s]]
        ny = None if Np is None else Np[TC.begin[s]:TC.end[s]]
        N[(t, s)] = kernel_matrix(kernel, X, Y, ny)
    if diag == DIAG_ROW_MEAN:
        # row i: mean of g(x_i, x_j) over j != i in the nearfield blocks of row i
        ssum = np.zeros(T.n)
        cnt = np.zeros(T.n)
        for (t, s), M in N.items():
            rows = np.arange(T.begin[t], T.end[t])
            cols = np.arange(T.begin[s], T.end[s])
            off = rows[:, None] != cols[None, :]
            ssum[rows] += np.where(off, M, 0.0).sum(axis=1)
            cnt[rows] += off.sum(axis=1)
        for (t, s), M in N.items():
            if t == s:
                for i in range(T.begin[t], T.end[t]):
                    M[i - T.begin[t], i - T.begin[t]] = ssum[i] / cnt[i] if cnt[i] > 0 else 0.0
    return H2Matrix(T, TC, blocks, V, W, S, N)


def identity_h2(tree: ClusterTree, eta: float, k: int) -> H2Matrix:
    """The identity as an H2 matrix: zero couplings, identity nearfield on the
    diagonal leaf blocks, zero elsewhere; orthonormal leaf bases."""
    T = tree
    blocks = BlockTree(T, T, eta)
    Vleaf, E = {}, {}
    for t in range(T.ncl):
        if T.is_leaf(t):
            Vleaf[t] = np.eye(T.size(t), k)
        if T.parent[t] >= 0:
            E[t] = np.eye(k)
    V = ClusterBasis(T, Vleaf, E, {t: k for t in range(T.ncl)})
    S = {b: np.zeros((k, k)) for b in blocks.adm}
    N = {}
    for (t, s) in blocks.inadm:
        N[(t, s)] = np.eye(T.size(t)) if t == s else np.zeros((T.size(t), T.size(s)))
    return H2Matrix(T, T, blocks, V, V, S, N)
