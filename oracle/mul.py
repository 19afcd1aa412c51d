"""FP64 oracle -- adaptive H2-matrix product with block-relative error control
(test infrastructure only; see oracle/tree.py for the usage rule).

Plain, slow, step-by-step form of the method, in the paper's order:

 1. Basis products P_s = W_{X,s}^* V_{Y,s} (Section 4.1), formed from the
    explicit nested bases.
 2. Exact product with explicit accumulators (Section 3, Definition 5):
    a root accumulator holding the triple (root_J) is routed and split down
    the induced block tree.  Each pending product X|_{t x s} Y|_{s x r} is
    routed by the four cases of Section 3.2 in their order:
      (1) (s,r) admissible in Y:   A_tr += X|_{t x s} V_{Y,s} S_{Y,sr}
      (2) (t,s) admissible in X:   B_tr += Y|_{s x r}^* W_{X,s} S_{X,ts}^*
      (3) either one an inadmissible leaf: N_tr += X|_{t x s} Y|_{s x r}
      (4) otherwise kept as a triple in P_tr.
    Splitting (Section 3.3): A_{t'r'} = A_tr|_{t'} F_{Y,r'}^*,
    B_{t'r'} = B_tr|_{r'} E_{X,t'}^*, N restricted, triples refined to the
    product-tree children (Definition 7).  A cluster without children takes
    itself as its only child with the identity as transfer (the rule of
    eq. block_children).  Splitting continues while P_tr is non-empty or the
    prescribed result block tree still subdivides (t,r).
 3. Coarsening (Section 5.1): for each admissible leaf b of the result tree,
    the exact factors of the induced sub-blocks below it are zero-extended and
    concatenated (exact agglomeration), G_b = U_b Z_b^*.  Then Z_b = Q R,
    condensed G^ = U_b R^*, SVD G^ = U S V^*, truncated at sigma_i > delta_c
    sigma_1 in one step (reading: single-shot truncation; Eckart-Young gives
    the same block-relative bound as the sequential scheme of Remark 13).
 4. Row basis (Section 5.2, 5.3): bottom-up; leaf s: SVD of
    [omega_{s,b}^{-1} G^c_b|_s]_{b in row*(s)}; non-leaf s: SVD of
    [omega^{-1} [G^_{s1,b}; G^_{s2,b}]]; rank = #{sigma > eps_r},
    eps_r = delta_r sqrt(1 - sigma theta); projections G^_{s,b} = V^_s^* [...].
    omega_{s,b} = theta^{(level s - level t)/2} ||G^c_b||_2.
 5. Column basis: the same on the adjoint blocks (r,t).
 6. Coupling matrices S_b = V_t^* G~_b W_r (Section 5.2).
Readings: delta_c = delta_r = delta_w = eps/4 (so the three errors sum to
3/4 eps); sigma = 2 (bisection), theta = 1/(2 sigma); the block norm is the
exact sigma_1 of the coarsening SVD (a lower bound by power iteration would
only tighten the tolerance); blocks with zero norm are left out of the basis
construction; strict comparisons sigma > tau.
"""
from __future__ import annotations

import math
from collections import defaultdict

import numpy as np

from .h2 import ClusterBasis, H2Matrix
from .tree import BlockTree


class MulInfo:
    """Intermediates kept for tests and counters."""

    def __init__(self):
        self.exact = {}          # adm result leaf b -> (U_b, Z_b) exact factors
        self.subblocks = {}      # b -> list of (t, r) induced leaves below/at b
        self.nu = {}             # b -> ||G_b||_2
        self.kappa = {}          # b -> coarsened rank
        self.sigma_coarse = {}   # b -> singular values of G_b
        self.coarse = {}         # b -> (U'_b, Z'_b, sigma_kappa)
        self.row_sv = {}         # cluster -> singular values of weighted matrix
        self.col_sv = {}
        # (cluster s, block b) -> (spectral, Frobenius) norm of the part of
        # the unweighted piece G^_{s,b} that the truncation at s drops,
        # ||(I - V^_s V^_s^*) G^_{s,b}|| (the local errors of Section 5.3)
        self.row_local = {}
        self.col_local = {}
        self.counts = defaultdict(int)
        self.induced_P = []      # (t, r, [s]) for every visited node with P_tr non-empty


def basis_products(X: H2Matrix, Y: H2Matrix):
    """P_s = W_{X,s}^* V_{Y,s} for every cluster s of the middle tree."""
    T = X.cols
    return {s: X.W.full(s).T @ Y.V.full(s) for s in range(T.ncl)}


def _sub(T, parent, child):
    """Offset of child's index range inside parent's."""
    return int(T.begin[child] - T.begin[parent])


def mul(X: H2Matrix, Y: H2Matrix, eps: float, TC: BlockTree | None = None,
        theta: float | None = None, budget=(0.25, 0.25, 0.25), info: MulInfo | None = None):
    if X.cols is not Y.rows:
        raise ValueError("incompatible middle trees")
    if not (0.0 < eps < 1.0):
        raise ValueError("eps must be in (0,1)")
    TI, TJ, TK = X.rows, X.cols, Y.cols
    if TC is None:
        TC = BlockTree(TI, TK, X.blocks.eta)
    info = info if info is not None else MulInfo()
    info.P = basis_products(X, Y)
    bx, by = X.blocks, Y.blocks

    finals = defaultdict(list)   # adm result leaf b -> [(t, r, U, Z)]
    near = {}                    # inadm result leaf b -> dense

    def route(t, r, A, B, N, pend):
        rest = []
        for s in pend:
            if by.is_adm(s, r):                                   # case (1)
                c = X.apply_block(t, s, Y.V.full(s) @ Y.S[(s, r)])
                A = c if A is None else A + c
                info.counts["case1"] += 1
            elif bx.is_adm(t, s):                                 # case (2)
                c = Y.apply_block_adjoint(s, r, X.W.full(s) @ X.S[(t, s)].T)
                B = c if B is None else B + c
                info.counts["case2"] += 1
            elif bx.is_inadm(t, s) or by.is_inadm(s, r):          # case (3)
                c = X.block_dense(t, s) @ Y.block_dense(s, r)
                N = c if N is None else N + c
                info.counts["case3"] += 1
            else:                                                 # case (4)
                rest.append(s)
        return A, B, N, rest

    def finalize(t, r, A, B, N, tc):
        U, Z = [], []
        if A is not None:
            U.append(A)
            Z.append(Y.W.full(r))
        if B is not None:
            U.append(X.V.full(t))
            Z.append(B)
        if N is not None:
            if TI.size(t) <= TK.size(r):
                U.append(np.eye(TI.size(t)))
                Z.append(N.T)
            else:
                U.append(N)
                Z.append(np.eye(TK.size(r)))
        kind, b = tc
        if kind == "node" and TC.is_inadm(*b):
            G = np.zeros((TI.size(t), TK.size(r)))
            for u, z in zip(U, Z):
                G += u @ z.T
            near[b] = G
        else:
            finals[b].append((t, r, U, Z))
        info.counts["final"] += 1

    def visit(t, r, A, B, N, pend, tc):
        info.counts["visit"] += 1
        A, B, N, rest = route(t, r, A, B, N, pend)
        if rest:
            info.induced_P.append((t, r, list(rest)))
        kind, b = tc
        tc_split = kind == "node" and TC.is_split(*b)
        if not rest and not tc_split:
            finalize(t, r, A, B, N, tc)
            return
        ct, cr = TI.chil_plus(t), TK.chil_plus(r)
        for t2 in ct:
            for r2 in cr:
                # refine the triples to the product-tree children (Definition 7)
                pend2 = []
                for s in rest:
                    ys = set(by.children[(s, r)])
                    for (tt, s2) in bx.children[(t, s)]:
                        if tt == t2 and (s2, r2) in ys:
                            pend2.append(s2)
                if t2 == t and r2 == r:
                    # both clusters are leaves: the triples are refined in place
                    visit(t, r, A, B, N, pend2, tc)
                    continue
                A2 = None if A is None else A[_sub(TI, t, t2):_sub(TI, t, t2) + TI.size(t2)]
                if A2 is not None and r2 != r:
                    A2 = A2 @ Y.W.transfer[r2].T
                B2 = None if B is None else B[_sub(TK, r, r2):_sub(TK, r, r2) + TK.size(r2)]
                if B2 is not None and t2 != t:
                    B2 = B2 @ X.V.transfer[t2].T
                N2 = None
                if N is not None:
                    i0, j0 = _sub(TI, t, t2), _sub(TK, r, r2)
                    N2 = N[i0:i0 + TI.size(t2), j0:j0 + TK.size(r2)].copy()
                if kind == "node" and TC.contains(t2, r2) and tc_split:
                    tc2 = ("node", (t2, r2))
                else:
                    tc2 = ("below", b)
                visit(t2, r2, A2, B2, N2, pend2, tc2)

    visit(0, 0, None, None, None, [0], ("node", (0, 0)))
    return _recompress(TI, TK, TC, finals, near, eps, theta, budget, info)


def _recompress(TI, TK, TC, finals, near, eps, theta, budget, info):
    """Steps 3-6 of the header on the exact factors `finals` (admissible result
    leaf b -> list of (t', r', [U], [Z]) pieces of G_b below or at b) and the
    dense nearfield `near`: coarsening, weighted row and column bases,
    couplings (Section 5)."""

    # ---------------- coarsening (Section 5.1) ----------------
    dc, dr, dw = (eps * f for f in budget)
    coarse = {}
    for b in TC.adm:
        t, r = b
        Us, Zs = [], []
        subs = []
        for (t2, r2, U, Z) in finals.get(b, []):
            subs.append((t2, r2))
            i0, j0 = _sub(TI, t, t2), _sub(TK, r, r2)
            for u, z in zip(U, Z):
                ue = np.zeros((TI.size(t), u.shape[1]))
                ue[i0:i0 + u.shape[0]] = u
                ze = np.zeros((TK.size(r), z.shape[1]))
                ze[j0:j0 + z.shape[0]] = z
                Us.append(ue)
                Zs.append(ze)
        Ub = np.hstack(Us) if Us else np.zeros((TI.size(t), 0))
        Zb = np.hstack(Zs) if Zs else np.zeros((TK.size(r), 0))
        info.exact[b] = (Ub, Zb)
        info.subblocks[b] = subs
        if Ub.shape[1] == 0:
            sig = np.zeros(0)
            Uc = np.zeros((TI.size(t), 0))
            Zc = np.zeros((TK.size(r), 0))
        else:
            Q, R = np.linalg.qr(Zb)
            Gh = Ub @ R.T
            Uh, sig, Vh = np.linalg.svd(Gh, full_matrices=False)
            kap = int(np.count_nonzero(sig > dc * sig[0])) if sig[0] > 0 else 0
            Uc = Uh[:, :kap] * sig[:kap]
            Zc = Q @ Vh[:kap].T
        nu = float(sig[0]) if len(sig) else 0.0
        kap = Uc.shape[1]
        info.nu[b], info.kappa[b], info.sigma_coarse[b] = nu, kap, sig
        coarse[b] = (Uc, Zc, sig[:kap])
    info.coarse = coarse

    # ---------------- weighted row / column bases (Sections 5.2, 5.3) ----------------
    sigma_br = max(2, max(len(c) for c in TI.children))
    th = theta if theta is not None else 1.0 / (2.0 * sigma_br)
    if not (0.0 < th * sigma_br < 1.0):
        raise ValueError("theta must satisfy theta < 1/sigma")
    scale = math.sqrt(1.0 - sigma_br * th)

    def build_basis(T, blocks_of, piece, lvl_block, tol, sv_store, local):
        """blocks_of(s): adm result leaves whose cluster on this side is s;
        piece(b): condensed block (rows = that cluster's indices)."""
        leaf, transfer, rank, proj = {}, {}, {}, {}
        anc_blocks = {}
        for s in range(T.ncl):
            acc = []
            for a in T.ancestors_or_self(s):
                acc.extend(blocks_of.get(a, []))
            anc_blocks[s] = [b for b in acc if info.nu[b] > 0.0 and info.kappa[b] > 0]
        order = sorted(range(T.ncl), key=lambda c: -T.level[c])
        for s in order:
            bl = anc_blocks[s]
            cols = []
            if T.is_leaf(s):
                for b in bl:
                    a = lvl_block(b)
                    w = th ** ((T.level[s] - T.level[a]) / 2.0) * info.nu[b]
                    pc = piece(b)[_sub(T, a, s):_sub(T, a, s) + T.size(s)]
                    cols.append(pc / w)
                nrows = T.size(s)
            else:
                ch = T.children[s]
                for b in bl:
                    a = lvl_block(b)
                    w = th ** ((T.level[s] - T.level[a]) / 2.0) * info.nu[b]
                    cols.append(np.vstack([proj[(c, b)] for c in ch]) / w)
                nrows = sum(rank[c] for c in ch)
            G = np.hstack(cols) if cols else np.zeros((nrows, 0))
            if G.shape[1] == 0 or nrows == 0:
                Ul = np.zeros((nrows, 0))
                sv = np.zeros(0)
            else:
                Ul, sv, _ = np.linalg.svd(G, full_matrices=False)
            ks = int(np.count_nonzero(sv > tol))
            sv_store[s] = sv
            Vs = Ul[:, :ks]
            rank[s] = ks
            if T.is_leaf(s):
                leaf[s] = Vs
                for b in bl:
                    a = lvl_block(b)
                    pc = piece(b)[_sub(T, a, s):_sub(T, a, s) + T.size(s)]
                    proj[(s, b)] = Vs.T @ pc
                    d = pc - Vs @ proj[(s, b)]
                    local[(s, b)] = (float(np.linalg.norm(d, 2)) if d.size else 0.0, float(np.linalg.norm(d)))
            else:
                off = 0
                for c in T.children[s]:
                    transfer[c] = Vs[off:off + rank[c]]
                    off += rank[c]
                for b in bl:
                    stacked = np.vstack([proj[(c, b)] for c in T.children[s]])
                    proj[(s, b)] = Vs.T @ stacked
                    d = stacked - Vs @ proj[(s, b)]
                    local[(s, b)] = (float(np.linalg.norm(d, 2)) if d.size else 0.0, float(np.linalg.norm(d)))
        return ClusterBasis(T, leaf, transfer, rank), proj

    row_blocks = defaultdict(list)
    col_blocks = defaultdict(list)
    for b in TC.adm:
        row_blocks[b[0]].append(b)
        col_blocks[b[1]].append(b)
    tol_r = dr * scale
    tol_w = dw * scale
    Vc, projV = build_basis(TI, row_blocks, lambda b: coarse[b][0], lambda b: b[0], tol_r, info.row_sv,
                            info.row_local)
    Wc, projW = build_basis(TK, col_blocks, lambda b: coarse[b][1] * coarse[b][2], lambda b: b[1],
                            tol_w, info.col_sv, info.col_local)

    # ---------------- coupling matrices (Section 5.2) ----------------
    S = {}
    for b in TC.adm:
        t, r = b
        Uc, Zc, _ = coarse[b]
        S[b] = (Vc.full(t).T @ Uc) @ (Wc.full(r).T @ Zc).T
    C = H2Matrix(TI, TK, TC, Vc, Wc, S, near)
    info.counts["adm_blocks"] = len(TC.adm)
    info.counts["inadm_blocks"] = len(TC.inadm)
    info.theta, info.tol_r, info.tol_w, info.delta_c = th, tol_r, tol_w, dc
    info.sigma_br = sigma_br
    return C, info


def recompress(TI, TK, eta, factors, near, eps, theta=None, budget=(0.25, 0.25, 0.25), info=None):
    """H -> H2 recompression with block-relative error (Section 5 on its own):
    an H-matrix on the block tree of (TI, TK, eta), given by factors
    factors[b] = (U_b, Z_b) with G_b = U_b Z_b^* for every admissible leaf b
    and dense blocks near[b] for every inadmissible leaf, becomes an H2-matrix
    with adaptive bases: the truncation of each G_b (the coarsening step with
    a single piece), then the weighted bases and the couplings."""
    if not (0.0 < eps < 1.0):
        raise ValueError("eps must be in (0,1)")
    TC = BlockTree(TI, TK, eta)
    if set(factors) != set(TC.adm) or set(near) != set(TC.inadm):
        raise ValueError("blocks do not match the block tree")
    info = info if info is not None else MulInfo()
    finals = {b: [(b[0], b[1], [np.asarray(factors[b][0], dtype=np.float64)],
                   [np.asarray(factors[b][1], dtype=np.float64)])] for b in TC.adm}
    nearf = {b: np.asarray(near[b], dtype=np.float64) for b in TC.inadm}
    return _recompress(TI, TK, TC, finals, nearf, eps, theta, budget, info)


def block_errors(X: H2Matrix, Y: H2Matrix, C: H2Matrix):
    """Dense check of the block-relative bound on every leaf block of C:
    returns {b: (||(XY)|_b - C|_b||_2, ||(XY)|_b||_2)} (permuted order)."""
    D = X.to_dense_permuted() @ Y.to_dense_permuted()
    TI, TK = C.rows, C.cols
    out = {}
    for b in list(C.blocks.adm) + list(C.blocks.inadm):
        t, r = b
        Ex = D[TI.begin[t]:TI.end[t], TK.begin[r]:TK.end[r]]
        Cb = C.block_dense(t, r)
        out[b] = (float(np.linalg.norm(Ex - Cb, 2)), float(np.linalg.norm(Ex, 2)))
    return out
