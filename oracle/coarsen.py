"""FP64 oracle -- the paper's sequential agglomeration (test infrastructure
only; see oracle/tree.py for the usage rule).

Remark 13 (Section 5.1): an n x m block matrix G = (G_ij) is agglomerated
first along every block row, left to right, then the agglomerated rows are
agglomerated top to bottom.  Each step replaces [A B] (or [A; B]) by its best
approximation with relative spectral error eps (singular values sigma_i >
eps * sigma_1 are kept), so the total error is at most
eps (mn + eps m n^2) ||G||_2, below eps_hat ||G||_2 for eps = eps_hat/(2mn).
The factored form G~ = U Z^* keeps every intermediate of size
rows x rank.
"""
from __future__ import annotations

import numpy as np


def _truncate(U, Z, eps):
    """Best approximation of U Z^* with sigma_i > eps sigma_1 kept: (U', Z')."""
    if U.shape[1] == 0:
        return U, Z
    Qz, Rz = np.linalg.qr(Z)
    Uh, sv, Vt = np.linalg.svd(U @ Rz.T, full_matrices=False)
    if sv[0] == 0.0:
        return U[:, :0], Z[:, :0]
    k = int(np.count_nonzero(sv > eps * sv[0]))
    return Uh[:, :k] * sv[:k], Qz @ Vt[:k].T


def agglomerate_sequential(blocks, eps_hat):
    """blocks[i][j]: factor pair (U_ij, Z_ij) of G_ij = U_ij Z_ij^* (n block
    rows, m block columns, consistent sizes).  Returns (U, Z, eps) with
    ||G - U Z^*||_2 <= eps_hat ||G||_2, eps the per-step tolerance used."""
    n, m = len(blocks), len(blocks[0])
    eps = eps_hat / (2.0 * m * n)
    rows = [b[0][0].shape[0] for b in blocks]
    cols = [blk[1].shape[0] for blk in blocks[0]]
    row_factors = []
    for i in range(n):
        U, Z = blocks[i][0]
        Z = np.vstack([Z, np.zeros((sum(cols[1:]), Z.shape[1]))])
        off = cols[0]
        for j in range(1, m):
            Uj, Zj = blocks[i][j]
            Zj = np.vstack([np.zeros((off, Zj.shape[1])), Zj, np.zeros((sum(cols) - off - cols[j], Zj.shape[1]))])
            U, Z = _truncate(np.hstack([U, Uj]), np.hstack([Z, Zj]), eps)
            off += cols[j]
        row_factors.append((U, Z))
    U, Z = row_factors[0]
    U = np.vstack([U, np.zeros((sum(rows[1:]), U.shape[1]))])
    off = rows[0]
    for i in range(1, n):
        Ui, Zi = row_factors[i]
        Ui = np.vstack([np.zeros((off, Ui.shape[1])), Ui, np.zeros((sum(rows) - off - rows[i], Ui.shape[1]))])
        U, Z = _truncate(np.hstack([U, Ui]), np.hstack([Z, Zi]), eps)
        off += rows[i]
    return U, Z, eps
