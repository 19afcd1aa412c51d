"""GPU parity at full size, in the launch configuration of the benchmark (the
product replayed from its HIP graph):
  * icosphere level 5 (n = 20480), single layer squared, leaf 64, eta 1,
    order 4, eps = 1e-6, FP64 (the timed workload);
  * icosphere level 6 (n = 81920), single layer times double layer, eps =
    1e-4, FP32 bulk with FP64 recompression requested.

The oracle cannot form the whole product at this size, so it forms whole
block columns of the exact product instead: for a sampled column cluster r,
(XY)[:, r] = X (Y E_r) with two H2 applications of its own operands (E_r the
identity columns of r).  Every result block (t, r) of that block column is
then checked against the block-relative bound (Section 5.3):
||(XY)|_b - C|_b||_2 <= eps ||(XY)|_b||_2.  The sample holds one leaf cluster
and one cluster a level above, so blocks of several levels, admissible and
inadmissible, are covered.
"""
import sys
import time

import numpy as np
import pytest

import oracle as O
from paper_2403_01566_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    "icosphere5_slp": dict(level=5, kx=1, ky=1, eps=1e-6, prec=0),
    "icosphere6_slp_dlp": dict(level=6, kx=1, ky=2, eps=1e-4, prec=1),
}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("case", sorted(CASES))
def test_sampled_block_columns(case):
    from paper_2403_01566_amd import h2
    c = CASES[case]
    EPS = c["eps"]
    _say(f"[{case}] icosphere {c['level']}, kernels {c['kx']} x {c['ky']}, eps {EPS}, precision {c['prec']}, graph")
    P, nrm = W.icosphere(c["level"])
    ctx = h2.Context(0)
    T = h2.Tree(ctx, P, 64)
    diag = {1: h2.DIAG_ROW_NEARFIELD_MEAN, 2: h2.DIAG_ZERO}
    A = h2.Matrix.interpolated(ctx, T, T, c["kx"], 4, 1.0, diag[c["kx"]], nrm)
    B = h2.Matrix.interpolated(ctx, T, T, c["ky"], 4, 1.0, diag[c["ky"]], nrm) if c["ky"] != c["kx"] else A
    opt = h2.default_options(precision=c["prec"], graph=1)
    t0 = time.time()
    h2.mul(ctx, A, B, EPS, opt)  # captures the graph
    C, st = h2.mul(ctx, A, B, EPS, opt)  # replays it
    _say(f"  gpu products {time.time() - t0:.2f} s (incl. planning), prec_used {st['prec_used']}, "
         f"n_adm {st['n_adm']}, ranks {st['rank_max_row']}/{st['rank_max_col']}")
    # the library may fall back to an FP64 bulk where FP32 rounding reaches the
    # truncation tolerance; the bound below holds either way
    blocks, nadm = C.blocks()
    b, e, par, lev = T.clusters()
    perm = T.permutation()

    t0 = time.time()
    To = O.ClusterTree(P, 64)
    assert np.array_equal(To.perm, perm)
    odiag = {1: O.DIAG_ROW_MEAN, 2: O.DIAG_ZERO}
    okern = {1: O.KERNEL_SLP, 2: O.KERNEL_DLP}
    Ao = O.build_interpolated(To, okern[c["kx"]], 4, 1.0, diag=odiag[c["kx"]], normals=nrm)
    Bo = O.build_interpolated(To, okern[c["ky"]], 4, 1.0, diag=odiag[c["ky"]], normals=nrm) \
        if c["ky"] != c["kx"] else Ao
    _say(f"  oracle operands {time.time() - t0:.1f} s")

    # sampled column clusters, numbered as in the library's tree (same order of points)
    rng = np.random.Generator(np.random.PCG64(2403))
    has_child = np.zeros(len(b), dtype=bool)
    has_child[par[par >= 0]] = True
    leaves = np.flatnonzero(~has_child)
    r_leaf = int(leaves[rng.integers(len(leaves))])
    r_up = int(par[leaves[rng.integers(len(leaves))]])
    checked_adm = checked_inadm = 0
    worst = 0.0
    for r in (r_leaf, r_up):
        t0 = time.time()
        nr = int(e[r] - b[r])
        E = np.zeros((To.n, nr))
        E[b[r] + np.arange(nr), np.arange(nr)] = 1.0
        Z = Ao.apply_block(0, 0, Bo.apply_block(0, 0, E))   # (XY)[:, r], rows in tree order
        mine = [i for i, (t, s) in enumerate(blocks) if s == r]
        for i in mine:
            t = blocks[i][0]
            ex = Z[b[t]:e[t]]
            cb = C.block_dense(i, int(e[t] - b[t]), int(e[r] - b[r]))
            nn = np.linalg.norm(ex, 2)
            err = np.linalg.norm(ex - cb, 2)
            rel = err / nn if nn > 0 else err
            worst = max(worst, rel)
            assert rel <= EPS, (i, t, r, rel)
            if i < nadm:
                checked_adm += 1
            else:
                checked_inadm += 1
        _say(f"  column cluster {r} (|r| = {nr}): {len(mine)} blocks, {time.time() - t0:.1f} s")
    _say(f"  checked {checked_adm} admissible and {checked_inadm} inadmissible blocks, worst {worst:.3e}")
    assert checked_adm > 0 and checked_inadm > 0
