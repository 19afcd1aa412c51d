"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

For every case the oracle builds its own trees and operands from the same
seeded points.  Checked per leaf block b of the result:
  * the block-relative bound  ||(XY)|_b - C|_b||_2 <= eps ||(XY)|_b||_2  against the
    exact product of the dense operands;
  * the distance to the oracle's result  ||C|_b - C_oracle|_b||_2 <= 2 eps ||(XY)|_b||_2;
  * inadmissible blocks equal the exact product to rounding.
Bases are compared only through block values (they are unique only up to
orthogonal transforms); rank differences are reported, not asserted.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2403_01566_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h2():
    from paper_2403_01566_amd import h2 as mod
    return mod


@pytest.fixture(scope="module")
def ctx(h2):
    return h2.Context(0)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _geometry(case):
    if case == "grid32":
        return dict(P=W.grid2d(32), nrm=None, leaf=32, kern=0, order=3, eta=0.5, diag=0)
    if case == "sphere3":
        P, n = W.icosphere(3)
        return dict(P=P, nrm=n, leaf=64, kern=1, order=3, eta=1.0, diag=1)
    if case == "sphere2dlp":
        P, n = W.icosphere(2)
        return dict(P=P, nrm=n, leaf=20, kern=1, order=2, eta=1.0, diag=1, dlp=True)
    if case == "random2d":
        return dict(P=W.uniform2d(900, 11), nrm=None, leaf=24, kern=0, order=4, eta=0.5, diag=0)
    if case == "cube_dlp":
        P, n = W.cube_surface(8)
        return dict(P=P, nrm=n, leaf=32, kern=2, order=3, eta=1.0, diag=0)
    if case == "tiny":
        return dict(P=W.uniform2d(30, 4), nrm=None, leaf=32, kern=0, order=3, eta=0.5, diag=0)
    raise KeyError(case)


def _build(h2, ctx, case):
    g = _geometry(case)
    T = h2.Tree(ctx, g["P"], g["leaf"])
    A = h2.Matrix.interpolated(ctx, T, T, g["kern"], g["order"], g["eta"], g["diag"], g["nrm"])
    To = O.ClusterTree(g["P"], g["leaf"])
    Ao = O.build_interpolated(To, g["kern"], g["order"], g["eta"], diag=g["diag"], normals=g["nrm"])
    if g.get("dlp"):
        B = h2.Matrix.interpolated(ctx, T, T, 2, g["order"], g["eta"], 0, g["nrm"])
        Bo = O.build_interpolated(To, 2, g["order"], g["eta"], normals=g["nrm"])
    else:
        B, Bo = A, Ao
    return T, A, B, To, Ao, Bo


def _compare(h2, T, Cg, Ao, Bo, Co, eps, prec=0):
    Ex = Ao.to_dense() @ Bo.to_dense()
    Cd = Cg.to_dense(T.n, T.n)
    Cod = Co.to_dense()
    blocks, nadm = Cg.blocks()
    b, e, par, lev = T.clusters()
    perm = T.permutation()
    worst, worst_o = 0.0, 0.0
    scale = np.abs(Ex).max()
    for i, (t, r) in enumerate(blocks):
        I = perm[b[t]:e[t]]
        J = perm[b[r]:e[r]]
        ex = Ex[np.ix_(I, J)]
        cb = Cd[np.ix_(I, J)]
        nn = np.linalg.norm(ex, 2)
        if i < nadm:
            if nn == 0:
                assert np.abs(cb).max() <= 1e-12 * scale
                continue
            rel = np.linalg.norm(ex - cb, 2) / nn
            ro = np.linalg.norm(cb - Cod[np.ix_(I, J)], 2) / nn
            worst, worst_o = max(worst, rel), max(worst_o, ro)
        elif prec == 0:
            # inadmissible blocks are exact up to FP64 rounding
            assert np.abs(ex - cb).max() <= 1e-11 * scale, (t, r)
        else:
            # FP32 bulk: exact product rounded in FP32, still within eps per block
            worst = max(worst, np.linalg.norm(ex - cb, 2) / nn)
    return worst, worst_o


CASES = [
    ("grid32", 1e-4, 0),
    ("sphere3", 1e-6, 0),
    ("sphere3", 1e-4, 1),
    ("sphere2dlp", 1e-4, 0),
    ("random2d", 1e-5, 0),
    ("random2d", 1e-4, 1),
    ("cube_dlp", 1e-4, 0),
    ("cube_dlp", 1e-6, 0),
]


@pytest.mark.parametrize("case,eps,prec", CASES)
def test_parity_against_oracle(h2, ctx, case, eps, prec):
    _say(f"[parity] {case} eps={eps} prec={prec}")
    T, A, B, To, Ao, Bo = _build(h2, ctx, case)
    Cg, st = h2.mul(ctx, A, B, eps, h2.default_options(precision=prec))
    assert st["prec_used"] == prec
    Co, info = O.mul(Ao, Bo, eps)
    worst, worst_o = _compare(h2, T, Cg, Ao, Bo, Co, eps, prec)
    rr, rc = Cg.ranks(T.ncl, T.ncl)
    _say(f"  worst block error {worst:.3e} (eps {eps}), distance to oracle {worst_o:.3e}, "
         f"ranks gpu {rr.max()}/{rc.max()} oracle {max(Co.V.rank.values())}/{max(Co.W.rank.values())}")
    assert worst <= eps
    assert worst_o <= 2 * eps


def test_single_leaf_is_exact_product(h2, ctx):
    _say("[parity] single leaf")
    T, A, B, To, Ao, Bo = _build(h2, ctx, "tiny")
    Cg, st = h2.mul(ctx, A, A, 1e-4)
    ref = Ao.to_dense() @ Ao.to_dense()
    assert np.abs(Cg.to_dense(T.n, T.n) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_repeat_is_bitwise_identical_and_plan_cached(h2, ctx):
    _say("[parity] determinism")
    T, A, B, To, Ao, Bo = _build(h2, ctx, "sphere3")
    C1, s1 = h2.mul(ctx, A, A, 1e-5)
    C2, s2 = h2.mul(ctx, A, A, 1e-5)
    assert s2["t_plan_ms"] == 0.0
    assert np.array_equal(C1.to_dense(T.n, T.n), C2.to_dense(T.n, T.n))
    # a different eps reuses the plan and changes only tolerances
    C3, s3 = h2.mul(ctx, A, A, 1e-3)
    assert s3["t_plan_ms"] == 0.0
    assert C3.info()["rank_max_row"] <= C1.info()["rank_max_row"]


def test_error_paths(h2, ctx):
    _say("[parity] error paths")
    T, A, B, To, Ao, Bo = _build(h2, ctx, "grid32")
    for bad in (0.0, 1.0, -1e-3, float("nan")):
        with pytest.raises(h2.H2Error) as ei:
            h2.mul(ctx, A, A, bad)
        assert ei.value.code == h2.H2_ERR_INVALID_ARG
    T2 = h2.Tree(ctx, W.uniform2d(1024, 3), 32)
    A2 = h2.Matrix.interpolated(ctx, T2, T2, 0, 3, 0.5)
    with pytest.raises(h2.H2Error) as ei:
        h2.mul(ctx, A, A2, 1e-4)
    assert ei.value.code == h2.H2_ERR_INCOMPATIBLE
    with pytest.raises(h2.H2Error) as ei:
        h2.Tree(ctx, np.array([[0.0, np.nan]]), 4)
    assert ei.value.code == h2.H2_ERR_INVALID_ARG
    with pytest.raises(h2.H2Error) as ei:
        h2.Matrix.interpolated(ctx, T, T, 2, 3, 0.5)  # double layer without normals
    assert ei.value.code == h2.H2_ERR_INVALID_ARG
    with pytest.raises(h2.H2Error) as ei:
        h2.mul(ctx, A, A, 1e-4, h2.default_options(max_rank=200))
    assert ei.value.code == h2.H2_ERR_INVALID_ARG


def test_handles_released_in_any_order(h2):
    """Releasing the context before its matrices keeps them usable until released."""
    _say("[parity] handle release order")
    c = h2.Context(0)
    T = h2.Tree(c, W.grid2d(16), 32)
    A = h2.Matrix.interpolated(c, T, T, 0, 3, 0.5)
    C, st = h2.mul(c, A, A, 1e-4)
    c.close()
    assert C.info()["n_adm"] > 0
    d = C.to_dense(T.n, T.n)
    assert np.isfinite(d).all()
    del A, C, T


@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_rectangular_product_three_trees(h2, ctx, eps):
    """X (I x J) Y (J x K) on three different point sets."""
    _say(f"[parity] rectangular eps={eps}")
    pts = [W.uniform2d(700, 31), W.uniform2d(900, 32), W.uniform2d(500, 33)]
    Tg = [h2.Tree(ctx, P, 24) for P in pts]
    To = [O.ClusterTree(P, 24) for P in pts]
    X = h2.Matrix.interpolated(ctx, Tg[0], Tg[1], h2.KERNEL_NEG_LOG, 4, 0.5)
    Y = h2.Matrix.interpolated(ctx, Tg[1], Tg[2], h2.KERNEL_NEG_LOG, 4, 0.5)
    Xo = O.build_interpolated(To[0], O.KERNEL_NEG_LOG, 4, 0.5, cols=To[1])
    Yo = O.build_interpolated(To[1], O.KERNEL_NEG_LOG, 4, 0.5, cols=To[2])
    assert np.abs(X.to_dense(Tg[0].n, Tg[1].n) - Xo.to_dense()).max() <= 1e-12 * np.abs(Xo.to_dense()).max()
    Cg, st = h2.mul(ctx, X, Y, eps)
    Co, info = O.mul(Xo, Yo, eps)
    Ex = Xo.to_dense() @ Yo.to_dense()
    Cd = Cg.to_dense(Tg[0].n, Tg[2].n)
    Cod = Co.to_dense()
    blocks, nadm = Cg.blocks()
    b0, e0, _, _ = Tg[0].clusters()
    b2, e2, _, _ = Tg[2].clusters()
    p0, p2 = Tg[0].permutation(), Tg[2].permutation()
    worst = worst_o = 0.0
    for i, (t, r) in enumerate(blocks):
        I, J = p0[b0[t]:e0[t]], p2[b2[r]:e2[r]]
        ex = Ex[np.ix_(I, J)]
        if i < nadm:
            nn = np.linalg.norm(ex, 2)
            worst = max(worst, np.linalg.norm(ex - Cd[np.ix_(I, J)], 2) / nn)
            worst_o = max(worst_o, np.linalg.norm(Cod[np.ix_(I, J)] - Cd[np.ix_(I, J)], 2) / nn)
        else:
            assert np.abs(ex - Cd[np.ix_(I, J)]).max() <= 1e-11 * np.abs(Ex).max()
    _say(f"  worst block error {worst:.3e} (eps {eps}), distance to oracle {worst_o:.3e}")
    assert worst <= eps and worst_o <= 2 * eps
    x = np.random.default_rng(4).standard_normal(Tg[2].n)
    assert np.abs(Cg.matvec(x) - Cd @ x).max() <= 1e-12 * np.abs(Cd).sum(axis=1).max() * np.abs(x).max()
