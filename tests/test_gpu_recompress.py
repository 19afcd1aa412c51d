"""GPU H -> H2 recompression (Section 5 on its own) through the C ABI against
the FP64 oracle: the block-relative bound against the input blocks, the
distance to the oracle's result, the copied nearfield, ranks of an input that
already is an H2-matrix, and the error paths."""
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


def _kernel_h(P, leaf, eta, kernel, nrm=None, rank_tol=1e-13):
    """Oracle tree and an H-matrix of the kernel matrix: truncated SVD factors
    of every admissible block, dense inadmissible blocks (tree order)."""
    T = O.ClusterTree(P, leaf)
    K = O.kernel_matrix(kernel, P, P, nrm)
    Kp = K[np.ix_(T.perm, T.perm)]
    bt = O.BlockTree(T, T, eta)
    factors, near = {}, {}
    for (t, s) in bt.adm:
        G = Kp[T.begin[t]:T.end[t], T.begin[s]:T.end[s]]
        U, sv, Vt = np.linalg.svd(G, full_matrices=False)
        k = min(128, max(1, int(np.count_nonzero(sv > rank_tol * sv[0]))))
        factors[(t, s)] = (U[:, :k] * sv[:k], Vt[:k].T)
    for (t, s) in bt.inadm:
        near[(t, s)] = Kp[T.begin[t]:T.end[t], T.begin[s]:T.end[s]].copy()
    return T, factors, near


def _run(h2, ctx, P, leaf, eta, factors, near, eps):
    Tg = h2.Tree(ctx, P, leaf)
    pairs, nadm = h2.block_tree_leaves(Tg, Tg, eta)
    keys = [tuple(int(v) for v in p) for p in pairs]
    assert set(keys[:nadm]) == set(factors) and set(keys[nadm:]) == set(near)
    C, st = h2.recompress(ctx, Tg, Tg, eta, [factors[k] for k in keys[:nadm]], [near[k] for k in keys[nadm:]], eps)
    return Tg, C, st, keys, nadm


def _compare(Tg, C, keys, nadm, factors, near, Co):
    b, e, _, _ = Tg.clusters()
    worst = worst_o = 0.0
    for i, (t, s) in enumerate(keys):
        cb = C.block_dense(i, e[t] - b[t], e[s] - b[s])
        if i < nadm:
            U, Z = factors[(t, s)]
            G = U @ Z.T
            nn = np.linalg.norm(G, 2)
            if nn > 0:
                worst = max(worst, np.linalg.norm(G - cb, 2) / nn)
                worst_o = max(worst_o, np.linalg.norm(Co.block_dense(t, s) - cb, 2) / nn)
        else:
            assert np.array_equal(cb, near[(t, s)])
    return worst, worst_o


CASES = [
    ("grid32_log", 1e-4), ("grid32_log", 1e-8), ("random2d_log", 1e-6), ("sphere3_slp", 1e-5), ("cube8_dlp", 1e-4),
]


def _case(name):
    if name == "grid32_log":
        return W.grid2d(32), 32, 0.5, O.KERNEL_NEG_LOG, None
    if name == "random2d_log":
        return W.uniform2d(900, 11), 24, 0.5, O.KERNEL_NEG_LOG, None
    if name == "sphere3_slp":
        P, n = W.icosphere(3)
        return P, 64, 1.0, O.KERNEL_SLP, None
    if name == "cube8_dlp":
        P, n = W.cube_surface(8)
        return P, 32, 1.0, O.KERNEL_DLP, n
    raise KeyError(name)


@pytest.mark.parametrize("name,eps", CASES)
def test_recompress_against_oracle(h2, ctx, name, eps):
    _say(f"[recompress] {name} eps={eps}")
    P, leaf, eta, kern, nrm = _case(name)
    T, factors, near = _kernel_h(P, leaf, eta, kern, nrm)
    Tg, C, st, keys, nadm = _run(h2, ctx, P, leaf, eta, factors, near, eps)
    Co, info = O.recompress(T, T, eta, factors, near, eps)
    worst, worst_o = _compare(Tg, C, keys, nadm, factors, near, Co)
    _say(f"  worst block error {worst:.3e} (eps {eps}), distance to oracle {worst_o:.3e}, ranks gpu "
         f"{st['rank_max_row']}/{st['rank_max_col']} oracle {max(Co.V.rank.values())}/{max(Co.W.rank.values())}")
    assert worst <= eps
    assert worst_o <= 2 * eps


def test_h2_input_keeps_its_ranks(h2, ctx):
    _say("[recompress] H2 input of rank 9")
    P = W.grid2d(32)
    T = O.ClusterTree(P, 32)
    A = O.build_interpolated(T, O.KERNEL_NEG_LOG, 3, 0.5)
    factors = {b: (A.V.full(b[0]) @ A.S[b], A.W.full(b[1])) for b in A.blocks.adm}
    near = {b: A.N[b] for b in A.blocks.inadm}
    Tg, C, st, keys, nadm = _run(h2, ctx, P, 32, 0.5, factors, near, 1e-10)
    assert st["rank_max_row"] <= 9 and st["rank_max_col"] <= 9
    Co, _ = O.recompress(T, T, 0.5, factors, near, 1e-10)
    worst, worst_o = _compare(Tg, C, keys, nadm, factors, near, Co)
    assert worst <= 1e-10


def test_recompress_matvec_and_dense(h2, ctx):
    """The result is an ordinary matrix handle: its matvec and dense form agree."""
    P, leaf, eta, kern, nrm = _case("grid32_log")
    T, factors, near = _kernel_h(P, leaf, eta, kern, nrm)
    Tg, C, st, keys, nadm = _run(h2, ctx, P, leaf, eta, factors, near, 1e-6)
    D = C.to_dense(Tg.n, Tg.n)
    x = np.random.default_rng(2).standard_normal(Tg.n)
    assert np.abs(C.matvec(x) - D @ x).max() <= 1e-12 * np.abs(D).sum(axis=1).max()


def test_recompress_error_paths(h2, ctx):
    _say("[recompress] error paths")
    P, leaf, eta, kern, nrm = _case("grid32_log")
    T, factors, near = _kernel_h(P, leaf, eta, kern, nrm)
    Tg = h2.Tree(ctx, P, leaf)
    pairs, nadm = h2.block_tree_leaves(Tg, Tg, eta)
    keys = [tuple(int(v) for v in p) for p in pairs]
    f = [factors[k] for k in keys[:nadm]]
    nb = [near[k] for k in keys[nadm:]]
    for bad in (0.0, 1.0, float("nan")):
        with pytest.raises(h2.H2Error) as ei:
            h2.recompress(ctx, Tg, Tg, eta, f, nb, bad)
        assert ei.value.code == h2.H2_ERR_INVALID_ARG
    f_bad = list(f)
    f_bad[0] = (np.zeros((f[0][0].shape[0], 129)), np.zeros((f[0][1].shape[0], 129)))
    with pytest.raises(h2.H2Error) as ei:
        h2.recompress(ctx, Tg, Tg, eta, f_bad, nb, 1e-4)
    assert ei.value.code == h2.H2_ERR_INVALID_ARG
    nb_bad = [x.copy() for x in nb]
    nb_bad[0][0, 0] = np.inf
    with pytest.raises(h2.H2Error) as ei:
        h2.recompress(ctx, Tg, Tg, eta, f, nb_bad, 1e-4)
    assert ei.value.code == h2.H2_ERR_INVALID_ARG
