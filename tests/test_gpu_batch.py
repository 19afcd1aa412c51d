"""Asynchronous products (batched and served products): each result is the
same, bit for bit, alone (h2_mul) and in a mix of overlapping products on the
context's lanes; the mix holds different operands, precisions and tolerances,
and one operand pair at several tolerances in flight at once."""
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


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _operands(h2, ctx):
    ops = []
    for n, p, seed in [(900, 3, 11), (1500, 4, 12), (2500, 5, 13), (700, 6, 14)]:
        T = h2.Tree(ctx, W.uniform2d(n, seed), 32 if p <= 4 else 64)
        ops.append((T, h2.Matrix.interpolated(ctx, T, T, h2.KERNEL_NEG_LOG, p, 0.5, h2.DIAG_ZERO)))
    P, nrm = W.icosphere(3)
    T = h2.Tree(ctx, P, 64)
    A = h2.Matrix.interpolated(ctx, T, T, h2.KERNEL_LAPLACE_SLP, 3, 1.0, h2.DIAG_ROW_NEARFIELD_MEAN, nrm)
    B = h2.Matrix.interpolated(ctx, T, T, h2.KERNEL_LAPLACE_DLP, 3, 1.0, h2.DIAG_ZERO, nrm)
    return ops, (T, A, B)


def _same(h2, C1, C2, n):
    return np.array_equal(C1.to_dense(n, n), C2.to_dense(n, n))


def test_batch_equals_products_alone(h2):
    ctx = h2.Context(0)
    h2.set_lanes(ctx, 4)
    ops, (Ts, A, B) = _operands(h2, ctx)
    reqs = [(X, X, eps, prec, T.n) for (T, X) in ops for eps, prec in [(1e-4, 0), (1e-6, 0)]]
    reqs += [(A, B, 1e-4, 1, Ts.n), (A, A, 1e-6, 0, Ts.n), (ops[0][1], ops[0][1], 1e-5, 1, ops[0][0].n)]
    _say(f"[batch] {len(reqs)} products alone")
    alone = [h2.mul(ctx, X, Y, eps, h2.default_options(precision=prec)) for X, Y, eps, prec, n in reqs]
    _say("[batch] the same products submitted together")
    jobs = [h2.submit(ctx, X, Y, eps, h2.default_options(precision=prec)) for X, Y, eps, prec, n in reqs]
    got = [j.wait() for j in jobs]
    for (X, Y, eps, prec, n), (Ca, sa), (Cb, sb) in zip(reqs, alone, got):
        assert sb["prec_used"] == sa["prec_used"]
        assert sb["rank_max_row"] == sa["rank_max_row"] and sb["rank_max_col"] == sa["rank_max_col"]
        assert _same(h2, Ca, Cb, n), (n, eps, prec)
    # in reverse order, all in flight before the first wait
    jobs = [h2.submit(ctx, X, Y, eps, h2.default_options(precision=prec)) for X, Y, eps, prec, n in reqs[::-1]]
    for (X, Y, eps, prec, n), (Ca, _), j in zip(reqs[::-1], alone[::-1], jobs):
        Cb, _ = j.wait()
        assert _same(h2, Ca, Cb, n)


def test_one_pair_at_several_tolerances_in_flight(h2):
    """Jobs of one plan share its lane; a new eps waits for the earlier jobs."""
    ctx = h2.Context(0)
    T = h2.Tree(ctx, W.grid2d(32), 32)
    A = h2.Matrix.interpolated(ctx, T, T, h2.KERNEL_NEG_LOG, 3, 0.5)
    epss = [1e-3, 1e-4, 1e-4, 1e-6, 1e-3, 1e-8]
    alone = [h2.mul(ctx, A, A, e)[0] for e in epss]
    jobs = [h2.submit(ctx, A, A, e) for e in epss]
    for Ca, j in zip(alone, jobs):
        Cb, _ = j.wait()
        assert _same(h2, Ca, Cb, T.n)


def test_batched_result_meets_the_bound(h2):
    ctx = h2.Context(0)
    P = W.uniform2d(900, 11)
    T = h2.Tree(ctx, P, 24)
    A = h2.Matrix.interpolated(ctx, T, T, h2.KERNEL_NEG_LOG, 4, 0.5)
    out = h2.mul_batch(ctx, [(A, A)] * 3, [1e-4, 1e-5, 1e-6])
    To = O.ClusterTree(P, 24)
    Ao = O.build_interpolated(To, O.KERNEL_NEG_LOG, 4, 0.5)
    D = Ao.to_dense()
    Ex = D @ D
    perm = T.permutation()
    b, e, _, _ = T.clusters()
    for (C, st), eps in zip(out, [1e-4, 1e-5, 1e-6]):
        Cd = C.to_dense(T.n, T.n)
        blocks, nadm = C.blocks()
        worst = 0.0
        for (t, r) in blocks[:nadm]:
            I, J = perm[b[t]:e[t]], perm[b[r]:e[r]]
            ex = Ex[np.ix_(I, J)]
            nn = np.linalg.norm(ex, 2)
            if nn > 0:
                worst = max(worst, np.linalg.norm(ex - Cd[np.ix_(I, J)], 2) / nn)
        _say(f"[batch] eps {eps}: worst block error {worst:.3e}")
        assert worst <= eps


def test_job_poll_wait_and_errors(h2):
    ctx = h2.Context(0)
    T = h2.Tree(ctx, W.grid2d(16), 32)
    A = h2.Matrix.interpolated(ctx, T, T, h2.KERNEL_NEG_LOG, 3, 0.5)
    j = h2.submit(ctx, A, A, 1e-4)
    with pytest.raises(h2.H2Error) as ei:
        h2.set_lanes(ctx, 2)  # a job is in flight
    assert ei.value.code == h2.H2_ERR_INVALID_ARG
    C, st = j.wait()
    assert j.poll()
    with pytest.raises(h2.H2Error) as ei:
        j.wait()
    assert ei.value.code == h2.H2_ERR_INVALID_ARG
    j.close()
    j2 = h2.submit(ctx, A, A, 1e-4)
    j2.close()  # dropped without wait: waits for its device work
    h2.set_lanes(ctx, 2)
    for bad in (0.0, 1.0):
        with pytest.raises(h2.H2Error) as ei:
            h2.submit(ctx, A, A, bad)
        assert ei.value.code == h2.H2_ERR_INVALID_ARG
    with pytest.raises(h2.H2Error):
        h2.set_lanes(ctx, 9)


def test_graph_replays_match_eager(h2):
    """A product captured as a HIP graph and replayed: every replay equals
    the eager product bit for bit, with other eager work, a tolerance change
    and host synchronisations between the replays."""
    ctx = h2.Context(0)
    P, nrm = W.icosphere(3)
    T = h2.Tree(ctx, P, 64)
    A = h2.Matrix.interpolated(ctx, T, T, h2.KERNEL_LAPLACE_SLP, 3, 1.0, h2.DIAG_ROW_NEARFIELD_MEAN, nrm)
    T2 = h2.Tree(ctx, W.uniform2d(900, 11), 24)
    B = h2.Matrix.interpolated(ctx, T2, T2, h2.KERNEL_NEG_LOG, 4, 0.5)
    ref = {eps: h2.mul(ctx, A, A, eps)[0].to_dense(T.n, T.n) for eps in (1e-4, 1e-6)}
    refB = h2.mul(ctx, B, B, 1e-5)[0].to_dense(T2.n, T2.n)
    g = h2.default_options(graph=1)
    for rep, eps in enumerate([1e-4, 1e-4, 1e-6, 1e-4, 1e-6, 1e-6]):
        C, st = h2.mul(ctx, A, A, eps, g)
        assert np.array_equal(C.to_dense(T.n, T.n), ref[eps]), (rep, eps)
        # eager work on another plan and a matrix-vector product in between
        CB, _ = h2.mul(ctx, B, B, 1e-5)
        assert np.array_equal(CB.to_dense(T2.n, T2.n), refB)
        A.matvec(np.ones(T.n))
    # graph replays of two plans submitted together
    jobs = [h2.submit(ctx, A, A, 1e-6, g), h2.submit(ctx, B, B, 1e-5, h2.default_options(graph=1))]
    CA, _ = jobs[0].wait()
    CB, _ = jobs[1].wait()
    assert np.array_equal(CA.to_dense(T.n, T.n), ref[1e-6])
    assert np.array_equal(CB.to_dense(T2.n, T2.n), refB)


def test_graph_recaptured_after_the_arena_moves(h2):
    """Regression: an FP32-bulk plan replayed from its graph after a larger
    plan has grown the (single) lane's arena, which re-emits the first plan
    against the new workspace: the graph is captured again and the results
    equal the eager ones."""
    ctx = h2.Context(0)
    h2.set_lanes(ctx, 1)
    T1 = h2.Tree(ctx, W.uniform2d(1200, 41), 32)
    A = h2.Matrix.interpolated(ctx, T1, T1, h2.KERNEL_NEG_LOG, 4, 0.5)
    T2 = h2.Tree(ctx, W.uniform2d(6000, 42), 32)
    B = h2.Matrix.interpolated(ctx, T2, T2, h2.KERNEL_NEG_LOG, 4, 0.5)
    f32g = h2.default_options(precision=h2.PREC_FP32_BULK, graph=1)
    refA = h2.mul(ctx, A, A, 1e-4, h2.default_options(precision=h2.PREC_FP32_BULK))[0].to_dense(T1.n, T1.n)
    C, st = h2.mul(ctx, A, A, 1e-4, f32g)               # captured on the small arena
    assert st["prec_used"] == h2.PREC_FP32_BULK
    assert np.array_equal(C.to_dense(T1.n, T1.n), refA)
    h2.mul(ctx, B, B, 1e-4, f32g)                        # the arena grows
    for _ in range(3):
        C, _ = h2.mul(ctx, A, A, 1e-4, f32g)             # re-emitted: a new capture
        assert np.array_equal(C.to_dense(T1.n, T1.n), refA)


def test_plans_rebased_after_the_arena_moves(h2):
    """A cached plan whose lane arena was replaced by a larger one is used
    again: its device descriptors are rebased to the new workspace (the host
    protos of its GEMM steps are gone), then patched to another tolerance.
    Every result equals, bit for bit, the same product in a fresh context."""
    ref = {}
    ctx0 = h2.Context(0)
    h2.set_lanes(ctx0, 1)
    pts = [W.uniform2d(1000, 51), W.uniform2d(5000, 52), W.uniform2d(9000, 53)]

    def ops(ctx):
        out = []
        for P in pts:
            T = h2.Tree(ctx, P, 32)
            out.append((T, h2.Matrix.interpolated(ctx, T, T, h2.KERNEL_NEG_LOG, 4, 0.5)))
        return out

    o0 = ops(ctx0)
    T1, A0 = o0[0]
    for eps in (1e-5, 1e-3):
        ref[eps] = h2.mul(ctx0, A0, A0, eps)[0].to_dense(T1.n, T1.n)
    ctx = h2.Context(0)
    h2.set_lanes(ctx, 1)
    o = ops(ctx)
    A = o[0][1]
    C, _ = h2.mul(ctx, A, A, 1e-5)
    assert np.array_equal(C.to_dense(T1.n, T1.n), ref[1e-5])
    for k, eps in ((1, 1e-3), (2, 1e-5), (1, 1e-5), (2, 1e-3)):
        Bk = o[k][1]
        h2.mul(ctx, Bk, Bk, 1e-4)  # a larger plan on the lane: the arena may move
        C, st = h2.mul(ctx, A, A, eps)
        assert st["t_plan_ms"] == 0.0
        assert np.array_equal(C.to_dense(T1.n, T1.n), ref[eps]), (k, eps)


def _used_device_bytes():
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    f, t = ctypes.c_size_t(), ctypes.c_size_t()
    assert hip.hipMemGetInfo(ctypes.byref(f), ctypes.byref(t)) == 0
    return t.value - f.value


def test_memory_admission_refuses_and_evicts(h2):
    """Admission with a device memory limit: a product that cannot fit is
    refused before anything is allocated and the cached plans are kept; a
    product that fits once idle cached plans are dropped runs after the
    least recently used ones were dropped, and a dropped plan is built again
    on its next use with the same result bit for bit."""
    ctx = h2.Context(0)
    h2.set_lanes(ctx, 1)
    ops = []
    for n, p, seed in ((800, 4, 61), (8000, 4, 62), (8000, 6, 63)):
        T = h2.Tree(ctx, W.uniform2d(n, seed), 32 if p <= 4 else 64)
        ops.append((T, h2.Matrix.interpolated(ctx, T, T, h2.KERNEL_NEG_LOG, p, 0.5)))
    (TA, A), (TB, B), (TD, D) = ops
    refA = h2.mul(ctx, A, A, 1e-6)[0].export()
    refB = h2.mul(ctx, B, B, 1e-6)[0].export()

    def same(C, ref):
        ex = C.export()
        return all(np.array_equal(np.asarray(ex[k]), np.asarray(v)) for k, v in ref.items())

    # no room at all: a new product whose workspace exceeds the lane's arena
    # and everything that could be dropped is refused, the cached plans stay
    h2.set_memory_limit(ctx, 1)
    with pytest.raises(h2.H2Error) as e:
        h2.mul(ctx, D, D, 1e-6)
    assert e.value.code == h2.H2_ERR_OUT_OF_MEMORY
    h2.set_memory_limit(ctx, 0)
    for X, ref in ((A, refA), (B, refB)):
        C, st = h2.mul(ctx, X, X, 1e-6)
        assert st["t_plan_ms"] == 0.0
        assert same(C, ref)
        del C
    # no free room beyond what is in use now: A's result fits only once the
    # idle cached plans (B's, D's) have been dropped
    h2.set_memory_limit(ctx, _used_device_bytes())
    C, st = h2.mul(ctx, A, A, 1e-6)
    assert st["t_plan_ms"] == 0.0
    assert same(C, refA)
    del C
    h2.set_memory_limit(ctx, 0)
    C, st = h2.mul(ctx, B, B, 1e-6)
    assert st["t_plan_ms"] > 0.0  # B's plan was dropped and is built again
    assert same(C, refB)
