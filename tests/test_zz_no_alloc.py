"""The allocation-free entry point h2_matvec_noalloc against h2_matvec.

h2_matvec_noalloc computes y = M x (or M^T x) with every device buffer of the
call in the library's static scratch array (no device allocation); it must
return what h2_matvec returns, bit for bit (the same kernels on the same
launch descriptors).  Two calls in a row, the second on a smaller input,
check that nothing of the first call's contents in the shared array leaks
into the second; a request above the array's size is refused before any
device work, and the next call still works.
"""
import sys

import numpy as np
import pytest

from paper_2403_01566_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_noalloc_matvec_equals_matvec():
    from paper_2403_01566_amd import h2
    ctx = h2.Context(0)
    rng = np.random.default_rng(2403)
    _say("[no-alloc] product on icosphere 3 (adaptive ranks), 3 vectors")
    P, nrm = W.icosphere(3)
    T = h2.Tree(ctx, P, 64)
    A = h2.Matrix.interpolated(ctx, T, T, h2.KERNEL_LAPLACE_SLP, 3, 1.0, h2.DIAG_ROW_NEARFIELD_MEAN, nrm)
    C, _ = h2.mul(ctx, A, A, 1e-6)
    x = rng.standard_normal((T.n, 3))
    y_ref = C.matvec(x)
    y = C.matvec_noalloc(x)
    assert np.array_equal(y, y_ref)
    _say("[no-alloc] second call: smaller input (16 x 16 grid, one vector)")
    T2 = h2.Tree(ctx, W.grid2d(16), 32)
    A2 = h2.Matrix.interpolated(ctx, T2, T2, h2.KERNEL_NEG_LOG, 3, 0.5)
    x2 = rng.standard_normal(T2.n)
    y2 = A2.matvec_noalloc(x2)
    assert np.array_equal(y2, A2.matvec(x2))
    assert np.abs(y2 - A2.to_dense(T2.n, T2.n) @ x2).max() <= 1e-12 * np.abs(y2).max()
    _say("[no-alloc] transposed, and the first matrix again")
    assert np.array_equal(C.matvec_noalloc(x, trans=True), C.matvec(x, trans=True))
    assert np.array_equal(C.matvec_noalloc(x), y_ref)
    _say("[no-alloc] above the scratch size")
    big = rng.standard_normal((T.n, 2000))  # 8 (1280 + 1280) 2000 bytes of vectors alone: 41 MB
    with pytest.raises(h2.H2Error) as ei:
        C.matvec_noalloc(big)
    assert ei.value.code == h2.H2_ERR_TOO_LARGE
    assert np.array_equal(C.matvec_noalloc(x[:, :1]), C.matvec(x[:, :1]))
    y0 = np.zeros_like(x)
    assert h2._lib.h2_matvec_noalloc(C.h, 0, 0, h2._dptr(x), h2._dptr(y0)) == h2.H2_ERR_INVALID_ARG  # nrhs 0
