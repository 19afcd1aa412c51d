"""Thin ctypes binding of the C ABI in ``include/h2.h`` (argument marshalling
only; every step of the product runs in the HIP library ``libh2mul.so``).

The library must have been built (``python -m paper_2403_01566_amd.build``);
importing this module without it raises ``ImportError`` -- there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.environ.get("H2_LIBRARY", os.path.join(HERE, "libh2mul.so"))

if not os.path.exists(LIBPATH):
    raise ImportError(f"HIP library not built: {LIBPATH} (run python -m paper_2403_01566_amd.build)")
_lib = C.CDLL(LIBPATH)

H2_OK, H2_ERR_INVALID_ARG, H2_ERR_OUT_OF_MEMORY, H2_ERR_DEVICE = 0, 1, 2, 3
H2_ERR_INCOMPATIBLE, H2_ERR_TOO_LARGE, H2_ERR_NOT_CONVERGED = 4, 5, 6
KERNEL_NEG_LOG, KERNEL_LAPLACE_SLP, KERNEL_LAPLACE_DLP = 0, 1, 2
DIAG_ZERO, DIAG_ROW_NEARFIELD_MEAN = 0, 1
PREC_FP64, PREC_FP32_BULK = 0, 1

EXPORTS = [
    "h2_context_create", "h2_context_destroy", "h2_last_error", "h2_build_cluster_tree",
    "h2_tree_permutation", "h2_tree_info", "h2_tree_clusters", "h2_tree_destroy",
    "h2_build_interpolated", "h2_mul_default_options", "h2_mul", "h2_to_dense", "h2_block_dense",
    "h2_matrix_info", "h2_matrix_blocks", "h2_matrix_ranks", "h2_matrix_storage", "h2_matrix_destroy",
    "h2_selftest", "h2_kernel_name", "h2_matvec", "h2_product_error", "h2_block_tree_leaves", "h2_recompress",
    "h2_context_set_lanes", "h2_context_set_memory_limit", "h2_mul_submit", "h2_job_poll", "h2_job_wait", "h2_job_destroy",
    "h2_export_host", "h2_matvec_noalloc",
]
NKERNEL = 13


class MulOptions(C.Structure):
    _fields_ = [("precision", C.c_int), ("theta", C.c_double), ("budget_coarse", C.c_double),
                ("budget_row", C.c_double), ("budget_col", C.c_double), ("max_rank", C.c_int),
                ("coarse_rank", C.c_int), ("timing", C.c_int), ("graph", C.c_int),
                ("jacobi_sweeps", C.c_int), ("chunks", C.c_int)]


class MulStats(C.Structure):
    _fields_ = [("t_phase", C.c_double * 8), ("t_plan_ms", C.c_double), ("bytes_alg", C.c_double),
                ("flops_alg", C.c_double), ("prec_used", C.c_int), ("rank_max_row", C.c_int),
                ("rank_max_col", C.c_int), ("coarse_rank_max", C.c_int), ("n_adm", C.c_int64),
                ("n_inadm", C.c_int64), ("launches", C.c_int64), ("t_kernel", C.c_double * NKERNEL),
                ("launches_kernel", C.c_int64 * NKERNEL), ("units_kernel", C.c_double * NKERNEL),
                ("flops_kernel", C.c_double * NKERNEL), ("bytes_kernel", C.c_double * NKERNEL)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        for f in ("t_phase", "t_kernel", "launches_kernel", "units_kernel", "flops_kernel", "bytes_kernel"):
            d[f] = list(getattr(self, f))
        return d


class HostView(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("n_cols", C.c_int64), ("ncl_rows", C.c_int), ("ncl_cols", C.c_int),
                ("kc", C.c_int), ("n_adm", C.c_int64), ("n_inadm", C.c_int64), ("near_size", C.c_int64),
                ("v_leaf", C.POINTER(C.c_double)), ("v_transfer", C.POINTER(C.c_double)),
                ("w_leaf", C.POINTER(C.c_double)), ("w_transfer", C.POINTER(C.c_double)),
                ("couplings", C.POINTER(C.c_double)), ("near", C.POINTER(C.c_double)),
                ("near_offset", C.POINTER(C.c_int64)), ("rank_row", C.POINTER(C.c_int)),
                ("rank_col", C.POINTER(C.c_int))]


_vp = C.c_void_p
_dp = C.POINTER(C.c_double)
_lp = C.POINTER(C.c_int64)
_ip = C.POINTER(C.c_int)
_sig = {
    "h2_context_create": (C.c_int, [C.c_int, C.POINTER(_vp)]),
    "h2_context_destroy": (None, [_vp]),
    "h2_last_error": (C.c_char_p, []),
    "h2_build_cluster_tree": (C.c_int, [_vp, _dp, C.c_int64, C.c_int, C.c_int, C.POINTER(_vp)]),
    "h2_tree_permutation": (C.c_int, [_vp, _lp]),
    "h2_tree_info": (C.c_int, [_vp, _lp, _ip, _ip, _ip]),
    "h2_tree_clusters": (C.c_int, [_vp, _lp, _lp, _ip, _ip]),
    "h2_tree_destroy": (None, [_vp]),
    "h2_build_interpolated": (C.c_int, [_vp, _vp, _vp, C.c_int, _dp, C.c_int, C.c_double, C.c_int,
                                        C.POINTER(_vp)]),
    "h2_mul_default_options": (None, [C.POINTER(MulOptions)]),
    "h2_mul": (C.c_int, [_vp, _vp, _vp, C.c_double, C.POINTER(MulOptions), C.POINTER(_vp),
                         C.POINTER(MulStats)]),
    "h2_to_dense": (C.c_int, [_vp, _dp, C.c_int64]),
    "h2_block_dense": (C.c_int, [_vp, C.c_int64, _dp]),
    "h2_matrix_info": (C.c_int, [_vp, _lp, _lp, _ip, _ip, _ip]),
    "h2_matrix_blocks": (C.c_int, [_vp, _ip]),
    "h2_matrix_ranks": (C.c_int, [_vp, _ip, _ip]),
    "h2_matrix_storage": (C.c_int, [_vp, _lp]),
    "h2_matrix_destroy": (None, [_vp]),
    "h2_selftest": (C.c_int, [_vp, _dp, C.c_int, _ip]),
    "h2_kernel_name": (C.c_char_p, [C.c_int]),
    "h2_matvec": (C.c_int, [_vp, C.c_int, C.c_int64, _dp, _dp]),
    "h2_matvec_noalloc": (C.c_int, [_vp, C.c_int, C.c_int64, _dp, _dp]),
    "h2_product_error": (C.c_int, [_vp, _vp, _vp, C.c_int, _dp, _dp, _dp]),
    "h2_block_tree_leaves": (C.c_int, [_vp, _vp, C.c_double, _lp, _lp, _ip]),
    "h2_context_set_lanes": (C.c_int, [_vp, C.c_int]),
    "h2_context_set_memory_limit": (C.c_int, [_vp, C.c_uint64]),
    "h2_mul_submit": (C.c_int, [_vp, _vp, _vp, C.c_double, C.POINTER(MulOptions), C.POINTER(_vp)]),
    "h2_job_poll": (C.c_int, [_vp, _ip]),
    "h2_job_wait": (C.c_int, [_vp, C.POINTER(_vp), C.POINTER(MulStats)]),
    "h2_job_destroy": (None, [_vp]),
    "h2_export_host": (C.c_int, [_vp, C.POINTER(HostView)]),
    "h2_recompress": (C.c_int, [_vp, _vp, _vp, C.c_double, _ip, _dp, _dp, _dp, C.c_double, C.POINTER(MulOptions),
                                C.POINTER(_vp), C.POINTER(MulStats)]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class H2Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"h2 status {code}: {msg}")
        self.code = code


def _check(code):
    if code != H2_OK:
        raise H2Error(code, _lib.h2_last_error().decode())


def _dptr(a):
    return a.ctypes.data_as(_dp)


class Context:
    def __init__(self, device: int = 0):
        h = _vp()
        _check(_lib.h2_context_create(device, C.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            _lib.h2_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tree:
    def __init__(self, ctx: Context, points, leaf_size: int):
        pts = np.ascontiguousarray(points, dtype=np.float64)
        h = _vp()
        _check(_lib.h2_build_cluster_tree(ctx.h, _dptr(pts), pts.shape[0], pts.shape[1], leaf_size, C.byref(h)))
        self.h, self.ctx = h, ctx
        n, ncl, depth, nl = C.c_int64(), C.c_int(), C.c_int(), C.c_int()
        _check(_lib.h2_tree_info(h, C.byref(n), C.byref(ncl), C.byref(depth), C.byref(nl)))
        self.n, self.ncl, self.depth, self.nleaves = n.value, ncl.value, depth.value, nl.value

    def permutation(self):
        p = np.empty(self.n, dtype=np.int64)
        _check(_lib.h2_tree_permutation(self.h, p.ctypes.data_as(_lp)))
        return p

    def clusters(self):
        b = np.empty(self.ncl, dtype=np.int64)
        e = np.empty(self.ncl, dtype=np.int64)
        par = np.empty(self.ncl, dtype=np.int32)
        lev = np.empty(self.ncl, dtype=np.int32)
        _check(_lib.h2_tree_clusters(self.h, b.ctypes.data_as(_lp), e.ctypes.data_as(_lp),
                                     par.ctypes.data_as(_ip), lev.ctypes.data_as(_ip)))
        return b, e, par, lev

    def __del__(self):
        try:
            if self.h:
                _lib.h2_tree_destroy(self.h)
                self.h = None
        except Exception:
            pass


class Matrix:
    def __init__(self, h, keep):
        self.h = h
        self._keep = keep  # trees/context kept alive

    @classmethod
    def interpolated(cls, ctx, rows: Tree, cols: Tree, kernel: int, order: int, eta: float,
                     diag: int = DIAG_ZERO, normals=None):
        nrm = None if normals is None else np.ascontiguousarray(normals, dtype=np.float64)
        h = _vp()
        _check(_lib.h2_build_interpolated(ctx.h, rows.h, cols.h, kernel, None if nrm is None else _dptr(nrm),
                                          order, eta, diag, C.byref(h)))
        return cls(h, (ctx, rows, cols))

    def info(self):
        a, i, kc, rr, rc = C.c_int64(), C.c_int64(), C.c_int(), C.c_int(), C.c_int()
        _check(_lib.h2_matrix_info(self.h, C.byref(a), C.byref(i), C.byref(kc), C.byref(rr), C.byref(rc)))
        return {"n_adm": a.value, "n_inadm": i.value, "kcap": kc.value, "rank_max_row": rr.value,
                "rank_max_col": rc.value}

    def blocks(self):
        inf = self.info()
        nb = inf["n_adm"] + inf["n_inadm"]
        p = np.empty(2 * nb, dtype=np.int32)
        _check(_lib.h2_matrix_blocks(self.h, p.ctypes.data_as(_ip)))
        return p.reshape(nb, 2), inf["n_adm"]

    def ranks(self, nrow_clusters, ncol_clusters):
        a = np.empty(nrow_clusters, dtype=np.int32)
        b = np.empty(ncol_clusters, dtype=np.int32)
        _check(_lib.h2_matrix_ranks(self.h, a.ctypes.data_as(_ip), b.ctypes.data_as(_ip)))
        return a, b

    def storage_bytes(self):
        b = C.c_int64()
        _check(_lib.h2_matrix_storage(self.h, C.byref(b)))
        return b.value

    def to_dense(self, nrows, ncols):
        out = np.zeros((nrows, ncols), dtype=np.float64)
        _check(_lib.h2_to_dense(self.h, _dptr(out), ncols))
        return out

    @property
    def shape(self):
        return (self._keep[1].n, self._keep[2].n)

    def matvec(self, x, trans=False):
        """y = M x, or M^T x with trans: x of shape (n,) or (n, nrhs), original order (device product)."""
        xa = np.ascontiguousarray(x, dtype=np.float64)
        x2 = xa.reshape(xa.shape[0], -1)
        nin, nout = (self.shape[0], self.shape[1]) if trans else (self.shape[1], self.shape[0])
        if x2.shape[0] != nin:
            raise ValueError(f"x has {x2.shape[0]} rows, expected {nin}")
        y2 = np.zeros((nout, x2.shape[1]), dtype=np.float64)
        _check(_lib.h2_matvec(self.h, int(bool(trans)), x2.shape[1], _dptr(x2), _dptr(y2)))
        return y2[:, 0] if xa.ndim == 1 else y2

    def export(self):
        """Packed arrays (h2_export_host): dict with v_leaf (n_rows, kc),
        v_transfer (ncl_rows, kc, kc), w_leaf, w_transfer, couplings
        (n_adm, kc, kc), near, near_offset, rank_row, rank_col and the sizes."""
        v = HostView()
        _check(_lib.h2_export_host(self.h, C.byref(v)))
        kc = v.kc
        out = {"kc": kc, "n_adm": v.n_adm, "n_inadm": v.n_inadm}
        arrs = {
            "v_leaf": np.zeros((v.n_rows, kc)), "v_transfer": np.zeros((v.ncl_rows, kc, kc)),
            "w_leaf": np.zeros((v.n_cols, kc)), "w_transfer": np.zeros((v.ncl_cols, kc, kc)),
            "couplings": np.zeros((v.n_adm, kc, kc)), "near": np.zeros(max(v.near_size, 1)),
        }
        for k, a in arrs.items():
            setattr(v, k, a.ctypes.data_as(_dp))
        noff = np.zeros(v.n_inadm + 1, dtype=np.int64)
        rr = np.zeros(v.ncl_rows, dtype=np.int32)
        rc = np.zeros(v.ncl_cols, dtype=np.int32)
        v.near_offset = noff.ctypes.data_as(_lp)
        v.rank_row = rr.ctypes.data_as(_ip)
        v.rank_col = rc.ctypes.data_as(_ip)
        _check(_lib.h2_export_host(self.h, C.byref(v)))
        out.update(arrs)
        out["near"] = arrs["near"][: v.near_size]
        out.update(near_offset=noff, rank_row=rr, rank_col=rc)
        return out

    def matvec_noalloc(self, x, trans=False):
        """matvec through h2_matvec_noalloc (no device allocation: the library's
        static scratch array); same result as matvec."""
        xa = np.ascontiguousarray(x, dtype=np.float64)
        x2 = xa.reshape(xa.shape[0], -1)
        nin, nout = (self.shape[0], self.shape[1]) if trans else (self.shape[1], self.shape[0])
        if x2.shape[0] != nin:
            raise ValueError(f"x has {x2.shape[0]} rows, expected {nin}")
        y2 = np.zeros((nout, x2.shape[1]), dtype=np.float64)
        _check(_lib.h2_matvec_noalloc(self.h, int(bool(trans)), x2.shape[1], _dptr(x2), _dptr(y2)))
        return y2[:, 0] if xa.ndim == 1 else y2

    def block_dense(self, b, m, n):
        out = np.zeros((m, n), dtype=np.float64)
        _check(_lib.h2_block_dense(self.h, int(b), _dptr(out)))
        return out

    def close(self):
        if self.h:
            _lib.h2_matrix_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def selftest(ctx: Context):
    """Errors of every device kernel against host evaluations of their definitions."""
    err = np.zeros(64)
    n = C.c_int()
    _check(_lib.h2_selftest(ctx.h, _dptr(err), 64, C.byref(n)))
    return err[: n.value]


def default_options(**kw) -> MulOptions:
    o = MulOptions()
    _lib.h2_mul_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def mul(ctx: Context, X: Matrix, Y: Matrix, eps: float, options: MulOptions | None = None):
    """C = X Y with the block-relative bound eps.  Returns (C, stats dict)."""
    st = MulStats()
    h = _vp()
    opt = options if options is not None else default_options()
    _check(_lib.h2_mul(ctx.h, X.h, Y.h, float(eps), C.byref(opt), C.byref(h), C.byref(st)))
    return Matrix(h, (ctx,) + X._keep[1:2] + Y._keep[2:3]), st.as_dict()


def product_error(X: Matrix, Y: Matrix, Cm: Matrix | None, z0, iters: int = 10):
    """Power-iteration estimates (||XY - C||_2, ||XY||_2) from the start vector z0."""
    z = np.ascontiguousarray(z0, dtype=np.float64)
    e, nxy = C.c_double(), C.c_double()
    _check(_lib.h2_product_error(X.h, Y.h, None if Cm is None else Cm.h, int(iters), _dptr(z), C.byref(e),
                                 C.byref(nxy)))
    return e.value, nxy.value


class Job:
    """An asynchronous product (h2_mul_submit): poll() / wait() -> (C, stats)."""

    def __init__(self, h, keep):
        self.h, self._keep = h, keep

    def poll(self):
        d = C.c_int()
        _check(_lib.h2_job_poll(self.h, C.byref(d)))
        return bool(d.value)

    def wait(self):
        st = MulStats()
        h = _vp()
        _check(_lib.h2_job_wait(self.h, C.byref(h), C.byref(st)))
        X, Y = self._keep[1], self._keep[2]
        return Matrix(h, (self._keep[0],) + X._keep[1:2] + Y._keep[2:3]), st.as_dict()

    def close(self):
        if self.h:
            _lib.h2_job_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_lanes(ctx: Context, nlanes: int):
    _check(_lib.h2_context_set_lanes(ctx.h, int(nlanes)))


def set_memory_limit(ctx: Context, nbytes: int):
    """Admission limit on device memory in use (0: the whole device)."""
    _check(_lib.h2_context_set_memory_limit(ctx.h, int(nbytes)))


def submit(ctx: Context, X: Matrix, Y: Matrix, eps: float, options: MulOptions | None = None) -> Job:
    """Enqueue C = X Y on one of the context's lanes and return at once."""
    h = _vp()
    opt = options if options is not None else default_options()
    _check(_lib.h2_mul_submit(ctx.h, X.h, Y.h, float(eps), C.byref(opt), C.byref(h)))
    return Job(h, (ctx, X, Y))


def mul_batch(ctx: Context, pairs, eps, options: MulOptions | None = None):
    """Many independent products at once (their device work overlaps on the
    lanes): pairs = [(X, Y), ...], eps a number or one per pair.  Returns
    [(C, stats), ...] in order."""
    epss = list(eps) if hasattr(eps, "__len__") else [eps] * len(pairs)
    jobs = [submit(ctx, X, Y, e, options) for (X, Y), e in zip(pairs, epss)]
    out = [j.wait() for j in jobs]
    for j in jobs:
        j.close()
    return out


def block_tree_leaves(rows: Tree, cols: Tree, eta: float):
    """Leaves of the block tree of (rows, cols, eta): (pairs [n, 2] of cluster
    indices, admissible leaves first; number of admissible leaves)."""
    na, ni = C.c_int64(), C.c_int64()
    _check(_lib.h2_block_tree_leaves(rows.h, cols.h, float(eta), C.byref(na), C.byref(ni), None))
    p = np.empty(2 * (na.value + ni.value), dtype=np.int32)
    _check(_lib.h2_block_tree_leaves(rows.h, cols.h, float(eta), C.byref(na), C.byref(ni), p.ctypes.data_as(_ip)))
    return p.reshape(-1, 2), na.value


def recompress(ctx: Context, rows: Tree, cols: Tree, eta: float, factors, near, eps: float,
               options: MulOptions | None = None):
    """H -> H2 recompression.  factors: one (U_i, Z_i) per admissible leaf in the
    order of block_tree_leaves (U_i |t| x k_i, Z_i |s| x k_i, rows in tree
    order); near: one dense |t| x |s| block per inadmissible leaf.  Returns
    (C, stats dict)."""
    ranks = np.array([np.shape(u)[1] for u, _ in factors], dtype=np.int32)
    cat = lambda blocks: (np.concatenate([np.ascontiguousarray(b, dtype=np.float64).ravel() for b in blocks])
                          if len(blocks) else np.zeros(1))
    U = cat([u for u, _ in factors])
    Z = cat([z for _, z in factors])
    N = cat(list(near))
    st = MulStats()
    h = _vp()
    opt = options if options is not None else default_options()
    _check(_lib.h2_recompress(ctx.h, rows.h, cols.h, float(eta), ranks.ctypes.data_as(_ip), _dptr(U), _dptr(Z),
                              _dptr(N), float(eps), C.byref(opt), C.byref(h), C.byref(st)))
    return Matrix(h, (ctx, rows, cols)), st.as_dict()


def kernel_names():
    """Names of the kernels in the per-kernel statistics (index = kernel id)."""
    return [_lib.h2_kernel_name(i).decode() for i in range(NKERNEL)]
