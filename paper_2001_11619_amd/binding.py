"""ctypes binding of the C ABI in include/rs.h (argument marshalling only)."""

from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBNAME = "librs_mi355x.so"

RS_STATUS = {
    0: "RS_OK", 1: "RS_ERR_ARG", 2: "RS_ERR_STATE", 3: "RS_ERR_ALLOC", 4: "RS_ERR_DEVICE",
    5: "RS_ERR_SINGULAR", 6: "RS_ERR_NOCONV", 7: "RS_ERR_OUT_OF_ROOT",
}


class RSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (RS_STATUS.get(status, str(status)), msg))
        self.status = status
        self.name = RS_STATUS.get(status, str(status))


class Params(ctypes.Structure):
    _fields_ = [
        ("lambda_", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("leaf_size", ctypes.c_int),
        ("n_proxy", ctypes.c_int),
        ("proxy_ratio", ctypes.c_double),
        ("rcond_min", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("refine_tol", ctypes.c_double),
        ("refine_max", ctypes.c_int),
        ("has_root", ctypes.c_int),
        ("root", ctypes.c_double * 3),
        ("solve_graph", ctypes.c_int),
        ("mixed_rcond_min", ctypes.c_double),
        ("apply_shape", ctypes.c_int),
        ("refine_update", ctypes.c_int),
        ("kernel", ctypes.c_int),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_nodes", ctypes.c_int), ("n_holes", ctypes.c_int), ("n_levels", ctypes.c_int),
        ("n_boxes", ctypes.c_int), ("root_skeleton", ctypes.c_int),
        ("max_box_unknowns", ctypes.c_int), ("max_rank", ctypes.c_int),
        ("guard_bumps", ctypes.c_int), ("factor_bytes", ctypes.c_longlong),
        ("flops_id", ctypes.c_double), ("flops_elim", ctypes.c_double),
        ("ms_factor", ctypes.c_double), ("ms_solve", ctypes.c_double),
        ("refine_iters", ctypes.c_int), ("ms_update", ctypes.c_double),
        ("boxes_recomputed", ctypes.c_int), ("apply_config", ctypes.c_int),
        ("apply_ms", ctypes.c_double), ("shape_trials", ctypes.c_int),
    ]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int), ("total_ms", ctypes.c_double)]


_lib = None
# every open context, closed by an exit hook that runs before the HIP runtime
# and any profiler tool tear down (a context released later, from a finalizer
# during interpreter shutdown, would call into a finalized runtime)
_live = weakref.WeakSet()


def close_all():
    """Destroy every open context (also registered to run at interpreter exit)."""
    for s in list(_live):
        s.close()


def library_path() -> str:
    return os.path.join(_HERE, _LIBNAME)


def load_library():
    """Load the built library; raise loudly when it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError("%s is not built; run `python -c 'import __graft_entry__ as g; g.build()'`" % path)
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    dp, ip, vp = P(ctypes.c_double), P(ctypes.c_int), ctypes.c_void_p
    h = ctypes.c_void_p
    lib.rs_default_params.argtypes = [P(Params)]
    lib.rs_default_params.restype = None
    lib.rs_build_tree.argtypes = [P(Params), ctypes.c_int, dp, dp, dp, dp, ip, ctypes.c_int, dp, P(h)]
    lib.rs_factor.argtypes = [h]
    lib.rs_solve.argtypes = [h, ctypes.c_int, dp, dp, dp]
    lib.rs_solve_dev.argtypes = [h, ctypes.c_int, vp, vp]
    lib.rs_update_moved_nodes.argtypes = [h, ctypes.c_int, ip, dp, dp, dp, dp, dp]
    lib.rs_update_geometry.argtypes = [h, ctypes.c_int, dp, dp, dp, dp, ip, ctypes.c_int, dp, ip]
    lib.rs_set_stream.argtypes = [h, vp]
    lib.rs_get_stats.argtypes = [h, P(Stats)]
    lib.rs_get_boxes.argtypes = [h, ctypes.c_int, ip, ip, ip, ip, dp]
    lib.rs_get_skeleton.argtypes = [h, ctypes.c_int, ctypes.c_int, ip, ip]
    lib.rs_apply.argtypes = [h, ctypes.c_int, dp, dp]
    lib.rs_apply_inverse.argtypes = [h, ctypes.c_int, dp, dp]
    lib.rs_apply_f32.argtypes = [h, ctypes.c_int, dp, dp, dp]
    lib.rs_apply_dev_noalloc.argtypes = [h, ctypes.c_int, vp, vp]
    lib.rs_dense_inverse.argtypes = [h, ctypes.c_int, dp, dp]
    lib.rs_evaluate.argtypes = [h, ctypes.c_int, dp, ctypes.c_int, dp, dp]
    lib.rs_factor_batch.argtypes = [P(h), ctypes.c_int]
    lib.rs_update_moved_nodes_batch.argtypes = [P(h), ctypes.c_int, ip, P(ip), P(dp), P(dp), P(dp), P(dp),
                                                P(dp)]
    lib.rs_solve_batch.argtypes = [P(h), ctypes.c_int, ctypes.c_int, P(vp), P(vp)]
    lib.rs_set_kernel_timing.argtypes = [h, ctypes.c_int]
    lib.rs_get_kernel_times.argtypes = [h, ctypes.c_int, P(KernelTime), ip, ctypes.c_int]
    lib.rs_destroy.argtypes = [h]
    lib.rs_destroy.restype = None
    lib.rs_reset_tuning.argtypes = []
    lib.rs_reset_tuning.restype = None
    lib.rs_last_error.argtypes = [h]
    lib.rs_last_error.restype = ctypes.c_char_p
    for name in ("rs_build_tree", "rs_factor", "rs_solve", "rs_solve_dev", "rs_update_moved_nodes",
                 "rs_update_geometry",
                 "rs_set_stream", "rs_get_stats", "rs_get_boxes", "rs_get_skeleton", "rs_apply",
                 "rs_apply_inverse", "rs_apply_dev_noalloc", "rs_apply_f32",
                 "rs_dense_inverse", "rs_evaluate", "rs_set_kernel_timing", "rs_get_kernel_times",
                 "rs_factor_batch", "rs_solve_batch", "rs_update_moved_nodes_batch"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    atexit.register(close_all)
    return lib


def exported_symbols():
    """Names declared in include/rs.h that the loaded library exports."""
    lib = load_library()
    out = []
    for name in ("rs_default_params", "rs_build_tree", "rs_factor", "rs_solve", "rs_solve_dev",
                 "rs_update_moved_nodes", "rs_update_geometry", "rs_set_stream", "rs_get_stats", "rs_get_boxes",
                 "rs_get_skeleton", "rs_apply", "rs_apply_inverse", "rs_dense_inverse", "rs_evaluate",
                 "rs_set_kernel_timing", "rs_get_kernel_times", "rs_factor_batch", "rs_solve_batch",
                 "rs_update_moved_nodes_batch", "rs_apply_dev_noalloc", "rs_apply_f32", "rs_reset_tuning",
                 "rs_destroy",
                 "rs_last_error"):
        if hasattr(lib, name):
            out.append(name)
    return out


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def default_params() -> Params:
    p = Params()
    load_library().rs_default_params(ctypes.byref(p))
    return p


def reset_tuning():
    """Forget every tuned launch shape in the process (rs_reset_tuning)."""
    load_library().rs_reset_tuning()


def factor_batch(solvers):
    """Factor several RSSolver contexts together (one launch per kernel per level)."""
    lib = load_library()
    n = len(solvers)
    arr = (ctypes.c_void_p * n)(*[sv._h.value for sv in solvers])
    st = lib.rs_factor_batch(arr, n)
    if st != 0:
        raise RSError(st, lib.rs_last_error(solvers[0]._h).decode())


def update_moved_nodes_batch(solvers, moves):
    """rs_update_moved_nodes for several contexts in shared launches; moves[i] =
    (idx, xy, normal, weight, curvature[, hole_xy]) for solvers[i]."""
    lib = load_library()
    n = len(solvers)
    keep = []
    idx_p = (ctypes.POINTER(ctypes.c_int) * n)()
    arr = [(ctypes.POINTER(ctypes.c_double) * n)() for _ in range(5)]
    counts = np.zeros(n, np.int32)
    any_hole = False
    for i, mv in enumerate(moves):
        idx = np.ascontiguousarray(mv[0], dtype=np.int32)
        m = idx.size
        vals = [np.ascontiguousarray(mv[1], dtype=np.float64).reshape(m, 2),
                np.ascontiguousarray(mv[2], dtype=np.float64).reshape(m, 2),
                np.ascontiguousarray(mv[3], dtype=np.float64).reshape(m),
                np.ascontiguousarray(mv[4], dtype=np.float64).reshape(m)]
        hole = None
        if len(mv) > 5 and mv[5] is not None:
            hole = np.ascontiguousarray(mv[5], dtype=np.float64).reshape(-1, 2)
            any_hole = True
        vals.append(hole)
        keep.append((idx, vals))
        counts[i] = m
        idx_p[i] = _iptr(idx)
        for k in range(5):
            arr[k][i] = _dptr(vals[k]) if vals[k] is not None else ctypes.POINTER(ctypes.c_double)()
    hs = (ctypes.c_void_p * n)(*[sv._h.value for sv in solvers])
    st = lib.rs_update_moved_nodes_batch(hs, n, _iptr(counts), idx_p, arr[0], arr[1], arr[2], arr[3],
                                         arr[4] if any_hole else None)
    if st != 0:
        raise RSError(st, "; ".join(lib.rs_last_error(sv._h).decode() for sv in solvers))


def solve_batch(solvers, f_devs, x_devs):
    """rs_solve_dev on each context; f_devs / x_devs are device tensors as for solve_dev."""
    lib = load_library()
    n = len(solvers)
    arr = (ctypes.c_void_p * n)(*[sv._h.value for sv in solvers])
    fp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in f_devs])
    xp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in x_devs])
    nrhs = int(f_devs[0].shape[0])
    st = lib.rs_solve_batch(arr, n, nrhs, fp, xp)
    if st != 0:
        raise RSError(st, "batch solve failed")


class RSSolver:
    """One factorization context on the current HIP device."""

    def __init__(self, xy, normal, weight, curvature, curve_id, hole_xy=None, *, tol=None,
                 leaf_size=None, n_proxy=None, proxy_ratio=None, lam=None, rcond_min=None,
                 precision=None, refine_tol=None, refine_max=None, root=None, solve_graph=None,
                 mixed_rcond_min=None, apply_shape=None, refine_update=None, kernel=None):
        lib = load_library()
        self._lib = lib
        self._h = ctypes.c_void_p()
        p = default_params()
        for name, val in (("tol", tol), ("leaf_size", leaf_size), ("n_proxy", n_proxy),
                          ("proxy_ratio", proxy_ratio), ("lambda_", lam), ("rcond_min", rcond_min),
                          ("precision", precision), ("refine_tol", refine_tol),
                          ("refine_max", refine_max), ("solve_graph", solve_graph),
                          ("mixed_rcond_min", mixed_rcond_min), ("apply_shape", apply_shape),
                          ("refine_update", refine_update), ("kernel", kernel)):
            if val is not None:
                setattr(p, name, val)
        if root is not None:
            p.has_root = 1
            for i in range(3):
                p.root[i] = float(root[i])
        self.params = p
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        N = xy.shape[0]
        normal = np.ascontiguousarray(normal, dtype=np.float64).reshape(N, 2)
        weight = np.ascontiguousarray(weight, dtype=np.float64).reshape(N)
        curvature = np.ascontiguousarray(curvature, dtype=np.float64).reshape(N)
        curve_id = np.ascontiguousarray(curve_id, dtype=np.int32).reshape(N)
        if p.kernel == 1:
            # the Laplace Neumann formulation has no augmentation: every curve,
            # holes included, is one boundary without border unknowns
            curve_id = np.zeros(N, dtype=np.int32)
            hole_xy = None
        n_holes = int(curve_id.max()) if N else 0
        hp = None
        if hole_xy is not None and n_holes:
            hole_xy = np.ascontiguousarray(hole_xy, dtype=np.float64).reshape(n_holes, 2)
            hp = _dptr(hole_xy)
        st = lib.rs_build_tree(ctypes.byref(p), N, _dptr(xy), _dptr(normal), _dptr(weight),
                               _dptr(curvature), _iptr(curve_id), n_holes, hp, ctypes.byref(self._h))
        if st != 0:
            raise RSError(st, lib.rs_last_error(None).decode())
        self.n_nodes = N
        self.n_holes = n_holes
        _live.add(self)

    @staticmethod
    def embed_scalar(f):
        """Node values (N,) or (N, ncols) of the Laplace Neumann kernel as the
        library's two-unknowns-per-node layout: f at unknown 2i, 0 at 2i + 1."""
        f = np.asarray(f, dtype=np.float64)
        out = np.zeros((2 * f.shape[0],) + f.shape[1:])
        out[0::2] = f
        return out

    @staticmethod
    def scalar_part(x):
        """The density mu (unknowns 2i) of a Laplace Neumann solution."""
        return np.ascontiguousarray(np.asarray(x)[0::2])

    @classmethod
    def from_geometry(cls, geom, **kw):
        if getattr(geom, "root", None) is not None and "root" not in kw:
            kw["root"] = geom.root
        return cls(geom.xy, geom.normal, geom.weight, geom.curvature, geom.curve_id,
                   geom.hole_xy if geom.n_holes else None, **kw)

    # -- helpers --
    def _check(self, st):
        if st != 0:
            raise RSError(st, self._lib.rs_last_error(self._h).decode())

    @property
    def n_dofs(self):
        return 2 * self.n_nodes

    @property
    def n_system(self):
        return 2 * self.n_nodes + 3 * self.n_holes

    # -- API --
    def factor(self):
        self._check(self._lib.rs_factor(self._h))
        return self

    def solve(self, f, residual: bool = False):
        f = np.asarray(f, dtype=np.float64)
        one = f.ndim == 1
        F = np.asfortranarray(f.reshape(self.n_dofs, -1))
        nrhs = F.shape[1]
        X = np.empty((self.n_system, nrhs), dtype=np.float64, order="F")
        res = np.empty(nrhs) if residual else None
        self._check(self._lib.rs_solve(self._h, nrhs, _dptr(F), _dptr(X),
                                       _dptr(res) if residual else None))
        x = X[:, 0] if one else np.ascontiguousarray(X)
        return (x, res) if residual else x

    def solve_dev(self, f_dev, x_dev):
        """f_dev, x_dev: device tensors laid out column-major ((2N) x nrhs, (2N+3p) x nrhs),
        i.e. torch tensors of shape (nrhs, 2N) and (nrhs, 2N+3p), contiguous, float64."""
        nrhs = int(f_dev.shape[0])
        self._check(self._lib.rs_solve_dev(self._h, nrhs, ctypes.c_void_p(f_dev.data_ptr()),
                                           ctypes.c_void_p(x_dev.data_ptr())))

    def apply(self, x):
        x = np.asarray(x, dtype=np.float64)
        one = x.ndim == 1
        Xf = np.asfortranarray(x.reshape(self.n_system, -1))
        Y = np.empty_like(Xf, order="F")
        self._check(self._lib.rs_apply(self._h, Xf.shape[1], _dptr(Xf), _dptr(Y)))
        return Y[:, 0] if one else np.ascontiguousarray(Y)

    def apply_f32(self, x):
        """(y, bound): the float32 matrix-core image of A x and, per node and
        column, a bound on |y - A x| over the node's two rows (rs_apply_f32)."""
        x = np.asarray(x, dtype=np.float64)
        one = x.ndim == 1
        Xf = np.asfortranarray(x.reshape(self.n_system, -1))
        Y = np.empty_like(Xf, order="F")
        B = np.empty((self.n_nodes, Xf.shape[1]), order="F")
        self._check(self._lib.rs_apply_f32(self._h, Xf.shape[1], _dptr(Xf), _dptr(Y), _dptr(B)))
        if one:
            return Y[:, 0], B[:, 0]
        return np.ascontiguousarray(Y), np.ascontiguousarray(B)

    def apply_dev_noalloc(self, x_dev, y_dev):
        """y = A x on device tensors without allocating (rs_apply_dev_noalloc):
        x_dev, y_dev of shape (ncols, 2N + 3p), contiguous, float64 (the
        column-major layout); enqueued on the context's stream."""
        ncols = int(x_dev.shape[0])
        self._check(self._lib.rs_apply_dev_noalloc(self._h, ncols, ctypes.c_void_p(x_dev.data_ptr()),
                                                   ctypes.c_void_p(y_dev.data_ptr())))

    def apply_inverse(self, b):
        """Factored inverse applied to (2N + 3p) or (2N + 3p, ncols) right-hand
        sides whose border rows may be nonzero."""
        b = np.asarray(b, dtype=np.float64)
        one = b.ndim == 1
        Bf = np.asfortranarray(b.reshape(self.n_system, -1))
        X = np.empty_like(Bf, order="F")
        self._check(self._lib.rs_apply_inverse(self._h, Bf.shape[1], _dptr(Bf), _dptr(X)))
        return X[:, 0] if one else np.ascontiguousarray(X)

    def evaluate(self, targets, x):
        """Velocity D mu + H lambda at target points (M, 2) off the boundary from a
        solution x ((2N + 3p) or (2N + 3p, ncols)); returns (M, 2) or (M, 2, ncols).
        With kernel 1 (Laplace Neumann) the pair is (S mu, d(S mu)/dx)."""
        T = np.ascontiguousarray(targets, dtype=np.float64).reshape(-1, 2)
        one = np.asarray(x).ndim == 1
        X = np.asfortranarray(np.asarray(x, dtype=np.float64).reshape(self.n_system, -1))
        U = np.empty((2 * T.shape[0], X.shape[1]), order="F")
        self._check(self._lib.rs_evaluate(self._h, T.shape[0], _dptr(T), X.shape[1], _dptr(X), _dptr(U)))
        U = np.ascontiguousarray(U).reshape(T.shape[0], 2, X.shape[1])
        return U[:, :, 0] if one else U

    def dense_inverse(self, a):
        """Inverse of a dense square matrix by the library's blocked
        Gauss-Jordan (the root-system inverse), computed on this context's
        device."""
        A = np.ascontiguousarray(a, dtype=np.float64)
        n = A.shape[0]
        if A.shape != (n, n):
            raise ValueError("square matrix expected")
        out = np.empty_like(A)
        self._check(self._lib.rs_dense_inverse(self._h, n, _dptr(A), _dptr(out)))
        return out

    def update_moved_nodes(self, idx, xy, normal, weight, curvature, hole_xy=None):
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        n = idx.size
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(n, 2)
        normal = np.ascontiguousarray(normal, dtype=np.float64).reshape(n, 2)
        weight = np.ascontiguousarray(weight, dtype=np.float64).reshape(n)
        curvature = np.ascontiguousarray(curvature, dtype=np.float64).reshape(n)
        hp = None
        if hole_xy is not None:
            hole_xy = np.ascontiguousarray(hole_xy, dtype=np.float64).reshape(-1, 2)
            hp = _dptr(hole_xy)
        self._check(self._lib.rs_update_moved_nodes(self._h, n, _iptr(idx), _dptr(xy), _dptr(normal),
                                                    _dptr(weight), _dptr(curvature), hp))
        return self

    def update_geometry(self, xy, normal, weight, curvature, curve_id, old_of_new, hole_xy=None):
        """A new boundary (curves inserted or deleted); old_of_new[j] = old index
        of new node j or -1."""
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        N = xy.shape[0]
        normal = np.ascontiguousarray(normal, dtype=np.float64).reshape(N, 2)
        weight = np.ascontiguousarray(weight, dtype=np.float64).reshape(N)
        curvature = np.ascontiguousarray(curvature, dtype=np.float64).reshape(N)
        curve_id = np.ascontiguousarray(curve_id, dtype=np.int32).reshape(N)
        if self.params.kernel == 1:
            curve_id = np.zeros(N, dtype=np.int32)    # no augmentation (as in the constructor)
            hole_xy = None
        oon = np.ascontiguousarray(old_of_new, dtype=np.int32).reshape(N)
        n_holes = int(curve_id.max()) if N else 0
        hp = None
        if hole_xy is not None and n_holes:
            hole_xy = np.ascontiguousarray(hole_xy, dtype=np.float64).reshape(n_holes, 2)
            hp = _dptr(hole_xy)
        self._check(self._lib.rs_update_geometry(self._h, N, _dptr(xy), _dptr(normal), _dptr(weight),
                                                 _dptr(curvature), _iptr(curve_id), n_holes, hp, _iptr(oon)))
        self.n_nodes = N
        self.n_holes = n_holes
        return self

    def set_stream(self, stream_ptr: int):
        self._check(self._lib.rs_set_stream(self._h, ctypes.c_void_p(stream_ptr)))

    def stats(self) -> dict:
        s = Stats()
        self._check(self._lib.rs_get_stats(self._h, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in Stats._fields_}

    def boxes(self) -> dict:
        nb = ctypes.c_int()
        self._lib.rs_get_boxes(self._h, 0, ctypes.byref(nb), None, None, None, None)
        n = nb.value
        lev = np.empty(n, np.int32)
        na = np.empty(n, np.int32)
        rk = np.empty(n, np.int32)
        geo = np.empty(3 * n, np.float64)
        self._check(self._lib.rs_get_boxes(self._h, n, ctypes.byref(nb), _iptr(lev), _iptr(na),
                                           _iptr(rk), _dptr(geo)))
        return {"level": lev, "n": na, "k": rk, "geom": geo.reshape(n, 3)}

    def skeleton(self, box: int) -> np.ndarray:
        ln = ctypes.c_int()
        self._lib.rs_get_skeleton(self._h, box, 0, None, ctypes.byref(ln))
        out = np.empty(max(ln.value, 1), np.int32)
        self._check(self._lib.rs_get_skeleton(self._h, box, out.size, _iptr(out), ctypes.byref(ln)))
        return out[: ln.value].copy()

    def set_kernel_timing(self, enable=True):
        """enable: False/0 off, True/1 per kernel family, 2 per family and tree
        level, 3 the pivoted-QR family only (no host phases)."""
        self._check(self._lib.rs_set_kernel_timing(self._h, int(enable)))

    def kernel_times(self, reset: bool = False) -> dict:
        n = ctypes.c_int()
        self._check(self._lib.rs_get_kernel_times(self._h, 0, None, ctypes.byref(n), 0))
        arr = (KernelTime * max(n.value, 1))()
        self._check(self._lib.rs_get_kernel_times(self._h, n.value, arr, ctypes.byref(n), 1 if reset else 0))
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(n.value)}

    def close(self):
        if self._h:
            self._lib.rs_destroy(self._h)
            self._h = ctypes.c_void_p()
        _live.discard(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
