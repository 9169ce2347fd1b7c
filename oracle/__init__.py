"""FP64 CPU oracle for the 3-D Laplace FMM -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never touches it, and the two share no code.

The C side (``fmm_oracle.c``) holds every step of the method; this module is
ctypes marshalling only.  Formulas and readings are documented in the C file.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_fmm_oracle.so")
_lib = None

_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_u64p = C.POINTER(C.c_uint64)
_i32p = C.POINTER(C.c_int32)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    lib.oracle_set_threads.argtypes = [C.c_int]
    lib.oracle_set_threads.restype = C.c_int
    lib.oracle_direct.argtypes = [C.c_int64, _dp, _dp, C.c_int64, _i64p, _dp, _dp]
    lib.oracle_direct.restype = None
    lib.oracle_num_coeffs.argtypes = [C.c_int]
    lib.oracle_num_coeffs.restype = C.c_int
    lib.oracle_multi_indices.argtypes = [C.c_int, _i32p]
    lib.oracle_taylor_T.argtypes = [C.c_int, _dp, _dp]
    lib.oracle_p2m.argtypes = [C.c_int, C.c_int64, _dp, _dp, _dp, _dp]
    lib.oracle_p2m_dip.argtypes = [C.c_int, C.c_int64, _dp, _dp, _dp, _dp]
    lib.oracle_m2m.argtypes = [C.c_int, _dp, _dp, _dp]
    lib.oracle_m2l.argtypes = [C.c_int, _dp, _dp, _dp]
    lib.oracle_l2l.argtypes = [C.c_int, _dp, _dp, _dp]
    lib.oracle_l2p.argtypes = [C.c_int, _dp, _dp, C.c_int64, _dp, _dp, _dp]
    lib.oracle_multipole_eval.argtypes = [C.c_int, _dp, _dp, C.c_int64, _dp, _dp]
    lib.oracle_plan_create.argtypes = [C.c_int64, _dp, C.c_int, C.c_float, C.c_int]
    lib.oracle_plan_create.restype = C.c_void_p
    lib.oracle_plan_destroy.argtypes = [C.c_void_p]
    lib.oracle_plan_counts.argtypes = [C.c_void_p, _i64p]
    lib.oracle_plan_root.argtypes = [C.c_void_p, _dp]
    lib.oracle_plan_cells.argtypes = [C.c_void_p, _i32p, _u64p, _i64p, _i64p, _i64p, _i32p]
    lib.oracle_plan_pairs.argtypes = [C.c_void_p, _i64p, _i64p]
    lib.oracle_plan_order.argtypes = [C.c_void_p, _i64p, _u64p]
    lib.oracle_fmm_eval.argtypes = [C.c_void_p, C.c_int, _dp, C.c_int, C.c_int64, _i64p, _dp, _dp, _dp, _dp]
    lib.oracle_direct_hessian.argtypes = [C.c_int64, _dp, _dp, C.c_int64, _i64p, _dp]
    lib.oracle_direct_dip.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_int64, _i64p, _dp, _dp]
    lib.oracle_direct_dip.restype = None
    lib.oracle_fmm_eval_dip.argtypes = [C.c_void_p, C.c_int, _dp, _dp, C.c_int, C.c_int64, _i64p, _dp, _dp, _dp]
    _lib = lib
    return lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def set_threads(n: int = 0) -> int:
    """Set the OpenMP thread count (n <= 0 keeps it); returns the count in use."""
    return _load().oracle_set_threads(int(n))


def direct_hessian(points, q, targets=None):
    """Exact Hessian of phi at the targets (FP64), [nt][6] in the order xx, yy, zz, xy, xz, yz."""
    lib = _load()
    pts = _d(points).reshape(-1, 3)
    qq = _d(q).reshape(-1)
    n = pts.shape[0]
    if targets is None:
        nt, tp = n, None
    else:
        tp = np.ascontiguousarray(targets, dtype=np.int64)
        nt = tp.shape[0]
    hess = np.zeros((nt, 6))
    lib.oracle_direct_hessian(n, _ptr(pts, _dp), _ptr(qq, _dp), nt, _ptr(tp, _i64p), _ptr(hess, _dp))
    return hess


def direct(points, q, targets=None):
    """Exact O(N^2) sum in FP64: phi_i = sum_{j!=i} q_j/|x_i-x_j| and its gradient."""
    lib = _load()
    pts = _d(points).reshape(-1, 3)
    qq = _d(q).reshape(-1)
    n = pts.shape[0]
    if targets is None:
        nt, tp = n, None
    else:
        tp = np.ascontiguousarray(targets, dtype=np.int64)
        nt = tp.shape[0]
    phi = np.zeros(nt)
    grad = np.zeros((nt, 3))
    lib.oracle_direct(n, _ptr(pts, _dp), _ptr(qq, _dp), nt, _ptr(tp, _i64p), _ptr(phi, _dp), _ptr(grad, _dp))
    return phi, grad


def direct_dip(points, q, dip, targets=None):
    """Exact potential and gradient of charges q and dipoles dip ([n][3]) at the points
    (or at the target indices): phi_i = sum_j q_j/|d| + g_j.d/|d|^3, d = x_i - x_j."""
    lib = _load()
    pts = _d(points).reshape(-1, 3)
    n = pts.shape[0]
    qq = _d(q).reshape(-1)
    gg = _d(dip).reshape(-1, 3)
    assert qq.shape[0] == n and gg.shape[0] == n
    if targets is None:
        nt, tp = n, None
    else:
        tp = np.ascontiguousarray(targets, dtype=np.int64)
        nt = tp.shape[0]
    phi = np.zeros(nt)
    grad = np.zeros((nt, 3))
    lib.oracle_direct_dip(n, _ptr(pts, _dp), _ptr(qq, _dp), _ptr(gg, _dp), nt if tp is not None else 0,
                          _ptr(tp, _i64p), _ptr(phi, _dp), _ptr(grad, _dp))
    return phi, grad


def direct_targets(sources, q, targets):
    """Field of source charges at separate target positions (FP64):
    phi(y_t) = sum_j q_j / |y_t - x_j| over the sources with x_j != y_t, and its gradient in y_t.
    The direct sum over the union of the two sets, the targets carrying zero charge, taken
    at the target rows: target-target terms vanish and j != i never excludes a source."""
    src = _d(sources).reshape(-1, 3)
    tgt = _d(targets).reshape(-1, 3)
    ns, nt = src.shape[0], tgt.shape[0]
    union = np.concatenate([src, tgt])
    qu = np.concatenate([_d(q).reshape(-1), np.zeros(nt)])
    return direct(union, qu, targets=np.arange(ns, ns + nt, dtype=np.int64))


# ---- single operators (Cartesian Taylor basis) --------------------------------

def num_coeffs(p: int) -> int:
    return _load().oracle_num_coeffs(p)


def multi_indices(p: int) -> np.ndarray:
    out = np.zeros((num_coeffs(p), 3), dtype=np.int32)
    _load().oracle_multi_indices(p, _ptr(out, _i32p))
    return out


def taylor_T(P: int, r) -> np.ndarray:
    out = np.zeros(num_coeffs(P))
    rr = _d(r)
    _load().oracle_taylor_T(P, _ptr(rr, _dp), _ptr(out, _dp))
    return out


def p2m(p, points, q, center):
    pts, qq, c = _d(points).reshape(-1, 3), _d(q).reshape(-1), _d(center)
    out = np.zeros(num_coeffs(p))
    _load().oracle_p2m(p, pts.shape[0], _ptr(pts, _dp), _ptr(qq, _dp), _ptr(c, _dp), _ptr(out, _dp))
    return out


def p2m_dip(p, points, dip, center):
    """Multipole of dipoles dip ([n][3]) at the points: M_a = sum_j sum_i g_ji a_i (x_j - c)^(a - e_i)."""
    pts = _d(points).reshape(-1, 3)
    gg = _d(dip).reshape(-1, 3)
    M = np.zeros(num_coeffs(p))
    _load().oracle_p2m_dip(p, pts.shape[0], _ptr(pts, _dp), _ptr(gg, _dp), _ptr(_d(center), _dp), _ptr(M, _dp))
    return M


def m2m(p, M, d):
    out = np.zeros(num_coeffs(p))
    M, d = _d(M), _d(d)
    _load().oracle_m2m(p, _ptr(M, _dp), _ptr(d, _dp), _ptr(out, _dp))
    return out


def m2l(p, M, D):
    out = np.zeros(num_coeffs(p))
    M, D = _d(M), _d(D)
    _load().oracle_m2l(p, _ptr(M, _dp), _ptr(D, _dp), _ptr(out, _dp))
    return out


def l2l(p, L, d):
    out = np.zeros(num_coeffs(p))
    L, d = _d(L), _d(d)
    _load().oracle_l2l(p, _ptr(L, _dp), _ptr(d, _dp), _ptr(out, _dp))
    return out


def l2p(p, L, center, x):
    L, c, xx = _d(L), _d(center), _d(x).reshape(-1, 3)
    phi = np.zeros(xx.shape[0])
    grad = np.zeros((xx.shape[0], 3))
    _load().oracle_l2p(p, _ptr(L, _dp), _ptr(c, _dp), xx.shape[0], _ptr(xx, _dp), _ptr(phi, _dp), _ptr(grad, _dp))
    return phi, grad


def multipole_eval(p, M, center, x):
    M, c, xx = _d(M), _d(center), _d(x).reshape(-1, 3)
    phi = np.zeros(xx.shape[0])
    _load().oracle_multipole_eval(p, _ptr(M, _dp), _ptr(c, _dp), xx.shape[0], _ptr(xx, _dp), _ptr(phi, _dp))
    return phi


# ---- tree, lists and the full FMM ---------------------------------------------

NEAR, FAR, BOTH = 1, 2, 3


class Plan:
    """Oracle octree + interaction lists for a fixed point set (FP32 values held in FP64)."""

    def __init__(self, points, ncrit: int, theta: float, lists: int = 0):
        lib = _load()
        self.points = _d(points).reshape(-1, 3)
        self.n = self.points.shape[0]
        self.ncrit = int(ncrit)
        self.theta = float(np.float32(theta))
        self.lists = int(lists)
        h = lib.oracle_plan_create(self.n, _ptr(self.points, _dp), self.ncrit, C.c_float(self.theta), self.lists)
        if not h:
            raise ValueError("oracle: invalid plan arguments")
        self._h = h
        cnt = np.zeros(5, dtype=np.int64)
        lib.oracle_plan_counts(h, _ptr(cnt, _i64p))
        self.ncells, self.nm2l, self.np2p, self.k, self.nleaves = (int(v) for v in cnt)
        x0 = np.zeros(3)
        lib.oracle_plan_root(h, _ptr(x0, _dp))
        self.x0 = x0

    def close(self):
        if getattr(self, "_h", None):
            _load().oracle_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def cells(self):
        nc = self.ncells
        level = np.zeros(nc, np.int32)
        prefix = np.zeros(nc, np.uint64)
        start = np.zeros(nc, np.int64)
        count = np.zeros(nc, np.int64)
        parent = np.zeros(nc, np.int64)
        leaf = np.zeros(nc, np.int32)
        _load().oracle_plan_cells(self._h, _ptr(level, _i32p), _ptr(prefix, _u64p), _ptr(start, _i64p),
                                  _ptr(count, _i64p), _ptr(parent, _i64p), _ptr(leaf, _i32p))
        return dict(level=level, prefix=prefix, start=start, count=count, parent=parent, leaf=leaf)

    def pairs(self):
        m2l = np.zeros((self.nm2l, 2), np.int64)
        p2p = np.zeros((self.np2p, 2), np.int64)
        _load().oracle_plan_pairs(self._h, _ptr(m2l, _i64p), _ptr(p2p, _i64p))
        return m2l, p2p

    def order(self):
        order = np.zeros(self.n, np.int64)
        keys = np.zeros(self.n, np.uint64)
        _load().oracle_plan_order(self._h, _ptr(order, _i64p), _ptr(keys, _u64p))
        return order, keys

    def eval_dip(self, q, dip, p: int, mode: int = BOTH, sample=None):
        """FMM potential and gradient (FP64) of charges q and dipoles dip ([n][3]).
        Returns (phi, grad)."""
        qq = _d(q).reshape(-1)
        gg = _d(dip).reshape(-1, 3)
        assert qq.shape[0] == self.n and gg.shape[0] == self.n
        if sample is None:
            ns, sp, nt = 0, None, self.n
        else:
            sp = np.ascontiguousarray(sample, dtype=np.int64)
            ns = nt = sp.shape[0]
        phi = np.zeros(nt)
        grad = np.zeros((nt, 3))
        _load().oracle_fmm_eval_dip(self._h, int(p), _ptr(qq, _dp), _ptr(gg, _dp), int(mode), ns, _ptr(sp, _i64p),
                                    _ptr(phi, _dp), _ptr(grad, _dp), None)
        return phi, grad

    def eval(self, q, p: int, mode: int = BOTH, sample=None, hessian=False):
        """FMM potential and gradient (FP64).  Returns (phi, grad, timing[4]), and the
        Hessian [nt][6] (xx, yy, zz, xy, xz, yz) as a fourth item when hessian=True."""
        qq = _d(q).reshape(-1)
        assert qq.shape[0] == self.n
        if sample is None:
            ns, sp, nt = 0, None, self.n
        else:
            sp = np.ascontiguousarray(sample, dtype=np.int64)
            ns = nt = sp.shape[0]
        phi = np.zeros(nt)
        grad = np.zeros((nt, 3))
        timing = np.zeros(4)
        hess = np.zeros((nt, 6)) if hessian else None
        _load().oracle_fmm_eval(self._h, int(p), _ptr(qq, _dp), int(mode), ns, _ptr(sp, _i64p),
                                _ptr(phi, _dp), _ptr(grad, _dp), _ptr(hess, _dp), _ptr(timing, _dp))
        if hessian:
            return phi, grad, timing, hess
        return phi, grad, timing
