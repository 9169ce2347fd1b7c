"""ctypes binding of the HIP FMM library (include/fmm.h).

Argument marshalling only: every step of the computation runs in the library's
device kernels.  PyTorch provides device memory and the current stream: when the
library is loaded, its workspace allocator (fmm_set_allocator) is bound to
PyTorch's caching allocator, so plan workspace shows in torch.cuda.memory_allocated()
and returns to PyTorch's pool at close().  When the library has not been built,
every entry point raises instead of falling back to anything else.
"""
import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_fmm_hip.so")

FMM_OK, FMM_EINVAL, FMM_ENOMEM, FMM_EDEVICE, FMM_ENONFINITE, FMM_EUNSUPPORTED = range(6)
FMM_PREC_FP32, FMM_PREC_MIXED = 0, 1
FMM_NEAR, FMM_FAR, FMM_ALL = 1, 2, 3
FMM_MAX_LEVELS = 22
FMM_NUM_PHASES = 9
PHASES = ["permute", "p2m", "m2m", "m2l", "l2l", "l2p", "p2p", "combine", "total"]

_STATUS = {FMM_EINVAL: "EINVAL", FMM_ENOMEM: "ENOMEM", FMM_EDEVICE: "EDEVICE",
           FMM_ENONFINITE: "ENONFINITE", FMM_EUNSUPPORTED: "EUNSUPPORTED"}


class FmmStats(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("p", C.c_int32), ("ncrit", C.c_int32), ("precision", C.c_int32), ("max_level", C.c_int32),
        ("theta", C.c_float),
        ("root_exponent", C.c_int32),
        ("root_corner", C.c_double * 3),
        ("ncells", C.c_int64), ("nleaves", C.c_int64),
        ("cells_per_level", C.c_int64 * FMM_MAX_LEVELS),
        ("leaves_per_level", C.c_int64 * FMM_MAX_LEVELS),
        ("m2l_pairs", C.c_int64), ("m2l_pairs_same_level", C.c_int64),
        ("m2l_keys", C.c_int64), ("m2l_keys_same_level", C.c_int64),
        ("m2l_targets", C.c_int64), ("m2l_tiles", C.c_int64), ("m2l_entries", C.c_int64), ("m2l_work_items", C.c_int64),
        ("p2p_pairs", C.c_int64),
        ("p2p_interactions", C.c_int64),
        ("ncoef", C.c_int64), ("ncoef_padded", C.c_int64),
        ("m2l_flops", C.c_double),
        ("p2p_flops", C.c_double),
        ("workspace_bytes", C.c_int64),
        ("m2l_tol", C.c_double), ("m2l_kept_fraction", C.c_double), ("lists", C.c_int64),
        ("p2p_work_items", C.c_int64), ("p2p_split_pieces", C.c_int64),
        ("m2l_pool_pairs", C.c_int64), ("m2l_slots", C.c_int64), ("m2l_slot_tiles", C.c_int64),
        ("svd_tol", C.c_double), ("m2l_svd_rank_mean", C.c_double),
    ]


class FMMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None
_vp = C.c_void_p
_ALLOC_T = C.CFUNCTYPE(_vp, C.c_size_t, _vp, _vp)     # fmm_alloc_fn
_FREE_T = C.CFUNCTYPE(None, _vp, _vp, _vp)            # fmm_free_fn
_installed = None                                     # the callbacks in use (kept alive here)


def load_library():
    """Load the built HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP FMM library not built ({LIB_PATH}); run __graft_entry__.build() "
                           "or python paper_1602_02244_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    lib.fmm_last_error.restype = C.c_char_p
    lib.fmm_last_error.argtypes = []
    lib.fmm_set_allocator.argtypes = [_vp, _vp, _vp]
    lib.fmm_plan.argtypes = [_vp, C.c_int64, C.c_int, C.c_int, C.c_float, C.c_int, _vp, C.POINTER(_vp)]
    lib.fmm_plan_ex.argtypes = [_vp, C.c_int64, C.c_int, C.c_int, C.c_float, C.c_int, C.c_double, C.c_int, _vp,
                                C.POINTER(_vp)]
    lib.fmm_eval.argtypes = [_vp, _vp, _vp, _vp, _vp]
    lib.fmm_eval_ex.argtypes = [_vp, _vp, _vp, _vp, C.c_int, _vp]
    lib.fmm_adjoint.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.fmm_eval_hessian.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
    lib.fmm_adjoint_ex.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.fmm_eval_dipoles.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
    lib.fmm_plan_targets.argtypes = [_vp, C.c_int64, _vp, C.c_int64, C.c_int, C.c_int, C.c_float, C.c_int, _vp,
                                     C.POINTER(_vp)]
    lib.fmm_plan_svd.argtypes = [_vp, C.c_int64, C.c_int, C.c_int, C.c_float, C.c_double, _vp, C.POINTER(_vp)]
    lib.fmm_eval_targets.argtypes = [_vp, _vp, _vp, _vp, _vp]
    lib.fmm_adjoint_targets.argtypes = [_vp] + [_vp] * 8
    lib.fmm_plan_stats.argtypes = [_vp, C.POINTER(FmmStats)]
    lib.fmm_plan_export.argtypes = [_vp] + [_vp] * 8
    lib.fmm_plan_set_timing.argtypes = [_vp, C.c_int]
    lib.fmm_plan_phase_times.argtypes = [_vp, C.POINTER(C.c_float)]
    lib.fmm_plan_destroy.argtypes = [_vp]
    lib.fmm_plan_destroy.restype = None
    for f in ("fmm_set_allocator", "fmm_plan", "fmm_plan_ex", "fmm_plan_svd", "fmm_eval", "fmm_eval_ex", "fmm_adjoint",
              "fmm_eval_hessian", "fmm_eval_dipoles", "fmm_adjoint_ex", "fmm_plan_targets", "fmm_eval_targets",
              "fmm_adjoint_targets", "fmm_plan_stats",
              "fmm_plan_export", "fmm_plan_set_timing", "fmm_plan_phase_times"):
        getattr(lib, f).restype = C.c_int
    _lib = lib
    use_torch_allocator()
    return lib


def set_allocator(alloc=None, free=None):
    """Route the library's device workspace through alloc(nbytes, stream) -> address (0 or
    None: out of memory) and free(address, stream); `stream` is the raw stream handle the
    library passes.  alloc=None gives the library its own device pool back.  Plans keep
    the allocator that was installed when they were created."""
    global _installed
    lib = load_library()
    if alloc is None:
        _check(lib.fmm_set_allocator(None, None, None))
        _installed = None
        return

    def _a(nbytes, stream, ctx):
        try:
            return int(alloc(int(nbytes), int(stream or 0)) or 0) or None
        except Exception:       # an allocation failure of any kind is FMM_ENOMEM for the library
            return None

    def _f(ptr, stream, ctx):
        try:
            free(int(ptr), int(stream or 0))
        except Exception:
            pass

    cbs = (_ALLOC_T(_a), _FREE_T(_f))
    _check(lib.fmm_set_allocator(C.cast(cbs[0], _vp), C.cast(cbs[1], _vp), None))
    # plans made under an earlier allocator still call it: keep every set of callbacks alive
    _all_installed.append(cbs)
    _installed = cbs


_all_installed = []


def _torch_alloc(nbytes, stream):
    return torch.cuda.caching_allocator_alloc(nbytes, stream=stream)


def _torch_free(ptr, stream):
    torch.cuda.caching_allocator_delete(ptr)


def use_torch_allocator():
    """Bind the library's workspace to PyTorch's caching allocator (the default)."""
    set_allocator(_torch_alloc, _torch_free)


def _check(st):
    if st != FMM_OK:
        msg = load_library().fmm_last_error().decode(errors="replace")
        if st == FMM_EINVAL:
            raise ValueError(f"EINVAL: {msg}")
        if st == FMM_ENOMEM:
            raise MemoryError(f"ENOMEM: {msg}")
        raise FMMError(st, msg)


def _dev_ptr(t, name, shape_tail=None, n=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None:
        want = (n,) + tuple(shape_tail or ())
        if tuple(t.shape) != want:
            raise ValueError(f"{name} must have shape {want}, got {tuple(t.shape)}")
    return _vp(t.data_ptr())


def _stream_handle():
    return _vp(torch.cuda.current_stream().cuda_stream)


_PREC = {"fp32": FMM_PREC_FP32, "mixed": FMM_PREC_MIXED}
_LISTS = {"dual": 0, "level-skip": 1}


class FMM:
    """A plan (octree + interaction lists) for a fixed point set on the device.

    points: float32 device tensor [n, 3].  The plan is built on the current stream.
    m2l_tol > 0 selects the variable-order M2L (operator blocks below that relative size
    are left out; FP32 only), 0 the dense operators.  svd_tol > 0 selects SVD-compressed
    operators (singular values of the bound-weighted operator at or below svd_tol times the
    largest dropped; FP32 only, not with m2l_tol or level-skip lists).  lists: "dual" (the
    dual traversal) or "level-skip" (one cell of a same-level pair split at a time).
    """

    def __init__(self, points, ncrit=64, p=10, theta=0.4, precision="fp32", m2l_tol=0.0, lists="dual", svd_tol=0.0):
        lib = load_library()
        if points.dim() != 2 or points.shape[1] != 3:
            raise ValueError("points must have shape [n, 3]")
        self.n = int(points.shape[0])
        if self.n < 1:
            raise ValueError("EINVAL: n must be >= 1")
        ptr = _dev_ptr(points, "points", (3,), self.n)
        if precision not in _PREC:
            raise ValueError(f"precision must be one of {list(_PREC)}")
        self.ncrit, self.p, self.theta, self.precision = int(ncrit), int(p), float(theta), precision
        self.m2l_tol = float(m2l_tol)
        if lists not in _LISTS:
            raise ValueError(f"lists must be one of {list(_LISTS)}")
        self.lists = lists
        self.device = points.device
        self.svd_tol = float(svd_tol)
        h = _vp()
        if self.svd_tol != 0.0:
            if self.m2l_tol != 0.0 or lists != "dual":
                raise ValueError("EINVAL: svd_tol takes the dense dual-traversal plan (m2l_tol = 0, lists = 'dual')")
            _check(lib.fmm_plan_svd(ptr, self.n, self.ncrit, self.p, C.c_float(self.theta), C.c_double(self.svd_tol),
                                    _stream_handle(), C.byref(h)))
        else:
            _check(lib.fmm_plan_ex(ptr, self.n, self.ncrit, self.p, C.c_float(self.theta), _PREC[precision],
                                   C.c_double(self.m2l_tol), _LISTS[lists], _stream_handle(), C.byref(h)))
        self._h = h

    # -------------------------------------------------------------- lifetime
    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            load_library().fmm_plan_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _handle(self):
        if self._h is None:
            raise ValueError("plan is closed")
        return self._h

    # -------------------------------------------------------------- compute
    def eval(self, charges, gradient=True, phases=FMM_ALL, out=None):
        """Potential phi [n] and (optionally) grad phi [n, 3] for charges [n]."""
        q = _dev_ptr(charges, "charges", (), self.n)
        if out is None:
            phi = torch.empty(self.n, device=self.device, dtype=torch.float32)
            grad = torch.empty(self.n, 3, device=self.device, dtype=torch.float32) if gradient else None
        else:
            phi, grad = out
        _check(load_library().fmm_eval_ex(self._handle(), q, _vp(phi.data_ptr()),
                                          _vp(grad.data_ptr()) if grad is not None else None, int(phases),
                                          _stream_handle()))
        return phi, grad

    def eval_hessian(self, charges):
        """(phi [n], grad phi [n, 3], Hessian [n, 6] in the order xx, yy, zz, xy, xz, yz)."""
        q = _dev_ptr(charges, "charges", (), self.n)
        phi = torch.empty(self.n, device=self.device, dtype=torch.float32)
        grad = torch.empty(self.n, 3, device=self.device, dtype=torch.float32)
        hess = torch.empty(self.n, 6, device=self.device, dtype=torch.float32)
        _check(load_library().fmm_eval_hessian(self._handle(), q, _vp(phi.data_ptr()), _vp(grad.data_ptr()),
                                               _vp(hess.data_ptr()), _stream_handle()))
        return phi, grad, hess

    def eval_dipoles(self, charges, dipoles):
        """(phi [n], grad phi [n, 3]) of charges [n] and dipoles [n, 3] at the points."""
        q = _dev_ptr(charges, "charges", (), self.n)
        d = _dev_ptr(dipoles, "dipoles", (3,), self.n)
        phi = torch.empty(self.n, device=self.device, dtype=torch.float32)
        grad = torch.empty(self.n, 3, device=self.device, dtype=torch.float32)
        _check(load_library().fmm_eval_dipoles(self._handle(), q, d, _vp(phi.data_ptr()), _vp(grad.data_ptr()),
                                               _stream_handle()))
        return phi, grad

    def adjoint(self, charges, dL_dphi, gradient_fwd=None, want_dq=True, want_dx=True, dL_dgrad=None):
        """(dL/dq [n], dL/dx [n, 3]) of L(phi, grad phi) with w = dL_dphi and, when given,
        g = dL_dgrad [n, 3], for the frozen plan."""
        if dL_dgrad is not None:
            q = _dev_ptr(charges, "charges", (), self.n)
            w = _dev_ptr(dL_dphi, "dL_dphi", (), self.n)
            g = _dev_ptr(dL_dgrad, "dL_dgrad", (3,), self.n)
            dq = torch.empty(self.n, device=self.device, dtype=torch.float32) if want_dq else None
            dx = torch.empty(self.n, 3, device=self.device, dtype=torch.float32) if want_dx else None
            _check(load_library().fmm_adjoint_ex(self._handle(), q, w, g,
                                                 _vp(dq.data_ptr()) if dq is not None else None,
                                                 _vp(dx.data_ptr()) if dx is not None else None, _stream_handle()))
            return dq, dx
        q = _dev_ptr(charges, "charges", (), self.n)
        w = _dev_ptr(dL_dphi, "dL_dphi", (), self.n)
        gf = _dev_ptr(gradient_fwd, "gradient_fwd", (3,), self.n) if gradient_fwd is not None else None
        dq = torch.empty(self.n, device=self.device, dtype=torch.float32) if want_dq else None
        dx = torch.empty(self.n, 3, device=self.device, dtype=torch.float32) if want_dx else None
        _check(load_library().fmm_adjoint(self._handle(), q, gf, w,
                                          _vp(dq.data_ptr()) if dq is not None else None,
                                          _vp(dx.data_ptr()) if dx is not None else None, _stream_handle()))
        return dq, dx

    # -------------------------------------------------------------- introspection
    def stats(self):
        st = FmmStats()
        _check(load_library().fmm_plan_stats(self._handle(), C.byref(st)))
        out = {}
        for name, _ in FmmStats._fields_:
            v = getattr(st, name)
            out[name] = list(v) if not isinstance(v, (int, float)) else v
        out["cells_per_level"] = out["cells_per_level"][: st.max_level + 1]
        out["leaves_per_level"] = out["leaves_per_level"][: st.max_level + 1]
        return out

    def export(self):
        """Tree and lists as host numpy arrays (for checks against an independent build)."""
        st = self.stats()
        nc, nm, npp = st["ncells"], st["m2l_pairs"], st["p2p_pairs"]
        level = np.zeros(nc, np.int32)
        prefix = np.zeros(nc, np.uint64)
        start = np.zeros(nc, np.int64)
        count = np.zeros(nc, np.int64)
        leaf = np.zeros(nc, np.int32)
        order = np.zeros(self.n, np.int64)
        m2l = np.zeros((nm, 2), np.int64)
        p2p = np.zeros((npp, 2), np.int64)
        ptr = lambda a: _vp(a.ctypes.data)
        _check(load_library().fmm_plan_export(self._handle(), ptr(level), ptr(prefix), ptr(start), ptr(count),
                                              ptr(leaf), ptr(order), ptr(m2l), ptr(p2p)))
        return dict(level=level, prefix=prefix, start=start, count=count, leaf=leaf, order=order, m2l=m2l, p2p=p2p)

    def set_timing(self, enable=True):
        _check(load_library().fmm_plan_set_timing(self._handle(), 1 if enable else 0))

    def phase_times(self):
        ms = (C.c_float * FMM_NUM_PHASES)()
        _check(load_library().fmm_plan_phase_times(self._handle(), ms))
        return dict(zip(PHASES, [float(v) for v in ms]))


def _opt_ptr(t):
    return _vp(t.data_ptr()) if t is not None else None


class FMMTargets(FMM):
    """A plan for separate sources [ns, 3] and targets [nt, 3]: the fields of the source
    charges at the targets (a target at a source's position skips that source).

    The octree and lists are those of the union point set (sources first); the targets carry
    no charge.  Only eval / adjoint below apply; the introspection calls see the union.
    """

    def __init__(self, sources, targets, ncrit=64, p=10, theta=0.4, precision="fp32"):
        lib = load_library()
        for name, t in (("sources", sources), ("targets", targets)):
            if t.dim() != 2 or t.shape[1] != 3:
                raise ValueError(f"{name} must have shape [n, 3]")
        self.ns, self.nt = int(sources.shape[0]), int(targets.shape[0])
        if self.ns < 1 or self.nt < 1:
            raise ValueError("EINVAL: ns and nt must be >= 1")
        ps = _dev_ptr(sources, "sources", (3,), self.ns)
        pt = _dev_ptr(targets, "targets", (3,), self.nt)
        if precision not in _PREC:
            raise ValueError(f"precision must be one of {list(_PREC)}")
        self.n = self.ns + self.nt
        self.ncrit, self.p, self.theta, self.precision = int(ncrit), int(p), float(theta), precision
        self.m2l_tol, self.lists = 0.0, "dual"
        self.device = sources.device
        h = _vp()
        _check(lib.fmm_plan_targets(ps, self.ns, pt, self.nt, self.ncrit, self.p, C.c_float(self.theta),
                                    _PREC[precision], _stream_handle(), C.byref(h)))
        self._h = h

    def eval(self, charges, gradient=True):
        """Potential [nt] and (optionally) its gradient [nt, 3] at the targets."""
        q = _dev_ptr(charges, "charges", (), self.ns)
        phi = torch.empty(self.nt, device=self.device, dtype=torch.float32)
        grad = torch.empty(self.nt, 3, device=self.device, dtype=torch.float32) if gradient else None
        _check(load_library().fmm_eval_targets(self._handle(), q, _vp(phi.data_ptr()), _opt_ptr(grad),
                                               _stream_handle()))
        return phi, grad

    def eval_hessian(self, charges):
        raise ValueError("EINVAL: the Hessian at separate targets is not provided")

    def adjoint(self, charges, dL_dphi, gradient_fwd=None, dL_dgrad=None, want_dq=True, want_dx_src=True,
                want_dx_tgt=True):
        """(dL/dq [ns], dL/dx_src [ns, 3], dL/dx_tgt [nt, 3]) for L(phi, grad phi) at the
        targets, with w = dL_dphi [nt] and, when given, g = dL_dgrad [nt, 3]."""
        q = _dev_ptr(charges, "charges", (), self.ns)
        w = _dev_ptr(dL_dphi, "dL_dphi", (), self.nt)
        gf = _dev_ptr(gradient_fwd, "gradient_fwd", (3,), self.nt) if gradient_fwd is not None else None
        g = _dev_ptr(dL_dgrad, "dL_dgrad", (3,), self.nt) if dL_dgrad is not None else None
        dq = torch.empty(self.ns, device=self.device, dtype=torch.float32) if want_dq else None
        dxs = torch.empty(self.ns, 3, device=self.device, dtype=torch.float32) if want_dx_src else None
        dxt = torch.empty(self.nt, 3, device=self.device, dtype=torch.float32) if want_dx_tgt else None
        _check(load_library().fmm_adjoint_targets(self._handle(), q, gf, w, g, _opt_ptr(dq), _opt_ptr(dxs),
                                                  _opt_ptr(dxt), _stream_handle()))
        return dq, dxs, dxt


class FMMTargetsFunction(torch.autograd.Function):
    """phi_t, grad_phi_t = FMM(sources, charges -> targets); backward through the adjoint on
    a rebuilt plan."""

    @staticmethod
    def forward(ctx, sources, charges, targets, ncrit, p, theta, precision):
        plan = FMMTargets(sources.detach(), targets.detach(), ncrit, p, theta, precision)
        phi, grad = plan.eval(charges.detach().contiguous())
        plan.close()
        ctx.save_for_backward(sources, charges, targets, grad)
        ctx.cfg = (ncrit, p, theta, precision)
        return phi, grad

    @staticmethod
    def backward(ctx, g_phi, g_grad):
        sources, charges, targets, grad = ctx.saved_tensors
        need_xs, need_q, need_xt = ctx.needs_input_grad[0], ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        through_grad = g_grad is not None and bool(torch.count_nonzero(g_grad))
        none = (None,) * 4
        if (g_phi is None and not through_grad) or not (need_xs or need_q or need_xt):
            return (None, None, None) + none
        if g_phi is None:
            g_phi = torch.zeros(targets.shape[0], device=targets.device, dtype=torch.float32)
        plan = FMMTargets(sources.detach(), targets.detach(), *ctx.cfg)
        dq, dxs, dxt = plan.adjoint(charges.detach().contiguous(), g_phi.contiguous(),
                                    gradient_fwd=None if through_grad else grad,
                                    dL_dgrad=g_grad.contiguous() if through_grad else None, want_dq=need_q,
                                    want_dx_src=need_xs, want_dx_tgt=need_xt)
        plan.close()
        return (dxs, dq, dxt) + none


def fmm_apply_targets(sources, charges, targets, ncrit=64, p=10, theta=0.4, precision="fp32"):
    """Differentiable FMM at separate targets: returns (phi [nt], grad phi [nt, 3])."""
    return FMMTargetsFunction.apply(sources, charges, targets, ncrit, p, theta, precision)


class FMMFunction(torch.autograd.Function):
    """phi, grad_phi = FMM(points, charges); backward gives dL/dq and dL/dx through the
    adjoint FMM.  The plan is rebuilt in backward (recomputed, not stored)."""

    @staticmethod
    def forward(ctx, points, charges, ncrit, p, theta, precision):
        plan = FMM(points.detach(), ncrit, p, theta, precision)
        phi, grad = plan.eval(charges.detach().contiguous())
        plan.close()
        ctx.save_for_backward(points, charges, grad)
        ctx.cfg = (ncrit, p, theta, precision)
        return phi, grad

    @staticmethod
    def backward(ctx, g_phi, g_grad):
        points, charges, grad = ctx.saved_tensors
        need_x, need_q = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        through_grad = g_grad is not None and bool(torch.count_nonzero(g_grad))
        if (g_phi is None and not through_grad) or not (need_x or need_q):
            return None, None, None, None, None, None
        if g_phi is None:
            g_phi = torch.zeros(charges.shape[0], device=charges.device, dtype=torch.float32)
        plan = FMM(points.detach(), *ctx.cfg)
        if through_grad:
            # losses through grad phi: the Hessian FMM (five evaluations on the plan)
            dq, dx = plan.adjoint(charges.detach().contiguous(), g_phi.contiguous(), want_dq=need_q,
                                  want_dx=need_x, dL_dgrad=g_grad.contiguous())
        else:
            dq, dx = plan.adjoint(charges.detach().contiguous(), g_phi.contiguous(), gradient_fwd=grad,
                                  want_dq=need_q, want_dx=need_x)
        plan.close()
        return dx, dq, None, None, None, None


def fmm_apply(points, charges, ncrit=64, p=10, theta=0.4, precision="fp32"):
    """Differentiable FMM: returns (phi [n], grad phi [n, 3])."""
    return FMMFunction.apply(points, charges, ncrit, p, theta, precision)
