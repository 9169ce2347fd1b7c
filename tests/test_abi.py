"""C ABI checks that need no GPU: the library loads, exports every function that
include/fmm.h declares, and rejects invalid arguments before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmm.h")
LIB = os.path.join(ROOT, "paper_1602_02244_amd", "_fmm_hip.so")

FMM_OK, FMM_EINVAL = 0, 1


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    return C.CDLL(LIB)


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(fmm_[a-z_0-9]+)\s*\(", src))
    typedefs = set(re.findall(r"\(\*\s*(fmm_[a-z_0-9]+)\)", src))
    return sorted(names - typedefs)


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("fmm_plan", "fmm_plan_ex", "fmm_eval", "fmm_eval_ex", "fmm_adjoint", "fmm_plan_stats", "fmm_plan_export",
                 "fmm_plan_destroy", "fmm_last_error", "fmm_set_allocator", "fmm_plan_set_timing",
                 "fmm_plan_phase_times"):
        assert want in names


def test_library_exports_every_declared_function(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def _plan(lib, pts, n, ncrit, p, theta, prec=0):
    lib.fmm_plan.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_float, C.c_int, C.c_void_p,
                             C.POINTER(C.c_void_p)]
    lib.fmm_plan.restype = C.c_int
    out = C.c_void_p(1234)
    st = lib.fmm_plan(pts, n, ncrit, p, theta, prec, None, C.byref(out))
    return st, out


@pytest.mark.parametrize("n,ncrit,p,theta,prec", [
    (0, 64, 4, 0.4, 0), (-5, 64, 4, 0.4, 0), (10, 0, 4, 0.4, 0), (10, 64, -1, 0.4, 0), (10, 64, 17, 0.4, 0),
    (10, 64, 4, 0.0, 0), (10, 64, 4, -0.1, 0), (10, 64, 4, 0.58, 0), (10, 64, 4, float("nan"), 0),
    (10, 64, 4, float("inf"), 0), (10, 64, 4, 0.4, 7),
])
def test_plan_rejects_invalid_arguments_before_any_device_call(lib, n, ncrit, p, theta, prec):
    fake = C.c_void_p(0x1000)          # never dereferenced: validation fails first
    st, out = _plan(lib, fake, n, ncrit, p, theta, prec)
    assert st == FMM_EINVAL and out.value is None
    lib.fmm_last_error.restype = C.c_char_p
    assert len(lib.fmm_last_error()) > 0


@pytest.mark.parametrize("tol,prec,lists", [(-1e-3, 0, 0), (float("nan"), 0, 0), (float("inf"), 0, 0), (1e-6, 1, 0),
                                            (0.0, 0, 2), (0.0, 0, -1)])
def test_plan_ex_rejects_bad_arguments_before_any_device_call(lib, tol, prec, lists):
    lib.fmm_plan_ex.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_float, C.c_int, C.c_double, C.c_int,
                                C.c_void_p, C.POINTER(C.c_void_p)]
    lib.fmm_plan_ex.restype = C.c_int
    out = C.c_void_p(1234)
    st = lib.fmm_plan_ex(C.c_void_p(0x1000), 10, 64, 4, 0.4, prec, tol, lists, None, C.byref(out))
    assert st == FMM_EINVAL and out.value is None


@pytest.mark.parametrize("tol", [-1e-3, 1.0, 2.0, float("nan"), float("inf")])
def test_plan_svd_rejects_bad_tolerance_before_any_device_call(lib, tol):
    lib.fmm_plan_svd.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_float, C.c_double, C.c_void_p,
                                 C.POINTER(C.c_void_p)]
    lib.fmm_plan_svd.restype = C.c_int
    out = C.c_void_p(1234)
    st = lib.fmm_plan_svd(C.c_void_p(0x1000), 10, 64, 4, 0.4, tol, None, C.byref(out))
    assert st == FMM_EINVAL and out.value is None


def test_null_pointers_rejected(lib):
    st, _ = _plan(lib, None, 10, 64, 4, 0.4)
    assert st == FMM_EINVAL
    lib.fmm_plan.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_float, C.c_int, C.c_void_p, C.c_void_p]
    assert lib.fmm_plan(C.c_void_p(0x1000), 10, 64, 4, C.c_float(0.4), 0, None, None) == FMM_EINVAL
    for f, nargs in (("fmm_eval", 5), ("fmm_eval_ex", 6), ("fmm_adjoint", 7)):
        fn = getattr(lib, f)
        fn.restype = C.c_int
        fn.argtypes = [C.c_void_p] + [C.c_void_p] * (nargs - 1) if f != "fmm_eval_ex" else \
            [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
        args = [None] * nargs if f != "fmm_eval_ex" else [None, None, None, None, 3, None]
        assert fn(*args) == FMM_EINVAL
    lib.fmm_plan_stats.argtypes = [C.c_void_p, C.c_void_p]
    assert lib.fmm_plan_stats(None, None) == FMM_EINVAL
    lib.fmm_plan_destroy.argtypes = [C.c_void_p]
    lib.fmm_plan_destroy(None)          # no-op


def test_dipole_eval_rejects_null_arguments_before_any_device_call(lib):
    f = lib.fmm_eval_dipoles
    f.restype = C.c_int
    f.argtypes = [C.c_void_p] * 6
    fake = C.c_void_p(0x1000)
    for args in ((None, fake, fake, fake, fake, None), (fake, None, fake, fake, fake, None),
                 (fake, fake, None, fake, fake, None), (fake, fake, fake, None, None, None)):
        assert f(*args) == FMM_EINVAL


def test_target_calls_reject_bad_arguments_before_any_device_call(lib):
    f = lib.fmm_plan_targets
    f.restype = C.c_int
    f.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_float, C.c_int, C.c_void_p,
                  C.POINTER(C.c_void_p)]
    src, tgt = C.c_void_p(0x1000), C.c_void_p(0x2000)
    for a in ((src, 10, None, 5), (src, 10, tgt, 0), (src, 0, tgt, 5), (None, 10, tgt, 5)):
        out = C.c_void_p(0x1)
        assert f(*a, 64, 4, C.c_float(0.4), 0, None, C.byref(out)) == FMM_EINVAL and out.value is None
    out = C.c_void_p(0x1)
    assert f(src, 10, tgt, 5, 64, 4, C.c_float(0.7), 0, None, C.byref(out)) == FMM_EINVAL   # theta
    for name, nargs in (("fmm_eval_targets", 5), ("fmm_adjoint_targets", 9)):
        fn = getattr(lib, name)
        fn.restype = C.c_int
        fn.argtypes = [C.c_void_p] * nargs
        assert fn(*([None] * nargs)) == FMM_EINVAL


def test_allocator_pair_must_be_complete(lib):
    lib.fmm_set_allocator.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    lib.fmm_set_allocator.restype = C.c_int
    assert lib.fmm_set_allocator(C.c_void_p(0x10), None, None) == FMM_EINVAL
    assert lib.fmm_set_allocator(None, None, None) == FMM_OK


def test_binding_rejects_host_tensors_without_a_device_call():
    import torch
    from paper_1602_02244_amd import FMM
    with pytest.raises(TypeError):
        FMM(torch.zeros(10, 3), 16, 4, 0.4)
    with pytest.raises(ValueError):
        FMM(torch.zeros(10, 2), 16, 4, 0.4)


def test_stats_struct_matches_header():
    """The ctypes mirror of struct fmm_stats has the header's field order."""
    from paper_1602_02244_amd.binding import FmmStats
    src = open(HEADER).read()
    body = src[src.index("struct fmm_stats {"):src.index("};", src.index("struct fmm_stats {"))]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl or decl.startswith("struct"):
            decl = decl.split("{", 1)[-1].strip()
        if not decl:
            continue
        names = decl.split(None, 1)[1]
        for nm in names.split(","):
            fields.append(re.sub(r"\[.*\]", "", nm).strip())
    assert [f for f, _ in FmmStats._fields_] == fields
