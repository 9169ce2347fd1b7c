"""fmm_adjoint_noalloc (static device scratch, no allocation) against fmm_adjoint.

Both are called through the C ABI on the same plans: two calls in a row, the second on a
smaller plan, each checked to the parity bar (relative L2 <= 1e-5; the two share every
kernel, so they agree bit for bit here); the no-allocation call makes no allocator call;
a plan above the static scratch's limit is rejected with EINVAL.
"""
import ctypes as C

import numpy as np
import pytest

from paper_1602_02244_amd import binding, inputs
from fmm_testlib import rel_l2

pytestmark = pytest.mark.gpu

_vp = C.c_void_p
MAX_N = 1 << 20


def _lib():
    lib = binding.load_library()
    lib.fmm_adjoint_noalloc.argtypes = [_vp] * 7
    lib.fmm_adjoint_noalloc.restype = C.c_int
    return lib


def _ptr(t):
    return _vp(t.data_ptr()) if t is not None else None


def _run(lib, fn, plan, q, gf, w, dq, dx):
    import torch
    st = fn(plan._handle(), _ptr(q), _ptr(gf), _ptr(w), _ptr(dq), _ptr(dx),
            _vp(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return st


def _case(lib, n, seed, with_gf):
    import torch
    from paper_1602_02244_amd import FMM
    x, q = inputs.make("plummer", n, seed)
    w = np.random.default_rng(seed + 1).standard_normal(n).astype(np.float32)
    xt, qt, wt = (torch.from_numpy(a).cuda() for a in (x, q, w))
    print(f"[noalloc] n={n} seed={seed} gradient_fwd={'given' if with_gf else 'NULL'}", flush=True)
    plan = FMM(xt, 64, 8, 0.4)
    gf = plan.eval(qt)[1] if with_gf else None
    out = {}
    for name in ("fmm_adjoint", "fmm_adjoint_noalloc"):
        dq = torch.full((n,), np.nan, device="cuda")
        dx = torch.full((n, 3), np.nan, device="cuda")
        assert _run(lib, getattr(lib, name), plan, qt, gf, wt, dq, dx) == binding.FMM_OK
        out[name] = (dq.cpu().numpy(), dx.cpu().numpy())
    a, b = out["fmm_adjoint"], out["fmm_adjoint_noalloc"]
    assert np.all(np.isfinite(b[0])) and np.all(np.isfinite(b[1]))
    assert rel_l2(b[0], a[0]) <= 1e-5 and rel_l2(b[1], a[1]) <= 1e-5
    # dL/dq alone (psi goes to the caller's buffer) and dL/dx alone (psi into the scratch)
    dq2 = torch.empty(n, device="cuda")
    assert _run(lib, lib.fmm_adjoint_noalloc, plan, qt, gf, wt, dq2, None) == binding.FMM_OK
    dx2 = torch.empty(n, 3, device="cuda")
    assert _run(lib, lib.fmm_adjoint_noalloc, plan, qt, gf, wt, None, dx2) == binding.FMM_OK
    assert rel_l2(dq2.cpu().numpy(), a[0]) <= 1e-5 and rel_l2(dx2.cpu().numpy(), a[1]) <= 1e-5
    plan.close()


def test_noalloc_matches_adjoint_two_calls():
    lib = _lib()
    _case(lib, 300000, 31, with_gf=True)
    _case(lib, 40000, 32, with_gf=False)     # second call: a smaller plan


def test_noalloc_makes_no_allocation():
    import torch
    from paper_1602_02244_amd import FMM
    lib = _lib()
    calls = []

    def alloc(nbytes, stream):
        calls.append(nbytes)
        return torch.cuda.caching_allocator_alloc(nbytes, stream=stream)

    x, q = inputs.make("cube", 50000, 41)
    w = np.random.default_rng(42).standard_normal(50000).astype(np.float32)
    xt, qt, wt = (torch.from_numpy(a).cuda() for a in (x, q, w))
    binding.set_allocator(alloc, lambda ptr, stream: torch.cuda.caching_allocator_delete(ptr))
    try:
        plan = FMM(xt, 64, 6, 0.4)
        built = len(calls)
        dq = torch.empty(50000, device="cuda")
        dx = torch.empty(50000, 3, device="cuda")
        assert _run(lib, lib.fmm_adjoint_noalloc, plan, qt, None, wt, dq, dx) == binding.FMM_OK
        assert len(calls) == built
        # the allocating entry point adds its scratch to the plan on first use
        assert _run(lib, lib.fmm_adjoint, plan, qt, None, wt, dq, dx) == binding.FMM_OK
        assert len(calls) > built
        plan.close()
    finally:
        binding.use_torch_allocator()


def test_noalloc_rejects_plans_above_its_limit():
    import torch
    from paper_1602_02244_amd import FMM
    lib = _lib()
    n = MAX_N + 1
    x = np.random.default_rng(7).random((n, 3)).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    qt = torch.ones(n, device="cuda")
    plan = FMM(xt, 64, 2, 0.4)
    dq = torch.empty(n, device="cuda")
    assert _run(lib, lib.fmm_adjoint_noalloc, plan, qt, None, qt, dq, None) == binding.FMM_EINVAL
    assert b"2^20" in lib.fmm_last_error()
    plan.close()
