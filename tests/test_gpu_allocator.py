"""Plan workspace through PyTorch's caching allocator (fmm_set_allocator).

The binding installs torch's allocator when the library loads: a live plan's workspace
shows in torch.cuda.memory_allocated() and is gone after close(); an allocator that
fails makes the plan call raise MemoryError and leaves the library usable; a counting
allocator sees every block released at destroy, and parity is unchanged.
"""
import numpy as np
import pytest

import oracle
from paper_1602_02244_amd import binding, inputs
from fmm_testlib import rel_l2

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def test_workspace_is_torch_memory():
    import torch
    from paper_1602_02244_amd import FMM
    binding.use_torch_allocator()
    x, q = inputs.make("cube", 200000, 7)
    xt, qt = _dev(x), _dev(q)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    plan = FMM(xt, 64, 8, 0.4)
    phi, grad = plan.eval(qt)
    torch.cuda.synchronize()
    ws = plan.stats()["workspace_bytes"]
    during = torch.cuda.memory_allocated()
    outputs = phi.numel() * 4 + grad.numel() * 4
    # the plan's live blocks (torch rounds sizes up to 512 B)
    assert during - before - outputs >= ws * 0.99, (during, before, ws)
    del phi, grad
    plan.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before


def test_failing_allocator_raises_memory_error_and_recovers():
    import torch
    from paper_1602_02244_amd import FMM
    x, q = inputs.make("plummer", 20000, 11)
    xt, qt = _dev(x), _dev(q)
    try:
        binding.set_allocator(lambda nbytes, stream: 0, lambda ptr, stream: None)
        with pytest.raises(MemoryError):
            FMM(xt, 32, 6, 0.4)
        # fails after some blocks were handed out: those must be returned
        state = {"left": 5, "live": set()}

        def five_then_fail(nbytes, stream):
            if state["left"] == 0:
                return 0
            state["left"] -= 1
            p = torch.cuda.caching_allocator_alloc(nbytes, stream=stream)
            state["live"].add(p)
            return p

        def free(ptr, stream):
            state["live"].discard(ptr)
            torch.cuda.caching_allocator_delete(ptr)

        binding.set_allocator(five_then_fail, free)
        with pytest.raises(MemoryError):
            FMM(xt, 32, 6, 0.4)
        assert not state["live"]
    finally:
        binding.use_torch_allocator()
    plan = FMM(xt, 32, 6, 0.4)
    phi, grad = plan.eval(qt)
    ora = oracle.Plan(x.astype(np.float64), 32, 0.4)
    ophi, ograd, _ = ora.eval(q.astype(np.float64), 6)
    assert max(rel_l2(phi.cpu().numpy(), ophi), rel_l2(grad.cpu().numpy(), ograd)) <= 1e-5
    plan.close()


def test_counting_allocator_parity_and_release():
    import torch
    from paper_1602_02244_amd import FMM
    live, streams, calls = {}, set(), [0]

    def alloc(nbytes, stream):
        p = torch.cuda.caching_allocator_alloc(nbytes, stream=stream)
        live[p] = nbytes
        streams.add(stream)
        calls[0] += 1
        return p

    def free(ptr, stream):
        assert ptr in live
        del live[ptr]
        torch.cuda.caching_allocator_delete(ptr)

    x, q = inputs.make("cube", 30000, 21)
    w = np.random.default_rng(5).standard_normal(x.shape[0]).astype(np.float32)
    xt, qt, wt = _dev(x), _dev(q), _dev(w)
    binding.set_allocator(alloc, free)
    try:
        plan = FMM(xt, 32, 8, 0.4)
        phi, grad = plan.eval(qt)
        dq, dx = plan.adjoint(qt, wt, gradient_fwd=grad)
        torch.cuda.synchronize()
        assert calls[0] > 0 and sum(live.values()) >= plan.stats()["workspace_bytes"] * 0.99
        plan.close()
        assert not live, f"{len(live)} blocks not released"
    finally:
        binding.use_torch_allocator()
    # the plan stream and the library's near-field side stream
    assert torch.cuda.current_stream().cuda_stream in streams and len(streams) == 2
    ora = oracle.Plan(x.astype(np.float64), 32, 0.4)
    ophi, ograd, _ = ora.eval(q.astype(np.float64), 8)
    opsi, ogpsi, _ = ora.eval(w.astype(np.float64), 8)
    odx = w[:, None] * ograd + q[:, None] * ogpsi
    errs = (rel_l2(phi.cpu().numpy(), ophi), rel_l2(grad.cpu().numpy(), ograd), rel_l2(dq.cpu().numpy(), opsi),
            rel_l2(dx.cpu().numpy(), odx))
    assert max(errs) <= 1e-5, errs
