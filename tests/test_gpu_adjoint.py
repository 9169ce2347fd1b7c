"""Adjoint of L = sum_i w_i phi_i through the FMM: dL/dq and dL/dx.

dL/dq = A w (A is symmetric), dL/dx_k = w_k grad phi(x_k) + q_k grad psi(x_k), psi = A w.
Checked against: the same FMM applied to w (bitwise), the dot-product identity, the
FP64 oracle's adjoint on the same plan, the exact FP64 gradient, and central finite
differences of the exact FP64 loss.
"""
import numpy as np
import pytest

import oracle
from paper_1602_02244_amd import inputs
from fmm_testlib import rel_l2

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def test_dq_is_fmm_of_w_and_dot_product():
    from paper_1602_02244_amd import FMM
    x, q = inputs.make("plummer", 30000, 41)
    w = inputs.adjoint_weights(30000, 7)
    plan = FMM(_dev(x), 32, 8, 0.4)
    phi, grad = plan.eval(_dev(q))
    psi, _ = plan.eval(_dev(w))
    dq, dx = plan.adjoint(_dev(q), _dev(w), gradient_fwd=grad)
    assert bool((dq == psi).all())
    a = float(np.dot(w.astype(np.float64), phi.cpu().numpy()))
    b = float(np.dot(q.astype(np.float64), psi.cpu().numpy()))
    assert abs(a - b) <= 1e-5 * max(abs(a), abs(b))
    # recomputing grad phi inside the adjoint gives the same dL/dx
    _, dx2 = plan.adjoint(_dev(q), _dev(w), gradient_fwd=None)
    assert bool((dx == dx2).all())


@pytest.mark.parametrize("dist,n,p,ncrit", [("plummer", 40000, 8, 32), ("cube", 30000, 10, 64)])
def test_adjoint_matches_oracle_fp64(dist, n, p, ncrit):
    from paper_1602_02244_amd import FMM
    x, q = inputs.make(dist, n, 43)
    w = inputs.adjoint_weights(n, 8)
    plan = FMM(_dev(x), ncrit, p, 0.4)
    dq, dx = plan.adjoint(_dev(q), _dev(w))
    ora = oracle.Plan(x.astype(np.float64), ncrit, 0.4)
    _, gphi, _ = ora.eval(q.astype(np.float64), p)
    psi, gpsi, _ = ora.eval(w.astype(np.float64), p)
    ref_dx = w.astype(np.float64)[:, None] * gphi + q.astype(np.float64)[:, None] * gpsi
    assert rel_l2(dq.cpu().numpy(), psi) <= 1e-5
    assert rel_l2(dx.cpu().numpy(), ref_dx) <= 1e-5


def test_autograd_function_matches_adjoint():
    import torch
    from paper_1602_02244_amd import FMM, fmm_apply
    x, q = inputs.make("sphere", 20000, 44)
    w = _dev(inputs.adjoint_weights(20000, 9))
    xt = _dev(x).requires_grad_(True)
    qt = _dev(q).requires_grad_(True)
    phi, grad = fmm_apply(xt, qt, ncrit=48, p=7, theta=0.4)
    loss = (w * phi).sum()
    loss.backward()
    plan = FMM(_dev(x), 48, 7, 0.4)
    dq, dx = plan.adjoint(_dev(q), w)
    assert torch.equal(qt.grad, dq) and torch.equal(xt.grad, dx)
    # a loss through grad phi goes through the Hessian FMM (fmm_adjoint_ex)
    xt.grad = None
    qt.grad = None
    phi, grad = fmm_apply(xt, qt, ncrit=48, p=7, theta=0.4)
    gw = _dev(np.random.default_rng(45).standard_normal((20000, 3)))
    ((w * phi).sum() + (gw * grad).sum()).backward()
    dq2, dx2 = plan.adjoint(_dev(q), w, dL_dgrad=gw)
    assert torch.equal(qt.grad, dq2) and torch.equal(xt.grad, dx2)


def _exact_loss_delta_fd(x, q, w, k, axis, h):
    """Central difference of L(x) = sum_i w_i phi_i(x) (exact, FP64) in coordinate (k, axis)."""
    x = x.astype(np.float64)
    q = q.astype(np.float64)
    w = w.astype(np.float64)
    c = w[k] * q + q[k] * w          # coefficient of G(x_k, x_i) in L
    mask = np.ones(x.shape[0], bool)
    mask[k] = False
    d = x[mask] - x[k]
    cc = c[mask]
    e = np.zeros(3)
    e[axis] = h
    gp = 1.0 / np.linalg.norm(d - e, axis=1)
    gm = 1.0 / np.linalg.norm(d + e, axis=1)
    return float(np.sum(cc * (gp - gm)) / (2 * h))


@pytest.mark.timeout(900)
def test_plummer_1M_finite_differences_and_fp64_gradient():
    """Differentiable workload: N = 2^20 Plummer, charges in (0,1], w ~ N(0,1), p = 10,
    ncrit = 64, theta = 0.4; central differences (h = 1e-3, Richardson with h/2 and h/4)
    on 64 random coordinates of the exact FP64 loss."""
    from paper_1602_02244_amd import FMM
    x, q = inputs.workload("plummer-1M")
    n = x.shape[0]
    w = inputs.adjoint_weights(n)
    plan = FMM(_dev(x), 64, 10, 0.4)
    phi, grad = plan.eval(_dev(q))
    dq, dx = plan.adjoint(_dev(q), _dev(w), gradient_fwd=grad)
    dx = dx.cpu().numpy().astype(np.float64)
    idx, ax = inputs.fd_coordinates(n)
    fd = []
    for k, a in zip(idx, ax):
        # central differences at h = 1e-3, h/2, h/4 combined by Richardson extrapolation (error O(h^6))
        d1, d2, d4 = (_exact_loss_delta_fd(x, q, w, k, a, h) for h in (1e-3, 5e-4, 2.5e-4))
        r1, r2 = (4 * d2 - d1) / 3, (4 * d4 - d2) / 3
        fd.append((16 * r2 - r1) / 15)
    fd = np.array(fd)
    got = dx[idx, ax]
    # exact FP64 gradient of the exact loss at the same coordinates
    samp = np.unique(idx)
    gphi, gpsi = oracle.direct(x, q, samp)[1], oracle.direct(x, w, samp)[1]
    pos = {s: i for i, s in enumerate(samp)}
    exact = np.array([w[k] * gphi[pos[k], a] + q[k] * gpsi[pos[k], a] for k, a in zip(idx, ax)])
    print("FD vs exact", rel_l2(fd, exact), "GPU vs exact", rel_l2(got, exact), "GPU vs FD", rel_l2(got, fd))
    assert rel_l2(fd, exact) < 2e-6            # the adjoint formula is the derivative of the loss
    assert rel_l2(got, fd) < 1e-4              # FMM gradient within the target tolerance
    assert rel_l2(got, exact) < 1e-4
    # FP64 oracle adjoint on the same plan (sampled targets): parity
    ora = oracle.Plan(x.astype(np.float64), 64, 0.4)
    _, ogphi, _ = ora.eval(q.astype(np.float64), 10, sample=samp)
    opsi, ogpsi, _ = ora.eval(w.astype(np.float64), 10, sample=samp)
    ref = np.array([w[k] * ogphi[pos[k], a] + q[k] * ogpsi[pos[k], a] for k, a in zip(idx, ax)])
    assert rel_l2(got, ref) <= 1e-5
    assert rel_l2(dq.cpu().numpy()[samp], opsi) <= 1e-5
