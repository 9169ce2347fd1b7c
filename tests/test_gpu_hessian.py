"""Hessian evaluation and the adjoint of losses through grad phi (fmm_eval_hessian,
fmm_adjoint_ex, FMMFunction.backward with a gradient on grad phi).

Parity: the GPU Hessian against the FP64 oracle's FMM Hessian on the same lists; the
adjoint against the same formula evaluated with the oracle's FMM with dipole sources
(FP64); and, on a small cloud, against the exact derivatives of the exact loss (direct
sums of charges, written with five sums so that no dipole code is involved)."""
import numpy as np
import pytest

import oracle
from paper_1602_02244_amd import inputs
from fmm_testlib import rel_l2

pytestmark = pytest.mark.gpu

IDX = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def _full(h):
    H = np.zeros((h.shape[0], 3, 3))
    for a, (i, j) in enumerate(IDX):
        H[:, i, j] = H[:, j, i] = h[:, a]
    return H


@pytest.mark.parametrize("dist,n,p,ncrit,theta", [("cube", 20000, 8, 32, 0.4), ("plummer", 20000, 10, 32, 0.4),
                                                  ("sphere", 16000, 12, 48, 0.45)])
def test_hessian_parity(dist, n, p, ncrit, theta):
    from paper_1602_02244_amd import FMM
    x, q = inputs.make(dist, n, 91)
    plan = FMM(_dev(x), ncrit, p, theta)
    phi, grad, hess = plan.eval_hessian(_dev(q))
    ora = oracle.Plan(x.astype(np.float64), ncrit, theta)
    ophi, ograd, _, ohess = ora.eval(q.astype(np.float64), p, hessian=True)
    e = (rel_l2(phi.cpu().numpy(), ophi), rel_l2(grad.cpu().numpy(), ograd), rel_l2(hess.cpu().numpy(), ohess))
    print(f"{dist} p={p}: phi {e[0]:.2e} grad {e[1]:.2e} hessian {e[2]:.2e}")
    assert max(e) <= 1e-5
    plan.close()


def _oracle_adjoint(ora, x, q, w, g, p):
    """The two-evaluation adjoint with the FP64 oracle FMM in place of every evaluation:
    dL/dq = Psi, dL/dx = w E + H g + q grad Psi (Psi the field of charges w and dipoles g)."""
    psi, gpsi = ora.eval_dip(w, g, p)
    _, E, _, h = ora.eval(q, p, hessian=True)
    dq = psi
    dx = w[:, None] * E + np.einsum("kab,kb->ka", _full(h), g) + q[:, None] * gpsi
    return dq, dx


def test_adjoint_through_grad_against_oracle():
    from paper_1602_02244_amd import FMM
    x, q = inputs.make("plummer", 15000, 92)
    rng = np.random.default_rng(93)
    w = rng.standard_normal(15000).astype(np.float32)
    g = rng.standard_normal((15000, 3)).astype(np.float32)
    plan = FMM(_dev(x), 32, 10, 0.4)
    dq, dx = plan.adjoint(_dev(q), _dev(w), dL_dgrad=_dev(g))
    ora = oracle.Plan(x.astype(np.float64), 32, 0.4)
    odq, odx = _oracle_adjoint(ora, x.astype(np.float64), q.astype(np.float64), w.astype(np.float64),
                               g.astype(np.float64), 10)
    e = (rel_l2(dq.cpu().numpy(), odq), rel_l2(dx.cpu().numpy(), odx))
    print(f"adjoint through grad phi vs oracle: dq {e[0]:.2e} dx {e[1]:.2e}")
    assert max(e) <= 1e-5
    plan.close()


def test_autograd_through_grad_matches_exact_derivatives():
    """Small cloud: autograd of L = sum w phi + sum g . grad phi against the exact
    derivatives of the exact loss (direct sums; the FMM error at p = 12 is ~1e-7)."""
    import torch
    from paper_1602_02244_amd import fmm_apply
    n = 3000
    x, q = inputs.make("cube", n, 94)
    rng = np.random.default_rng(95)
    w = rng.standard_normal(n)
    g = rng.standard_normal((n, 3))
    xt = _dev(x).requires_grad_(True)
    qt = _dev(q).requires_grad_(True)
    phi, grad = fmm_apply(xt, qt, 16, 12, 0.4)
    loss = (phi * _dev(w)).sum() + (grad * _dev(g)).sum()
    loss.backward()
    xd, qd = x.astype(np.float64), q.astype(np.float64)
    psi, gpsi = oracle.direct(xd, w)
    _, E = oracle.direct(xd, qd)
    H = _full(oracle.direct_hessian(xd, qd))
    edq = psi.copy()
    edx = w[:, None] * E + qd[:, None] * gpsi + np.einsum("kab,kb->ka", H, g)
    for a in range(3):
        _, ga = oracle.direct(xd, g[:, a])
        edq -= ga[:, a]
        edx -= qd[:, None] * _full(oracle.direct_hessian(xd, g[:, a]))[:, :, a]
    e = (rel_l2(qt.grad.cpu().numpy(), edq), rel_l2(xt.grad.cpu().numpy(), edx))
    print(f"autograd through grad phi vs exact: dq {e[0]:.2e} dx {e[1]:.2e}")
    assert max(e) <= 1e-4
