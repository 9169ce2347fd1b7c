"""Charges with dipole sources (fmm_eval_dipoles), the evaluation behind the two-evaluation
adjoint through grad phi.  Parity against the FP64 oracle's FMM with dipoles on the same
lists (<= 1e-5, FP32 and mixed precision), against the exact direct sum on a small cloud,
and the charge-only case against the ordinary evaluation."""
import numpy as np
import pytest

import oracle
from paper_1602_02244_amd import inputs
from fmm_testlib import rel_l2

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


@pytest.mark.parametrize("dist,n,p,ncrit,theta,prec", [("cube", 20000, 8, 32, 0.4, "fp32"),
                                                       ("plummer", 20000, 10, 32, 0.4, "fp32"),
                                                       ("sphere", 16000, 12, 48, 0.45, "fp32"),
                                                       ("plummer", 20000, 10, 32, 0.4, "mixed")])
def test_dipole_parity(dist, n, p, ncrit, theta, prec):
    from paper_1602_02244_amd import FMM
    x, q = inputs.make(dist, n, 96)
    g = np.random.default_rng(97).standard_normal((n, 3)).astype(np.float32)
    plan = FMM(_dev(x), ncrit, p, theta, prec)
    print(f"[dipoles] {dist} n={n} p={p} {prec}", flush=True)
    phi, grad = plan.eval_dipoles(_dev(q), _dev(g))
    ora = oracle.Plan(x.astype(np.float64), ncrit, theta)
    ophi, ograd = ora.eval_dip(q.astype(np.float64), g.astype(np.float64), p)
    ora.close()
    e = (rel_l2(phi.cpu().numpy(), ophi), rel_l2(grad.cpu().numpy(), ograd))
    print(f"{dist} p={p} {prec}: phi {e[0]:.2e} grad {e[1]:.2e}")
    assert max(e) <= 1e-5
    plan.close()


def test_dipoles_against_the_direct_sum():
    from paper_1602_02244_amd import FMM
    x, q = inputs.make("cube", 4000, 98)
    g = np.random.default_rng(99).standard_normal((4000, 3)).astype(np.float32)
    plan = FMM(_dev(x), 32, 12, 0.4)
    phi, grad = plan.eval_dipoles(_dev(q), _dev(g))
    plan.close()
    ephi, egrad = oracle.direct_dip(x.astype(np.float64), q.astype(np.float64), g.astype(np.float64))
    e = (rel_l2(phi.cpu().numpy(), ephi), rel_l2(grad.cpu().numpy(), egrad))
    print(f"dipoles vs direct: phi {e[0]:.2e} grad {e[1]:.2e}")
    assert max(e) <= 1e-5


def test_zero_dipoles_give_the_charge_field_and_bad_arguments_are_rejected():
    import torch
    from paper_1602_02244_amd import FMM
    x, q = inputs.make("plummer", 10000, 100)
    plan = FMM(_dev(x), 32, 8, 0.4)
    phi0, grad0 = plan.eval(_dev(q))
    phi, grad = plan.eval_dipoles(_dev(q), torch.zeros(10000, 3, device="cuda"))
    assert rel_l2(phi.cpu().numpy(), phi0.cpu().numpy()) <= 1e-6
    assert rel_l2(grad.cpu().numpy(), grad0.cpu().numpy()) <= 1e-6
    with pytest.raises(ValueError):
        plan.eval_dipoles(_dev(q), torch.zeros(10000, 2, device="cuda"))
    # the ordinary evaluation after a dipole one is unchanged (no dipole state left behind)
    phi1, grad1 = plan.eval(_dev(q))
    assert torch.equal(phi1, phi0) and torch.equal(grad1, grad0)
    plan.close()
