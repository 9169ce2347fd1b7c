"""Variable-order M2L (fmm_plan_ex with m2l_tol > 0): operator blocks whose weighted size
is below the tolerance are left out.  Checked against the FP64 oracle's full-order FMM:
the extra error must stay of the order of the tolerance, vanish at tol = 0, and the
applied fraction of blocks must fall as the tolerance grows."""
import numpy as np
import pytest

import oracle
from paper_1602_02244_amd import inputs
from fmm_testlib import rel_l2

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


@pytest.mark.parametrize("dist,n,p,ncrit,theta", [("cube", 30000, 10, 32, 0.4), ("plummer", 25000, 8, 32, 0.4),
                                                  ("sphere", 24000, 12, 48, 0.45)])
def test_variable_order_against_oracle(dist, n, p, ncrit, theta):
    from paper_1602_02244_amd import FMM
    x, q = inputs.make(dist, n, 77)
    ora = oracle.Plan(x.astype(np.float64), ncrit, theta)
    ophi, ograd, _ = ora.eval(q.astype(np.float64), p)
    errs, kept = {}, {}
    for tol in (0.0, 1e-8, 1e-6, 1e-4):
        plan = FMM(_dev(x), ncrit, p, theta, m2l_tol=tol)
        phi, grad = plan.eval(_dev(q))
        st = plan.stats()
        kept[tol] = st["m2l_kept_fraction"]
        errs[tol] = max(rel_l2(phi.cpu().numpy(), ophi), rel_l2(grad.cpu().numpy(), ograd))
        plan.close()
        print(f"{dist} p={p} tol={tol:g}: kept {kept[tol]:.3f}, error vs oracle {errs[tol]:.2e}")
    assert kept[0.0] == 1.0 and errs[0.0] <= 1e-5
    assert kept[1e-8] < 1.0 and kept[1e-4] <= kept[1e-6] <= kept[1e-8]
    assert errs[1e-8] <= 1e-5                      # FP32 parity bar at the default tolerance
    assert errs[1e-6] <= 1e-5 + 10 * 1e-6          # the added error scales with the tolerance
    assert errs[1e-4] <= 1e-5 + 10 * 1e-4


def test_zero_tolerance_is_the_dense_path():
    from paper_1602_02244_amd import FMM
    x, q = inputs.make("cube", 20000, 78)
    out = []
    for tol in (None, 0.0):
        plan = FMM(_dev(x), 32, 8, 0.4) if tol is None else FMM(_dev(x), 32, 8, 0.4, m2l_tol=tol)
        phi, grad = plan.eval(_dev(q))
        out.append((phi.cpu().numpy(), grad.cpu().numpy()))
        plan.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_variable_order_rejects_mixed_and_bad_tolerance():
    from paper_1602_02244_amd import FMM
    x, _ = inputs.make("cube", 1000, 79)
    with pytest.raises(ValueError):
        FMM(_dev(x), 32, 6, 0.4, precision="mixed", m2l_tol=1e-6)
    for bad in (-1e-3, float("nan"), float("inf")):
        with pytest.raises(ValueError):
            FMM(_dev(x), 32, 6, 0.4, m2l_tol=bad)
