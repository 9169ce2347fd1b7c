"""Level-skip lists (fmm_plan_ex lists = level skip): the GPU plan equals the oracle's plan
built with the same rule, and the GPU FMM matches the oracle's FMM on those lists (1e-5)."""
import numpy as np
import pytest

import oracle
from paper_1602_02244_amd import inputs
from fmm_testlib import compare_plans, rel_l2

pytestmark = pytest.mark.gpu

CASES = [("cube", 30011, 8, 32, 0.4), ("plummer", 25000, 10, 32, 0.4), ("sphere", 24000, 7, 48, 0.45),
         ("cube", 6000, 12, 24, 0.5)]


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(str(v) for v in c))
def test_level_skip_plan_and_parity(case):
    from paper_1602_02244_amd import FMM
    dist, n, p, ncrit, theta = case
    x, q = inputs.make(dist, n, 81)
    plan = FMM(_dev(x), ncrit, p, theta, lists="level-skip")
    ora = oracle.Plan(x.astype(np.float64), ncrit, theta, lists=1)
    compare_plans(plan.export(), ora)
    st = plan.stats()
    assert st["lists"] == 1 and st["m2l_pairs"] < oracle.Plan(x.astype(np.float64), ncrit, theta).nm2l
    phi, grad = plan.eval(_dev(q))
    ophi, ograd, _ = ora.eval(q.astype(np.float64), p)
    e = (rel_l2(phi.cpu().numpy(), ophi), rel_l2(grad.cpu().numpy(), ograd))
    print(f"{case}: level skip, {st['m2l_pairs']} M2L pairs, vs oracle {e[0]:.2e} {e[1]:.2e}")
    assert max(e) <= 1e-5
    plan.close()


def test_level_skip_adjoint_identity():
    """Symmetric lists keep the FMM operator symmetric: <w, A q> = <q, A w>."""
    from paper_1602_02244_amd import FMM
    x, q = inputs.make("cube", 20000, 82)
    w = np.random.default_rng(83).standard_normal(20000).astype(np.float32)
    plan = FMM(_dev(x), 32, 8, 0.4, lists="level-skip")
    aq, _ = plan.eval(_dev(q))
    aw, _ = plan.eval(_dev(w))
    lhs = float(np.dot(w.astype(np.float64), aq.cpu().numpy().astype(np.float64)))
    rhs = float(np.dot(q.astype(np.float64), aw.cpu().numpy().astype(np.float64)))
    assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), abs(rhs))
    plan.close()
