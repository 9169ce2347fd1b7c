"""Every expansion order p = 0..16, plain FP32 and mixed precision, against the FP64
oracle's FMM on the same tree and lists (relative L2 <= 1e-5 for phi and grad phi).

The GEMM kernels are instantiated per order: the coefficient padding (the last
16-wide chunk of (p+1)^2 coefficients and the k steps of it that hold only padding),
the row blocks per wave and, for the split-FP16 M2L, the waves per workgroup all
change with p.  One small cloud with a few tree levels runs every instantiation.
"""
import numpy as np
import pytest

import oracle
from paper_1602_02244_amd import inputs
from fmm_testlib import rel_l2

pytestmark = pytest.mark.gpu

N, NCRIT, THETA = 2000, 24, 0.4


@pytest.fixture(scope="module")
def cloud():
    x, q = inputs.make("cube", N, 501)
    ora = oracle.Plan(x.astype(np.float64), NCRIT, THETA)
    assert ora.nm2l > 0
    return x, q, ora


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


@pytest.mark.parametrize("p", range(17))
def test_order_against_oracle(cloud, p):
    from paper_1602_02244_amd import FMM
    x, q, ora = cloud
    ophi, ograd, _ = ora.eval(q.astype(np.float64), p)
    for prec in ("fp32", "mixed"):
        plan = FMM(_dev(x), NCRIT, p, THETA, precision=prec)
        phi, grad = plan.eval(_dev(q))
        e = (rel_l2(phi.cpu().numpy(), ophi), rel_l2(grad.cpu().numpy(), ograd))
        print(f"p={p} {prec}: phi {e[0]:.2e} grad {e[1]:.2e}")
        assert max(e) <= 1e-5, (p, prec, e)
        plan.close()
