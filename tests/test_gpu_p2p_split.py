"""Near field of leaves whose lists are split into pieces (adaptive trees).

In the Plummer cloud a few coarse leaves of the outer halo (tens of bodies) hold near
fields of ~5e5 source bodies each; the plan cuts such a leaf into pieces of about
kP2PPieceWork interactions that run as separate workgroups and are summed in piece
order.  The near field alone (phases = FMM_NEAR) at the bodies of those leaves, and at
random bodies, is compared with the FP64 oracle's near field; reruns are bit-identical.
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


def _heavy_targets(x, ncrit, theta, nleaves=3):
    """Input indices of the bodies of the nleaves leaves with the largest near fields."""
    ora = oracle.Plan(x.astype(np.float64), ncrit, theta)
    c = ora.cells()
    _, p2p = ora.pairs()
    cnt = c["count"]
    a, b = p2p[:, 0], p2p[:, 1]
    work = np.zeros(ora.ncells)
    np.add.at(work, a, cnt[a] * cnt[b])
    heavy = np.argsort(work)[::-1][:nleaves]
    order, _ = ora.order()
    idx = np.concatenate([order[c["start"][h]:c["start"][h] + cnt[h]] for h in heavy])
    return ora, idx, work[heavy]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("mixed", 1e-6)])
def test_plummer_split_leaves_near_field(precision, tol):
    import torch
    from paper_1602_02244_amd import FMM
    from paper_1602_02244_amd.binding import FMM_NEAR
    n0, dist, p, ncrit, theta = inputs.WORKLOADS["plummer-1M"]
    x, q = inputs.workload("plummer-1M")
    ora, heavy, work = _heavy_targets(x, ncrit, theta)
    assert work.min() > 8 * (1 << 20)            # these leaves are split
    plan = FMM(_dev(x), ncrit, p, theta, precision=precision)
    st = plan.stats()
    # at least the three heavy leaves are cut (each into >= 8 pieces); every other leaf is one item
    assert st["p2p_split_pieces"] >= 24 and st["p2p_work_items"] > st["nleaves"]
    qt = _dev(q)
    phi, grad = plan.eval(qt, phases=FMM_NEAR)
    phi2, grad2 = plan.eval(qt, phases=FMM_NEAR)
    assert torch.equal(phi, phi2) and torch.equal(grad, grad2)
    samp = np.concatenate([heavy, inputs.sample_targets(x.shape[0], 200)])
    ophi, ograd, _ = ora.eval(q.astype(np.float64), p, mode=oracle.NEAR, sample=samp)
    phi, grad = phi.cpu().numpy()[samp], grad.cpu().numpy()[samp]
    nh = heavy.shape[0]
    e_heavy = (rel_l2(phi[:nh], ophi[:nh]), rel_l2(grad[:nh], ograd[:nh]))
    e_rand = (rel_l2(phi[nh:], ophi[nh:]), rel_l2(grad[nh:], ograd[nh:]))
    print(f"plummer-1M {precision}: {st['p2p_split_pieces']} pieces in {st['p2p_work_items']} items; "
          f"near field vs oracle: split leaves {e_heavy[0]:.2e} {e_heavy[1]:.2e}, random {e_rand[0]:.2e} {e_rand[1]:.2e}")
    assert max(e_heavy) <= tol and max(e_rand) <= tol
