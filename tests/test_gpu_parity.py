"""GPU path against the FP64 oracle: plan identity, per-phase and full parity, edge cases.

Parity bar (FP32 at fixed p): relative L2 error <= 1e-5 for phi and for grad phi,
against the oracle's FMM with the same tree, lists and truncation.
"""
import numpy as np
import pytest

import oracle
from paper_1602_02244_amd import inputs
from fmm_testlib import compare_plans, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5

CASES = [
    # dist, n, p, ncrit, theta
    ("cube", 30011, 6, 32, 0.4),
    ("cube", 20000, 10, 64, 0.5),
    ("plummer", 25000, 8, 32, 0.4),
    ("sphere", 24000, 7, 48, 0.45),
    ("cube", 6000, 12, 24, 0.3),
    ("cube", 5000, 0, 32, 0.4),
    ("plummer", 3000, 16, 64, 0.4),
]


def _ids(c):
    return "-".join(str(x) for x in c)


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def _run(torch, x, q, p, ncrit, theta, phases=3):
    from paper_1602_02244_amd import FMM
    xt = torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
    qt = torch.from_numpy(np.ascontiguousarray(q, np.float32)).cuda()
    plan = FMM(xt, ncrit=ncrit, p=p, theta=theta)
    phi, grad = plan.eval(qt, phases=phases)
    torch.cuda.synchronize()
    return plan, phi.cpu().numpy(), grad.cpu().numpy()


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_plan_identical_to_oracle(torch_mod, case):
    dist, n, p, ncrit, theta = case
    x, q = inputs.make(dist, n, 100 + n)
    plan, _, _ = _run(torch_mod, x, q, p, ncrit, theta)
    ora = oracle.Plan(x.astype(np.float64), ncrit, theta)
    compare_plans(plan.export(), ora)
    st = plan.stats()
    assert st["ncells"] == ora.ncells and st["m2l_pairs"] == ora.nm2l and st["p2p_pairs"] == ora.np2p


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_parity_near_far_full(torch_mod, case):
    dist, n, p, ncrit, theta = case
    x, q = inputs.make(dist, n, 100 + n)
    x64, q64 = x.astype(np.float64), q.astype(np.float64)
    ora = oracle.Plan(x64, ncrit, theta)
    for mode in (oracle.NEAR, oracle.FAR, oracle.BOTH):
        _, phi, grad = _run(torch_mod, x, q, p, ncrit, theta, phases=mode)
        ophi, ograd, _ = ora.eval(q64, p, mode=mode)
        e_phi, e_grad = rel_l2(phi, ophi), rel_l2(grad, ograd)
        print(f"{case} mode={mode} phi {e_phi:.2e} grad {e_grad:.2e}")
        assert e_phi <= TOL and e_grad <= TOL, (mode, e_phi, e_grad)


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_parity_every_pair_through_the_slot_pool(torch_mod, monkeypatch, case):
    """The same clouds with every M2L pair regrouped into slots (the test mode that pools
    every (tile, key) cell and keeps the pool whatever its shape): full FMM parity."""
    dist, n, p, ncrit, theta = case
    monkeypatch.setenv("FMM_M2L_DENSE_PCT", "101")
    x, q = inputs.make(dist, n, 100 + n)
    plan, phi, grad = _run(torch_mod, x, q, p, ncrit, theta)
    st = plan.stats()
    assert st["m2l_pairs"] == 0 or st["m2l_slots"] > 0
    ora = oracle.Plan(x.astype(np.float64), ncrit, theta)
    ophi, ograd, _ = ora.eval(q.astype(np.float64), p)
    e_phi, e_grad = rel_l2(phi, ophi), rel_l2(grad, ograd)
    print(f"{case} pooled: slots {st['m2l_slots']} phi {e_phi:.2e} grad {e_grad:.2e}")
    assert e_phi <= TOL and e_grad <= TOL


def test_full_accuracy_against_direct_sum(torch_mod):
    x, q = inputs.workload("uniform-4k")
    _, phi, grad = _run(torch_mod, x, q, 6, 64, 0.4)
    dphi, dgrad = oracle.direct(x.astype(np.float64), q.astype(np.float64))
    assert rel_l2(phi, dphi) < 1e-4 and rel_l2(grad, dgrad) < 1e-4


@pytest.mark.parametrize("n", [1, 2, 17, 64])
def test_single_leaf_is_direct_sum(torch_mod, n):
    x, q = inputs.uniform_cube(n, 5 + n)
    plan, phi, grad = _run(torch_mod, x, q, 5, 64, 0.4)
    st = plan.stats()
    assert st["ncells"] == 1 and st["m2l_pairs"] == 0
    dphi, dgrad = oracle.direct(x.astype(np.float64), q.astype(np.float64))
    if n == 1:
        assert phi[0] == 0.0 and np.all(grad == 0.0)
    else:
        np.testing.assert_allclose(phi, dphi, rtol=2e-6, atol=1e-6 * np.abs(dphi).max())
        np.testing.assert_allclose(grad, dgrad, rtol=2e-5, atol=1e-5 * np.abs(dgrad).max())


def test_two_bodies_closed_form(torch_mod):
    x = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0]], np.float32)
    q = np.array([2.0, -5.0], np.float32)
    _, phi, grad = _run(torch_mod, x, q, 3, 1, 0.4)
    np.testing.assert_allclose(phi, [-1.0, 0.4], rtol=1e-6)
    np.testing.assert_allclose(grad[0], [-0.12, -0.16, 0.0], rtol=1e-5, atol=1e-7)


def test_coincident_and_duplicate_points(torch_mod):
    x, q = inputs.uniform_cube(4000, 77)
    x[3000:3400] = x[100]            # 401 copies of one point
    x[3500:3600] = x[2000:2100]      # pairs of duplicates
    plan, phi, grad = _run(torch_mod, x, q, 6, 32, 0.4)
    ora = oracle.Plan(x.astype(np.float64), 32, 0.4)
    compare_plans(plan.export(), ora)
    ophi, ograd, _ = ora.eval(q.astype(np.float64), 6)
    assert rel_l2(phi, ophi) <= TOL and rel_l2(grad, ograd) <= TOL
    assert plan.stats()["max_level"] == 21           # the 401 copies cannot be separated


def test_deterministic_bitwise(torch_mod):
    import torch
    from paper_1602_02244_amd import FMM
    x, q = inputs.make("plummer", 20000, 9)
    xt, qt = torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda()
    a = FMM(xt, 32, 7, 0.4)
    b = FMM(xt, 32, 7, 0.4)
    p1, g1 = a.eval(qt)
    p2, g2 = a.eval(qt)
    p3, g3 = b.eval(qt)
    assert torch.equal(p1, p2) and torch.equal(g1, g2) and torch.equal(p1, p3) and torch.equal(g1, g3)


def test_slot_pool_order_deterministic_bitwise(torch_mod, monkeypatch):
    """Every pair through the slot pool: the traversal writes its slot records in an order
    that depends on which workgroup finishes first, and the pool sorts them by (target,
    key of the first pooled pair); two plans of one cloud must still give bit-identical
    results, and both match the oracle."""
    import torch
    from paper_1602_02244_amd import FMM
    monkeypatch.setenv("FMM_M2L_DENSE_PCT", "101")
    x, q = inputs.make("cube", 40000, 31)
    xt, qt = torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda()
    a = FMM(xt, 32, 6, 0.4)
    b = FMM(xt, 32, 6, 0.4)
    assert a.stats()["m2l_slots"] > 0 and a.stats()["m2l_slots"] == b.stats()["m2l_slots"]
    p1, g1 = a.eval(qt)
    p2, g2 = b.eval(qt)
    assert torch.equal(p1, p2) and torch.equal(g1, g2)
    ora = oracle.Plan(x.astype(np.float64), 32, 0.4)
    ophi, ograd, _ = ora.eval(q.astype(np.float64), 6)
    assert rel_l2(p1.cpu().numpy(), ophi) <= TOL and rel_l2(g1.cpu().numpy(), ograd) <= TOL
    a.close()
    b.close()


def test_nonfinite_coordinates_rejected(torch_mod):
    import torch
    from paper_1602_02244_amd import FMM, FMMError
    x, _ = inputs.uniform_cube(1000, 3)
    x[17, 1] = np.nan
    with pytest.raises(FMMError, match="ENONFINITE"):
        FMM(torch.from_numpy(x).cuda(), 32, 4, 0.4)
    x[17, 1] = np.inf
    with pytest.raises(FMMError, match="ENONFINITE"):
        FMM(torch.from_numpy(x).cuda(), 32, 4, 0.4)


def test_invalid_arguments_raise(torch_mod):
    import torch
    from paper_1602_02244_amd import FMM
    x = torch.rand(100, 3, device="cuda")
    for kw in (dict(ncrit=0), dict(p=-1), dict(p=17), dict(theta=0.0), dict(theta=0.58), dict(theta=float("nan"))):
        args = dict(ncrit=16, p=4, theta=0.4)
        args.update(kw)
        with pytest.raises(ValueError):
            FMM(x, **args)
