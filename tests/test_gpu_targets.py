"""Separate source and target sets: phi(y_t) = sum_j q_j / |y_t - x_j| at nt targets.

The plan is that of the union (sources first, targets with zero charge); the checks:
- bitwise equality with the one-set FMM on the union point set, sliced at the target rows
  (and its adjoint sliced at the source / target rows);
- parity with the FP64 oracle FMM on the union sampled at the target rows (the same tree,
  lists and truncation), relative L2 <= 1e-5 (FP32);
- accuracy against the two-set direct sum, and the adjoint against exact FP64 derivatives.
"""
import numpy as np
import pytest

import oracle
from paper_1602_02244_amd import inputs
from fmm_testlib import compare_plans, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def _np(t):
    return t.cpu().numpy()


def _sets(case):
    sdist, ns, tdist, nt, seed = case
    x, q = inputs.make(sdist, ns, seed)
    y, _ = inputs.make(tdist, nt, seed + 1)
    if tdist == "cube" and sdist != "cube":
        y = (y - 0.5) * 3.0            # a wider box than the sources: the union root grows
    return x, q, y.astype(np.float32)


CASES = [
    # sources, ns, targets, nt, seed
    ("plummer", 20000, "cube", 7001, 11),
    ("cube", 5000, "cube", 30000, 12),
    ("sphere", 16000, "plummer", 9000, 13),
    ("cube", 1, "cube", 1, 14),
    ("cube", 257, "cube", 3, 15),
]


def _ids(c):
    return "-".join(str(v) for v in c)


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("p,ncrit", [(8, 32), (10, 64)])
def test_targets_union_and_oracle_parity(case, p, ncrit):
    from paper_1602_02244_amd import FMM, FMMTargets
    x, q, y = _sets(case)
    ns, nt = len(x), len(y)
    plan = FMMTargets(_dev(x), _dev(y), ncrit, p, 0.4)
    phi, grad = plan.eval(_dev(q))
    phi_only, none = plan.eval(_dev(q), gradient=False)
    assert none is None
    union = np.concatenate([x, y])
    qu = np.concatenate([q, np.zeros(nt, np.float32)])
    one = FMM(_dev(union), ncrit, p, 0.4)
    uphi, ugrad = one.eval(_dev(qu))
    # the target plan keeps only the pairs that carry something, so it matches the one-set
    # plan on the union to rounding (the dropped pairs add exact zeros there)
    assert rel_l2(_np(phi), _np(uphi)[ns:]) <= 1e-6 and rel_l2(_np(grad), _np(ugrad)[ns:]) <= 1e-6
    assert np.array_equal(_np(phi_only), _np(phi))
    ora = oracle.Plan(union.astype(np.float64), ncrit, 0.4)
    ophi, ograd, _ = ora.eval(qu.astype(np.float64), p, sample=np.arange(ns, ns + nt))
    e = (rel_l2(_np(phi), ophi), rel_l2(_np(grad), ograd))
    print(f"{_ids(case)} p={p}: vs oracle phi {e[0]:.2e} grad {e[1]:.2e}")
    assert max(e) <= TOL
    if ns * nt <= 2e8:
        dphi, dgrad = oracle.direct_targets(x.astype(np.float64), q.astype(np.float64), y.astype(np.float64))
        ed = rel_l2(_np(phi), dphi)
        print(f"   vs direct sum phi {ed:.2e}")
        assert ed <= (1e-3 if p == 8 else 2e-4)
    plan.close()
    one.close()


@pytest.mark.parametrize("case", CASES[:3], ids=_ids)
def test_target_plan_keeps_the_pairs_that_carry_something(case):
    """The target plan's tree is the union's; its lists are the union's lists (the oracle's)
    without the pairs (A, B), A != B, in which neither A holds a target and B a source nor
    A a source and B a target."""
    from paper_1602_02244_amd import FMMTargets
    x, q, y = _sets(case)
    ns = len(x)
    plan = FMMTargets(_dev(x), _dev(y), 32, 8, 0.4)
    ora = oracle.Plan(np.concatenate([x, y]).astype(np.float64), 32, 0.4)
    oc = ora.cells()
    order, _ = ora.order()
    is_src = (order < ns).astype(np.int64)
    pre = np.concatenate([[0], np.cumsum(is_src)])
    start, count = np.asarray(oc["start"]), np.asarray(oc["count"])
    nsrc = pre[start + count] - pre[start]
    kind = (nsrc > 0).astype(np.int64) | ((count - nsrc > 0).astype(np.int64) << 1)

    def keep(pairs):
        ka, kb = kind[pairs[:, 0]], kind[pairs[:, 1]]
        return (pairs[:, 0] == pairs[:, 1]) | (((ka & 2) > 0) & ((kb & 1) > 0)) | (((ka & 1) > 0) & ((kb & 2) > 0))
    compare_plans(plan.export(), ora, keep)
    om2l, op2p = ora.pairs()
    st = plan.stats()
    print(f"{_ids(case)}: M2L pairs {st['m2l_pairs']} of {len(om2l)}, P2P pairs {st['p2p_pairs']} of {len(op2p)}")
    ora.close()
    plan.close()


def test_targets_on_sources_skip_the_coincident_source():
    """Targets placed exactly on the sources: the field of the other sources (the one-set
    potential), to FMM accuracy, with no non-finite value."""
    from paper_1602_02244_amd import FMMTargets
    x, q = inputs.make("plummer", 12000, 21)
    plan = FMMTargets(_dev(x), _dev(x), 32, 10, 0.4)
    phi, grad = plan.eval(_dev(q))
    assert bool(np.isfinite(_np(phi)).all() and np.isfinite(_np(grad)).all())
    ephi, egrad = oracle.direct(x.astype(np.float64), q.astype(np.float64))
    e = (rel_l2(_np(phi), ephi), rel_l2(_np(grad), egrad))
    print(f"targets on sources vs direct: phi {e[0]:.2e} grad {e[1]:.2e}")
    assert max(e) <= 1e-4


def test_mixed_precision_targets():
    from paper_1602_02244_amd import FMMTargets
    x, q, y = _sets(("plummer", 20000, "cube", 8000, 31))
    ns, nt = len(x), len(y)
    plan = FMMTargets(_dev(x), _dev(y), 32, 10, 0.4, precision="mixed")
    phi, grad = plan.eval(_dev(q))
    union = np.concatenate([x, y]).astype(np.float64)
    ora = oracle.Plan(union, 32, 0.4)
    qu = np.concatenate([q.astype(np.float64), np.zeros(nt)])
    ophi, ograd, _ = ora.eval(qu, 10, sample=np.arange(ns, ns + nt))
    e = (rel_l2(_np(phi), ophi), rel_l2(_np(grad), ograd))
    print(f"mixed targets vs oracle: phi {e[0]:.2e} grad {e[1]:.2e}")
    assert max(e) <= 1e-6


def test_target_adjoint_matches_union_and_oracle():
    """dL/dq = psi at the sources, dL/dx_tgt = w grad phi, dL/dx_src = q grad psi, with
    psi = sum_t w_t / |x - y_t|: the one-set adjoint on the union, sliced, to rounding, and
    the FP64 oracle's FMM of the same formulas to 1e-5."""
    from paper_1602_02244_amd import FMM, FMMTargets
    x, q, y = _sets(("plummer", 15000, "cube", 6000, 41))
    ns, nt = len(x), len(y)
    w = inputs.adjoint_weights(nt, 42)
    plan = FMMTargets(_dev(x), _dev(y), 32, 10, 0.4)
    phi, grad = plan.eval(_dev(q))
    dq, dxs, dxt = plan.adjoint(_dev(q), _dev(w), gradient_fwd=grad)
    dq2, dxs2, dxt2 = plan.adjoint(_dev(q), _dev(w))          # grad phi recomputed inside
    assert all(np.array_equal(_np(a), _np(b)) for a, b in ((dq, dq2), (dxs, dxs2), (dxt, dxt2)))
    only_dq, none_s, none_t = plan.adjoint(_dev(q), _dev(w), want_dx_src=False, want_dx_tgt=False)
    assert none_s is None and none_t is None and np.array_equal(_np(only_dq), _np(dq))
    union = np.concatenate([x, y])
    qu = np.concatenate([q, np.zeros(nt, np.float32)])
    wu = np.concatenate([np.zeros(ns, np.float32), w])
    one = FMM(_dev(union), 32, 10, 0.4)
    udq, udx = one.adjoint(_dev(qu), _dev(wu))
    assert rel_l2(_np(dq), _np(udq)[:ns]) <= 1e-6
    assert rel_l2(_np(dxs), _np(udx)[:ns]) <= 1e-6 and rel_l2(_np(dxt), _np(udx)[ns:]) <= 1e-6
    ora = oracle.Plan(union.astype(np.float64), 32, 0.4)
    _, gphi, _ = ora.eval(qu.astype(np.float64), 10)
    psi, gpsi, _ = ora.eval(wu.astype(np.float64), 10)
    e = (rel_l2(_np(dq), psi[:ns]), rel_l2(_np(dxs), q.astype(np.float64)[:, None] * gpsi[:ns]),
         rel_l2(_np(dxt), w.astype(np.float64)[:, None] * gphi[ns:]))
    print(f"target adjoint vs oracle: dq {e[0]:.2e} dx_src {e[1]:.2e} dx_tgt {e[2]:.2e}")
    assert max(e) <= TOL
    plan.close()
    one.close()


def test_target_adjoint_through_grad_matches_union():
    from paper_1602_02244_amd import FMM, FMMTargets
    x, q, y = _sets(("cube", 9000, "plummer", 7000, 51))
    ns, nt = len(x), len(y)
    rng = np.random.default_rng(52)
    w = rng.standard_normal(nt).astype(np.float32)
    g = rng.standard_normal((nt, 3)).astype(np.float32)
    plan = FMMTargets(_dev(x), _dev(y), 32, 8, 0.4)
    dq, dxs, dxt = plan.adjoint(_dev(q), _dev(w), dL_dgrad=_dev(g))
    union = np.concatenate([x, y])
    one = FMM(_dev(union), 32, 8, 0.4)
    udq, udx = one.adjoint(_dev(np.concatenate([q, np.zeros(nt, np.float32)])),
                           _dev(np.concatenate([np.zeros(ns, np.float32), w])),
                           dL_dgrad=_dev(np.concatenate([np.zeros((ns, 3), np.float32), g])))
    assert rel_l2(_np(dq), _np(udq)[:ns]) <= 1e-6
    assert rel_l2(_np(dxs), _np(udx)[:ns]) <= 1e-6 and rel_l2(_np(dxt), _np(udx)[ns:]) <= 1e-6
    plan.close()
    one.close()


def _full(h6):
    h = np.empty((len(h6), 3, 3))
    for k, (a, b) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        h[:, a, b] = h6[:, k]
        h[:, b, a] = h6[:, k]
    return h


def test_autograd_targets_matches_exact_derivatives():
    """L = sum_t w_t phi_t + sum_t g_t . grad phi_t on a small problem (p = 12): autograd
    through fmm_apply_targets against the exact derivatives of the exact loss.  These are the
    one-set formulas on the union (charges [q; 0], weights [w; g] placed at the targets):
      dL/dq = psi - sum_a d_a phi^(a),  dL/dx = w E + q grad psi + H g - q sum_a H^(a) e_a
    with psi the direct sum of the weights w, E and H the gradient and Hessian of the direct
    sum of q, phi^(a) and H^(a) those of the charges g_a; the source rows give dL/dq and
    dL/dx_src, the target rows dL/dy."""
    import torch
    from paper_1602_02244_amd import FMMTargets, fmm_apply_targets
    x, q, y = _sets(("cube", 2500, "cube", 1500, 61))
    ns, nt = len(x), len(y)
    rng = np.random.default_rng(62)
    w = rng.standard_normal(nt)
    g = rng.standard_normal((nt, 3))
    xt, qt, yt = _dev(x).requires_grad_(True), _dev(q).requires_grad_(True), _dev(y).requires_grad_(True)
    phi, grad = fmm_apply_targets(xt, qt, yt, 16, 12, 0.4)
    ((phi * _dev(w)).sum() + (grad * _dev(g)).sum()).backward()
    # exact derivatives on the union (targets with zero charge, sources with zero weights)
    ud = np.concatenate([x, y]).astype(np.float64)
    qu = np.concatenate([q.astype(np.float64), np.zeros(nt)])
    wu = np.concatenate([np.zeros(ns), w])
    gu = np.concatenate([np.zeros((ns, 3)), g])
    psi, gpsi = oracle.direct(ud, wu)
    _, E = oracle.direct(ud, qu)
    H = _full(oracle.direct_hessian(ud, qu))
    edq = psi.copy()
    edx = wu[:, None] * E + qu[:, None] * gpsi + np.einsum("kab,kb->ka", H, gu)
    for a in range(3):
        _, ga = oracle.direct(ud, gu[:, a])
        edq -= ga[:, a]
        edx -= qu[:, None] * _full(oracle.direct_hessian(ud, gu[:, a]))[:, :, a]
    e = (rel_l2(_np(qt.grad), edq[:ns]), rel_l2(_np(xt.grad), edx[:ns]), rel_l2(_np(yt.grad), edx[ns:]))
    print(f"autograd targets vs exact: dq {e[0]:.2e} dx_src {e[1]:.2e} dx_tgt {e[2]:.2e}")
    assert max(e) <= 1e-4
    # the loss through phi alone takes the cheaper adjoint; it equals the plan's adjoint bitwise
    for t in (xt, qt, yt):
        t.grad = None
    phi, grad = fmm_apply_targets(xt, qt, yt, 16, 12, 0.4)
    (phi * _dev(w)).sum().backward()
    plan = FMMTargets(_dev(x), _dev(y), 16, 12, 0.4)
    dq, dxs, dxt = plan.adjoint(_dev(q), _dev(w))
    assert torch.equal(qt.grad, dq) and torch.equal(xt.grad, dxs) and torch.equal(yt.grad, dxt)
    plan.close()


def test_one_set_and_target_calls_do_not_mix():
    import ctypes as C
    from paper_1602_02244_amd import FMM, FMMTargets
    from paper_1602_02244_amd.binding import load_library
    x, q, y = _sets(("cube", 3000, "cube", 1000, 71))
    tp = FMMTargets(_dev(x), _dev(y), 32, 6, 0.4)
    with pytest.raises(ValueError, match="EINVAL"):
        FMM.eval(tp, _dev(np.zeros(tp.n, np.float32)))
    with pytest.raises(ValueError, match="EINVAL"):
        tp.eval_hessian(_dev(q))
    one = FMM(_dev(x), 32, 6, 0.4)
    lib = load_library()
    qd, out = _dev(q), _dev(np.zeros(3000, np.float32))
    assert lib.fmm_eval_targets(one._handle(), C.c_void_p(qd.data_ptr()), C.c_void_p(out.data_ptr()), None,
                                None) == 1
    with pytest.raises(ValueError, match="charges"):
        tp.eval(_dev(np.zeros(4000, np.float32)))   # charges are [ns]
    tp.close()
    one.close()
