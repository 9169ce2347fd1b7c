"""Pins of the oracle's dipole sources (CPU).

A dipole g at x is the derivative of a unit charge's field as the charge moves along g,
so every dipole quantity of the oracle is checked against central differences of the
corresponding charge quantity with the sources displaced (no formula is retyped): the
direct sum, the dipole multipole, and the FMM with dipoles against the direct sum
(geometric convergence in p)."""
import numpy as np

import oracle
from fmm_testlib import rel_l2


def _cloud(seed, ns=60, nt=25):
    rng = np.random.default_rng(seed)
    src = rng.random((ns, 3))
    tgt = 2.0 + rng.random((nt, 3))          # well apart from the sources
    g = rng.standard_normal((ns, 3))
    return src, tgt, g


def _field_at_targets(src, tgt, q_src):
    """Charge field of the sources at the separate targets (the targets carry no charge)."""
    pts = np.vstack([src, tgt])
    q = np.concatenate([q_src, np.zeros(len(tgt))])
    idx = np.arange(len(src), len(pts))
    return oracle.direct(pts, q, idx)


def test_direct_dipole_sum_is_the_derivative_of_moving_charges():
    src, tgt, g = _cloud(11)
    ones = np.ones(len(src))
    h = 1e-4
    fp, gp = _field_at_targets(src + h * g, tgt, ones)
    fm, gm = _field_at_targets(src - h * g, tgt, ones)
    fd_phi, fd_grad = (fp - fm) / (2 * h), (gp - gm) / (2 * h)
    pts = np.vstack([src, tgt])
    dip = np.vstack([g, np.zeros_like(tgt)])
    phi, grad = oracle.direct_dip(pts, np.zeros(len(pts)), dip, np.arange(len(src), len(pts)))
    assert rel_l2(phi, fd_phi) < 1e-7
    assert rel_l2(grad, fd_grad) < 1e-7


def test_direct_dipole_sum_adds_to_the_charge_sum_and_skips_itself():
    rng = np.random.default_rng(12)
    x = rng.random((80, 3))
    q = rng.standard_normal(80)
    g = rng.standard_normal((80, 3))
    phi_q, grad_q = oracle.direct(x, q)
    phi_0, grad_0 = oracle.direct_dip(x, q, np.zeros_like(g))
    assert np.array_equal(phi_q, phi_0) or rel_l2(phi_0, phi_q) < 1e-15
    assert rel_l2(grad_0, grad_q) < 1e-15
    # a point's own dipole contributes nothing to its field: the field at point i from the
    # others only, computed with point i's dipole changed, is unchanged
    g2 = g.copy()
    g2[7] *= -3.0
    a = oracle.direct_dip(x, q, g, [7])
    b = oracle.direct_dip(x, q, g2, [7])
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_dipole_multipole_is_the_derivative_of_the_charge_multipole():
    rng = np.random.default_rng(13)
    x = rng.random((30, 3)) - 0.5
    g = rng.standard_normal((30, 3))
    c = np.array([0.05, -0.02, 0.01])
    def cd(p, h):
        return (oracle.p2m(p, x + h * g, np.ones(30), c) - oracle.p2m(p, x - h * g, np.ones(30), c)) / (2 * h)
    for p in (0, 3, 8):
        h = 1e-3
        fd = (4 * cd(p, h / 2) - cd(p, h)) / 3          # Richardson: the h^2 term cancels
        m = oracle.p2m_dip(p, x, g, c)
        if p == 0:
            assert np.all(m == 0.0) and np.allclose(fd, 0.0, atol=1e-9)
        else:
            assert rel_l2(m, fd) < 1e-7


def test_fmm_with_dipoles_converges_to_the_direct_sum():
    rng = np.random.default_rng(14)
    n = 3000
    x = rng.random((n, 3))
    q = rng.standard_normal(n)
    g = rng.standard_normal((n, 3))
    ex_phi, ex_grad = oracle.direct_dip(x, q, g)
    plan = oracle.Plan(x, 32, 0.4)
    errs = []
    for p in (4, 8, 12):
        phi, grad = plan.eval_dip(q, g, p)
        errs.append(max(rel_l2(phi, ex_phi), rel_l2(grad, ex_grad)))
    plan.close()
    assert errs[2] < 1e-6
    assert errs[1] < errs[0] / 10 and errs[2] < errs[1] / 3
    # the charges alone through eval_dip equal the charge FMM
    plan = oracle.Plan(x, 32, 0.4)
    a = plan.eval_dip(q, np.zeros_like(g), 8)
    b = plan.eval(q, 8)
    plan.close()
    assert rel_l2(a[0], b[0]) < 1e-14 and rel_l2(a[1], b[1]) < 1e-14
