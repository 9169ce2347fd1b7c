"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's formulas: each checks a closed form, an
invariant, a library routine, or a brute-force count.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.special import eval_legendre

import oracle
from paper_1602_02244_amd import inputs

ROOT_GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


# ---------------------------------------------------------------- P1 direct sum
def test_direct_two_bodies_closed_form():
    x = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0]])
    q = np.array([2.0, -5.0])
    phi, g = oracle.direct(x, q)
    assert phi[0] == -1.0 and phi[1] == 0.4           # q_j / 5
    np.testing.assert_allclose(g[0], [-5 * 3 / 125, -5 * 4 / 125, 0], rtol=0, atol=1e-16)  # grad = +q (x_j-x_i)/r^3
    np.testing.assert_allclose(g[1], [-2 * 3 / 125, -2 * 4 / 125, 0], rtol=0, atol=1e-16)


def test_direct_newton_third_law_and_symmetry():
    x, q = inputs.uniform_cube(500, 7)
    x = x.astype(np.float64)
    q = q.astype(np.float64)
    phi, g = oracle.direct(x, q)
    f = q[:, None] * g
    assert np.abs(f.sum(0)).max() < 1e-12 * np.abs(f).sum()
    w = np.random.default_rng(1).standard_normal(500)
    psi, _ = oracle.direct(x, w)
    assert abs(w @ phi - q @ psi) < 1e-12 * (np.abs(w) @ np.abs(phi))


def test_direct_power_of_two_scaling_exact_and_permutation():
    x, q = inputs.uniform_cube(300, 8)
    x = x.astype(np.float64); q = q.astype(np.float64)
    phi, g = oracle.direct(x, q)
    phi2, g2 = oracle.direct(x * 8.0, q)
    assert np.array_equal(phi2, phi / 8.0)
    assert np.array_equal(g2, g / 64.0)
    perm = np.random.default_rng(2).permutation(300)
    phip, gp = oracle.direct(x[perm], q[perm])
    np.testing.assert_allclose(phip, phi[perm], rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(gp, g[perm], rtol=1e-13, atol=1e-13)


def test_direct_skips_coincident_points():
    x = np.array([[0.0, 0, 0], [0.0, 0, 0], [1.0, 0, 0]])
    q = np.array([1.0, 1.0, 1.0])
    phi, g = oracle.direct(x, q)
    assert phi.tolist() == [1.0, 1.0, 2.0]


# ---------------------------------------------------------------- P2 T tensors
@pytest.mark.parametrize("x", [[0.3, -1.1, 0.7], [2.0, 0.1, -0.4], [-0.05, 0.02, 1.3]])
def test_taylor_tensors_legendre_identity(x):
    """sum_{|a|=n} (-y)^a T_a(x) = |y|^n P_n(cos g) / |x|^(n+1): the degree-n term of 1/|x-y|."""
    P = 16
    T = oracle.taylor_T(P, x)
    mi = oracle.multi_indices(P)
    x = np.asarray(x)
    for y in ([0.1, 0.2, -0.05], [-0.3, 0.0, 0.2]):
        y = np.asarray(y)
        cosg = x @ y / np.linalg.norm(x) / np.linalg.norm(y)
        for n in range(P + 1):
            sel = mi.sum(1) == n
            lhs = np.sum(np.prod((-y) ** mi[sel], axis=1) * T[sel])
            rhs = np.linalg.norm(y) ** n * eval_legendre(n, cosg) / np.linalg.norm(x) ** (n + 1)
            assert abs(lhs - rhs) <= 1e-13 * max(abs(rhs), np.linalg.norm(y) ** n / np.linalg.norm(x) ** (n + 1))


def test_taylor_tensors_symbolic_low_order():
    sp = pytest.importorskip("sympy")
    X, Y, Z = sp.symbols("X Y Z")
    f = 1 / sp.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    pt = {X: sp.Rational(3, 10), Y: sp.Rational(-7, 10), Z: sp.Rational(11, 10)}
    T = oracle.taylor_T(4, [0.3, -0.7, 1.1])
    for k, (a, b, c) in enumerate(oracle.multi_indices(4)):
        d = f
        if a: d = sp.diff(d, X, int(a))
        if b: d = sp.diff(d, Y, int(b))
        if c: d = sp.diff(d, Z, int(c))
        val = float(d.subs(pt)) / (math.factorial(a) * math.factorial(b) * math.factorial(c))
        assert abs(T[k] - val) <= 1e-13 * max(1.0, abs(val))


# ---------------------------------------------------------------- P3 multipole truncation
@pytest.mark.parametrize("p", [0, 3, 6, 10])
def test_multipole_truncation_on_axis_closed_form(p):
    a, r = 0.3, 1.7
    for direction in ([0, 0, 1.0], [1.0, 0, 0], np.array([1.0, 2.0, -2.0]) / 3.0):
        d = np.asarray(direction, float)
        M = oracle.p2m(p, (a * d)[None, :], [1.0], [0, 0, 0])
        val = oracle.multipole_eval(p, M, [0, 0, 0], (r * d)[None, :])[0]
        exact_err = a ** (p + 1) / (r ** (p + 1) * (r - a))
        assert abs((1 / (r - a) - val) - exact_err) < 1e-14
    # off-axis: error bounded by the same expression
    M = oracle.p2m(p, [[0.1, -0.2, 0.15]], [1.0], [0, 0, 0])
    xt = np.array([[1.0, 0.9, -0.8]])
    rr, aa = np.linalg.norm(xt), np.linalg.norm([0.1, -0.2, 0.15])
    err = abs(1 / np.linalg.norm(xt[0] - [0.1, -0.2, 0.15]) - oracle.multipole_eval(p, M, [0, 0, 0], xt)[0])
    assert err <= aa ** (p + 1) / (rr ** (p + 1) * (rr - aa)) * (1 + 1e-9) + 1e-15


# ---------------------------------------------------------------- P4 M2M / L2L exactness
def test_m2m_exact_translation():
    rng = np.random.default_rng(3)
    p = 8
    y = rng.uniform(-0.25, 0.25, (20, 3)) + [0.25, -0.25, 0.25]
    q = rng.uniform(-1, 1, 20)
    child_c = np.array([0.25, -0.25, 0.25])
    Mc = oracle.p2m(p, y, q, child_c)
    Mp = oracle.m2m(p, Mc, child_c - 0.0)
    Mref = oracle.p2m(p, y, q, [0, 0, 0])
    np.testing.assert_allclose(Mp, Mref, rtol=1e-12, atol=1e-14)


def test_l2l_exact_translation():
    rng = np.random.default_rng(4)
    p = 7
    L = rng.standard_normal(oracle.num_coeffs(p))
    c, cc = np.zeros(3), np.array([-0.25, 0.25, 0.25])
    Lc = oracle.l2l(p, L, cc - c)
    x = cc + rng.uniform(-0.25, 0.25, (10, 3))
    f1, g1 = oracle.l2p(p, L, c, x)
    f2, g2 = oracle.l2p(p, Lc, cc, x)
    np.testing.assert_allclose(f2, f1, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(g2, g1, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- P5 M2L truncation rule
@pytest.mark.parametrize("p", [1, 4, 7])
def test_m2l_collinear_full_square_truncation(p):
    """Charge at z=a about c_B=0, local centre at z=D, target at z=D+b.  The
    truncated value is sum_{n<=p} sum_{j<=p} C(n+j,j) a^n (-b)^j / D^(n+j+1)."""
    a, D, b = Fraction(1, 4), Fraction(2), Fraction(-3, 16)
    exact = sum(Fraction(math.comb(n + j, j)) * a ** n * (-b) ** j / D ** (n + j + 1)
                for n in range(p + 1) for j in range(p + 1))
    tri = sum(Fraction(math.comb(n + j, j)) * a ** n * (-b) ** j / D ** (n + j + 1)
              for n in range(p + 1) for j in range(p + 1 - n))
    M = oracle.p2m(p, [[0, 0, float(a)]], [1.0], [0, 0, 0])
    L = oracle.m2l(p, M, [0, 0, float(D)])
    phi, _ = oracle.l2p(p, L, [0, 0, float(D)], [[0, 0, float(D + b)]])
    assert abs(phi[0] - float(exact)) < 1e-14 * abs(float(exact))
    assert abs(float(exact) - float(tri)) > 1e-6       # the two readings differ


# ---------------------------------------------------------------- P6 convergence, P7 single leaf
def test_fmm_converges_geometrically_with_order():
    x, q = inputs.workload("uniform-4k")
    x = x.astype(np.float64); q = q.astype(np.float64)
    ref, gref = oracle.direct(x, q)
    pl = oracle.Plan(x, 64, 0.4)
    errs, gerrs = [], []
    ps = [2, 4, 6, 8]
    for p in ps:
        phi, g, _ = pl.eval(q, p)
        errs.append(np.linalg.norm(phi - ref) / np.linalg.norm(ref))
        gerrs.append(np.linalg.norm(g - gref) / np.linalg.norm(gref))
    for e in (errs, gerrs):
        slope = np.polyfit(ps, np.log(e), 1)[0]
        assert math.exp(slope) < math.sqrt(3) * 0.4      # worst-case ratio sqrt(3)*theta
        assert all(e2 < e1 for e1, e2 in zip(e, e[1:]))
        assert e[2] < 1e-4                               # p = 6 meets the 1e-4 target


def test_single_leaf_is_direct_sum():
    x, q = inputs.uniform_cube(50, 11)
    x = x.astype(np.float64); q = q.astype(np.float64)
    pl = oracle.Plan(x, 64, 0.4)
    assert pl.ncells == 1 and pl.nm2l == 0 and pl.np2p == 1
    phi, g, _ = pl.eval(q, 4)
    ref, gref = oracle.direct(x, q)
    np.testing.assert_allclose(phi, ref, rtol=1e-13)
    np.testing.assert_allclose(g, gref, rtol=1e-12, atol=1e-13)


def test_sampled_mode_matches_full():
    x, q = inputs.uniform_cube(3000, 12)
    x = x.astype(np.float64); q = q.astype(np.float64)
    pl = oracle.Plan(x, 32, 0.4)
    phi, g, _ = pl.eval(q, 5)
    s = np.array([0, 17, 2999, 1500, 640])
    phs, gs, _ = pl.eval(q, 5, sample=s)
    np.testing.assert_allclose(phs, phi[s], rtol=1e-13)
    np.testing.assert_allclose(gs, g[s], rtol=1e-12, atol=1e-13)
    nf, _, _ = pl.eval(q, 5, mode=oracle.NEAR)
    ff, _, _ = pl.eval(q, 5, mode=oracle.FAR)
    np.testing.assert_allclose(nf + ff, phi, rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- P8 lists
def _coverage(pl):
    c = pl.cells()
    m2l, p2p = pl.pairs()
    n = pl.n
    cov = np.zeros((n, n), np.int16)
    for a, b in np.concatenate([m2l, p2p]):
        cov[c["start"][a]:c["start"][a] + c["count"][a], c["start"][b]:c["start"][b] + c["count"][b]] += 1
    return cov


@pytest.mark.parametrize("dist,theta,ncrit", [("cube", 0.4, 16), ("cube", 0.5, 8), ("plummer", 0.4, 10),
                                              ("sphere", 0.3, 12)])
def test_every_pair_covered_exactly_once(dist, theta, ncrit):
    x, q = inputs.make(dist, 1500, 21)
    pl = oracle.Plan(x.astype(np.float64), ncrit, theta)
    cov = _coverage(pl)
    assert cov.min() == 1 and cov.max() == 1
    m2l, p2p = pl.pairs()
    s1 = set(map(tuple, m2l)); s2 = set(map(tuple, p2p))
    assert s1 == {(b, a) for a, b in s1} and s2 == {(b, a) for a, b in s2}
    c = pl.cells()
    # MAC holds for every M2L pair, leaf occupancy respects ncrit
    side = 2.0 ** (pl.k - c["level"].astype(np.float64))
    ctr = np.zeros((pl.ncells, 3))
    for i in range(pl.ncells):
        l, pref = int(c["level"][i]), int(c["prefix"][i])
        ic = [0, 0, 0]
        for bb in range(l):
            ic[0] |= ((pref >> (3 * bb + 2)) & 1) << bb
            ic[1] |= ((pref >> (3 * bb + 1)) & 1) << bb
            ic[2] |= ((pref >> (3 * bb)) & 1) << bb
        ctr[i] = pl.x0 + (np.array(ic) + 0.5) * side[i]
    d = np.linalg.norm(ctr[m2l[:, 0]] - ctr[m2l[:, 1]], axis=1)
    assert np.all(theta * d >= 0.5 * (side[m2l[:, 0]] + side[m2l[:, 1]]) * (1 - 1e-6))
    assert np.all(c["count"][c["leaf"] == 1] <= ncrit)
    # every point lies in its leaf's box
    order, _ = pl.order()
    leaf = np.nonzero(c["leaf"])[0]
    for li in leaf:
        pts = pl.points[order[c["start"][li]:c["start"][li] + c["count"][li]]]
        assert np.all(np.abs(pts - ctr[li]) <= side[li] / 2 + 1e-12)


def _golden_counts():
    rows = {}
    with open(f"{ROOT_GOLDEN}/interaction_list_counts.txt") as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                t, m, nn, k = line.split()
                rows[float(t)] = (int(m), int(nn), int(k))
    return rows


@pytest.mark.parametrize("theta", [0.5, 0.4])
def test_interior_list_counts_match_paper(theta):
    """Uniform 16^3 lattice, one point per finest box: interior boxes have the
    paper's 189-source list at theta=1/2 (Sec. 2.2) and 567 at theta=0.4."""
    m_exp, near_exp, keys_exp = _golden_counts()[theta]
    g = (np.arange(16) + 0.5) / 16
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pl = oracle.Plan(x, 1, theta)
    c = pl.cells()
    m2l, p2p = pl.pairs()
    lev = c["level"]
    assert lev.max() == 4 and np.all(c["leaf"][lev == 4] == 1) and np.sum(lev == 4) == 4096
    # box coordinates at level 4
    def coords(i):
        pref = int(c["prefix"][i]); ic = [0, 0, 0]
        for bb in range(4):
            ic[0] |= ((pref >> (3 * bb + 2)) & 1) << bb
            ic[1] |= ((pref >> (3 * bb + 1)) & 1) << bb
            ic[2] |= ((pref >> (3 * bb)) & 1) << bb
        return np.array(ic)
    l4 = np.nonzero(lev == 4)[0]
    co = {i: coords(i) for i in l4}
    lo, hi = (2, 13) if theta == 0.5 else (4, 11)
    interior = [i for i in l4 if np.all(co[i] >= lo) and np.all(co[i] <= hi)]
    nm = np.bincount(m2l[:, 0], minlength=pl.ncells)
    npp = np.bincount(p2p[:, 0], minlength=pl.ncells)
    assert all(nm[i] == m_exp for i in interior)
    assert all(npp[i] == near_exp for i in interior)
    assert max(nm[i] for i in l4) == m_exp
    sel = (lev[m2l[:, 0]] == 4) & (lev[m2l[:, 1]] == 4)
    offs = {tuple(co[a] - co[b]) for a, b in m2l[sel]}
    assert len(offs) == keys_exp


def test_root_cube_is_the_closed_box():
    """Points on the upper face of [0,1]^3 keep the unit root cube (they sit in the closure of
    the last cell); a cloud one ulp wider doubles it.  The lists still cover every pair once."""
    g = np.arange(17) / 16.0                      # includes 0 and 1
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pl = oracle.Plan(x, 4, 0.5)
    assert pl.k == 0 and np.all(pl.x0 == 0.0)
    cov = _coverage(pl)
    assert cov.min() == 1 and cov.max() == 1
    c = pl.cells()
    order, _ = pl.order()
    side = 2.0 ** (pl.k - c["level"].astype(np.float64))
    for li in np.nonzero(c["leaf"])[0]:
        l, pref = int(c["level"][li]), int(c["prefix"][li])
        ic = [sum(((pref >> (3 * bb + 2 - a)) & 1) << bb for bb in range(l)) for a in range(3)]
        ctr = (np.array(ic) + 0.5) * side[li]
        pts = x[order[c["start"][li]:c["start"][li] + c["count"][li]]]
        assert np.all(np.abs(pts - ctr) <= side[li] / 2)
    y = x.copy()
    y[-1, 0] = np.nextafter(1.0, 2.0)
    assert oracle.Plan(y, 4, 0.5).k == 1


@pytest.mark.parametrize("dist,theta,ncrit", [("cube", 0.4, 16), ("plummer", 0.5, 10), ("sphere", 0.35, 12)])
def test_level_skip_lists_cover_every_pair_once(dist, theta, ncrit):
    """Level skip (one cell of a same-level pair split at a time): still an exact partition
    of all ordered point pairs, symmetric, the MAC holds for every M2L pair (including the
    mixed-level ones it creates), and fewer M2L pairs than the dual traversal."""
    x, q = inputs.make(dist, 1500, 23)
    pl = oracle.Plan(x.astype(np.float64), ncrit, theta, lists=1)
    cov = _coverage(pl)
    assert cov.min() == 1 and cov.max() == 1
    m2l, p2p = pl.pairs()
    s1 = set(map(tuple, m2l)); s2 = set(map(tuple, p2p))
    assert s1 == {(b, a) for a, b in s1} and s2 == {(b, a) for a, b in s2}
    c = pl.cells()
    side = 2.0 ** (pl.k - c["level"].astype(np.float64))
    ctr = np.zeros((pl.ncells, 3))
    for i in range(pl.ncells):
        l, pref = int(c["level"][i]), int(c["prefix"][i])
        ic = [sum(((pref >> (3 * bb + 2 - a)) & 1) << bb for bb in range(l)) for a in range(3)]
        ctr[i] = pl.x0 + (np.array(ic) + 0.5) * side[i]
    d = np.linalg.norm(ctr[m2l[:, 0]] - ctr[m2l[:, 1]], axis=1)
    assert np.all(theta * d >= 0.5 * (side[m2l[:, 0]] + side[m2l[:, 1]]) * (1 - 1e-6))
    assert np.any(c["level"][m2l[:, 0]] != c["level"][m2l[:, 1]])
    assert pl.nm2l < oracle.Plan(x.astype(np.float64), ncrit, theta).nm2l


def test_level_skip_fmm_converges():
    x, q = inputs.make("cube", 3000, 24)
    x = x.astype(np.float64); q = q.astype(np.float64)
    pl = oracle.Plan(x, 16, 0.4, lists=1)
    ref, _ = oracle.direct(x, q)
    errs = []
    for p in (4, 8, 12):
        phi, _, _ = pl.eval(q, p)
        errs.append(np.linalg.norm(phi - ref) / np.linalg.norm(ref))
    assert errs[2] < 1e-6 and errs[2] < errs[1] < errs[0]


# ---------------------------------------------------------------- Hessian (losses through grad phi)
def test_direct_hessian_closed_form_and_laplace():
    """Two bodies: H = q (3 d d^T - |d|^2 I) / |d|^5; any cloud: H symmetric by layout and
    traceless away from the sources (phi is harmonic)."""
    x = np.array([[0.1, 0.2, 0.3], [0.7, -0.5, 1.3]])
    q = np.array([0.0, 2.5])
    h = oracle.direct_hessian(x, q)[0]
    d = x[0] - x[1]
    r = np.linalg.norm(d)
    H = 2.5 * (3 * np.outer(d, d) - r * r * np.eye(3)) / r ** 5
    assert np.allclose(h, [H[0, 0], H[1, 1], H[2, 2], H[0, 1], H[0, 2], H[1, 2]], rtol=1e-13,
                       atol=1e-14 * np.abs(H).max())
    x, q = inputs.make("plummer", 400, 31)
    hh = oracle.direct_hessian(x.astype(np.float64), q.astype(np.float64))
    scale = np.abs(hh).max(axis=1)
    assert np.all(np.abs(hh[:, 0] + hh[:, 1] + hh[:, 2]) <= 1e-9 * scale)


def test_direct_hessian_is_the_derivative_of_the_gradient():
    x, q = inputs.make("cube", 300, 32)
    x = x.astype(np.float64); q = q.astype(np.float64)
    t = np.array([5, 77, 200])
    h = oracle.direct_hessian(x, q, t)
    eps = 1e-5
    for a, (i, j) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
        for r, ti in enumerate(t):                 # one target moved at a time
            xp = x.copy(); xm = x.copy()
            xp[ti, j] += eps; xm[ti, j] -= eps
            gp = oracle.direct(xp, q, [ti])[1]; gm = oracle.direct(xm, q, [ti])[1]
            fd = (gp[0, i] - gm[0, i]) / (2 * eps)
            assert abs(h[r, a] - fd) <= 1e-6 * np.abs(h[r]).max()


def test_fmm_hessian_converges_to_direct():
    x, q = inputs.make("cube", 3000, 33)
    x = x.astype(np.float64); q = q.astype(np.float64)
    pl = oracle.Plan(x, 16, 0.4)
    ref = oracle.direct_hessian(x, q)
    errs = []
    for p in (4, 8, 12):
        _, _, _, h = pl.eval(q, p, hessian=True)
        errs.append(np.linalg.norm(h - ref) / np.linalg.norm(ref))
    assert errs[2] < 1e-5 and errs[2] < errs[1] < errs[0]


def _grad_loss_adjoint_direct(x, q, w, g):
    """dL/dq and dL/dx of L = sum w phi + sum g . grad phi, from exact direct sums:
    dL/dq_j = psi_j + chi_j, chi_j = -sum_a d_a phi^(g_a)(x_j);
    dL/dx_k = w_k E_k + q_k grad psi_k + H_k g_k - q_k sum_a H^(g_a)_k e_a."""
    idx = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]

    def full(h):
        H = np.zeros((h.shape[0], 3, 3))
        for a, (i, j) in enumerate(idx):
            H[:, i, j] = H[:, j, i] = h[:, a]
        return H
    psi, gpsi = oracle.direct(x, w)
    _, E = oracle.direct(x, q)
    H = full(oracle.direct_hessian(x, q))
    dq = psi.copy()
    dx = w[:, None] * E + q[:, None] * gpsi + np.einsum("kab,kb->ka", H, g)
    for a in range(3):
        _, ga = oracle.direct(x, g[:, a])
        dq -= ga[:, a]
        Ha = full(oracle.direct_hessian(x, g[:, a]))
        dx -= q[:, None] * Ha[:, :, a]
    return dq, dx


def test_adjoint_through_grad_phi_matches_finite_differences():
    """The adjoint formula for losses through grad phi, checked on the exact loss."""
    rng = np.random.default_rng(34)
    n = 60
    x = rng.random((n, 3)); q = rng.uniform(-1, 1, n); w = rng.standard_normal(n); g = rng.standard_normal((n, 3))

    def loss(xx, qq):
        phi, E = oracle.direct(xx, qq)
        return float(np.dot(w, phi) + np.sum(g * E))
    dq, dx = _grad_loss_adjoint_direct(x, q, w, g)
    eps = 1e-6
    for j in (0, 17, 59):
        qp = q.copy(); qp[j] += eps; qm = q.copy(); qm[j] -= eps
        assert abs((loss(x, qp) - loss(x, qm)) / (2 * eps) - dq[j]) <= 1e-6 * (1 + abs(dq[j]))
        for a in range(3):
            xp = x.copy(); xp[j, a] += eps; xm = x.copy(); xm[j, a] -= eps
            fd = (loss(xp, q) - loss(xm, q)) / (2 * eps)
            assert abs(fd - dx[j, a]) <= 1e-5 * (1 + abs(dx[j, a]))


def test_adjoint_through_grad_phi_with_dipoles_matches_finite_differences():
    """The same adjoint in two evaluations: dL/dq = Psi and dL/dx = w grad phi + H g +
    q grad Psi, Psi the field of charges w and dipoles g (a dipole g_i at x_i is the
    derivative of a unit charge's field as it moves along g_i); checked on the exact loss."""
    rng = np.random.default_rng(35)
    n = 60
    x = rng.random((n, 3)); q = rng.uniform(-1, 1, n); w = rng.standard_normal(n); g = rng.standard_normal((n, 3))
    full = lambda h: np.stack([np.stack([h[:, 0], h[:, 3], h[:, 4]], 1), np.stack([h[:, 3], h[:, 1], h[:, 5]], 1),
                               np.stack([h[:, 4], h[:, 5], h[:, 2]], 1)], 1)

    def loss(xx, qq):
        phi, E = oracle.direct(xx, qq)
        return float(np.dot(w, phi) + np.sum(g * E))
    psi, gpsi = oracle.direct_dip(x, w, g)
    _, E = oracle.direct(x, q)
    H = full(oracle.direct_hessian(x, q))
    dq = psi
    dx = w[:, None] * E + np.einsum("kab,kb->ka", H, g) + q[:, None] * gpsi
    eps = 1e-6
    for j in (0, 23, 59):
        qp = q.copy(); qp[j] += eps; qm = q.copy(); qm[j] -= eps
        assert abs((loss(x, qp) - loss(x, qm)) / (2 * eps) - dq[j]) <= 1e-6 * (1 + abs(dq[j]))
        for a in range(3):
            xp = x.copy(); xp[j, a] += eps; xm = x.copy(); xm[j, a] -= eps
            fd = (loss(xp, q) - loss(xm, q)) / (2 * eps)
            assert abs(fd - dx[j, a]) <= 1e-5 * (1 + abs(dx[j, a]))


# ---- separate target set ------------------------------------------------------

def test_direct_targets_closed_form_and_brute_force():
    """One unit source at the origin: phi = 1/r, grad = -y/r^3 (closed form); a target on a
    source skips it; small random sets against a broadcast sum written out here."""
    phi, grad = oracle.direct_targets(np.zeros((1, 3)), np.array([2.0]),
                                      np.array([[3.0, 0, 4.0], [0, 0, 0], [1.0, 2.0, 2.0]]))
    assert np.allclose(phi, [2 / 5, 0.0, 2 / 3], rtol=1e-15, atol=0)
    assert np.allclose(grad[0], [-2 * 3 / 125, 0, -2 * 4 / 125], rtol=1e-15)
    assert np.all(grad[1] == 0)
    rng = np.random.default_rng(5)
    x, q, y = rng.random((40, 3)), rng.standard_normal(40), rng.random((25, 3))
    y[3] = x[7]                     # a target on a source
    d = y[:, None, :] - x[None, :, :]
    r = np.sqrt((d * d).sum(-1))
    inv = np.where(r > 0, 1 / np.where(r > 0, r, 1), 0.0)
    ephi = (q[None, :] * inv).sum(1)
    egrad = -(q[None, :, None] * d * inv[:, :, None] ** 3).sum(1)
    phi, grad = oracle.direct_targets(x, q, y)
    assert np.allclose(phi, ephi, rtol=1e-13, atol=0) and np.allclose(grad, egrad, rtol=1e-12, atol=1e-12)


def test_union_fmm_at_targets_converges_to_direct_targets():
    """The oracle FMM on the union (zero target charges), sampled at the target rows,
    approaches the two-set direct sum geometrically in p."""
    x, q = inputs.make("plummer", 3000, 61)
    y, _ = inputs.make("cube", 2000, 62)
    xd, yd, qd = x.astype(np.float64), y.astype(np.float64), q.astype(np.float64)
    ephi, egrad = oracle.direct_targets(xd, qd, yd)
    plan = oracle.Plan(np.concatenate([xd, yd]), 32, 0.4)
    qu = np.concatenate([qd, np.zeros(len(yd))])
    errs = []
    for p in (4, 8):
        phi, grad, _ = plan.eval(qu, p, sample=np.arange(3000, 5000))
        errs.append(np.linalg.norm(phi - ephi) / np.linalg.norm(ephi))
    assert errs[1] < 1e-4 and errs[1] < errs[0] / 10


def test_two_set_adjoint_reduction_matches_finite_differences():
    """L = sum_t w_t phi(y_t) for separate sources x (charges q) and targets y.  Its exact
    derivatives by central differences of the direct sum against the one-set adjoint on the
    union with charges [q; 0] and weights [0; w]: dL/dq = psi(x), dL/dx = q grad psi(x),
    dL/dy = w grad phi(y), psi the field of the weights."""
    rng = np.random.default_rng(17)
    x, q = rng.random((12, 3)), rng.standard_normal(12)
    y, w = rng.random((9, 3)) + 0.05, rng.standard_normal(9)

    def loss(xx, qq, yy):
        return float(np.dot(w, oracle.direct_targets(xx, qq, yy)[0]))

    union = np.concatenate([x, y])
    psi, gpsi = oracle.direct(union, np.concatenate([np.zeros(12), w]))
    _, gphi = oracle.direct(union, np.concatenate([q, np.zeros(9)]))
    dq, dx, dy = psi[:12], q[:, None] * gpsi[:12], w[:, None] * gphi[12:]
    h = 1e-5
    for j in range(12):
        qp, qm = q.copy(), q.copy()
        qp[j] += h
        qm[j] -= h
        assert (loss(x, qp, y) - loss(x, qm, y)) / (2 * h) == pytest.approx(dq[j], rel=1e-7, abs=1e-9)
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[j, a] += h
            xm[j, a] -= h
            assert (loss(xp, q, y) - loss(xm, q, y)) / (2 * h) == pytest.approx(dx[j, a], rel=1e-5, abs=1e-7)
    for t in range(9):
        for a in range(3):
            yp, ym = y.copy(), y.copy()
            yp[t, a] += h
            ym[t, a] -= h
            assert (loss(x, q, yp) - loss(x, q, ym)) / (2 * h) == pytest.approx(dy[t, a], rel=1e-5, abs=1e-7)
