"""Randomised checks of the oracle's plan and FMM on small, awkward point clouds
(clusters, planes, lines, duplicates, wide dynamic range), and of the seeded inputs."""
import os
import secrets

import numpy as np
import pytest
from hypothesis import HealthCheck, given, seed, settings
from hypothesis import strategies as st

import oracle
from paper_1602_02244_amd import inputs


def _cloud(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "cube":
        x = rng.random((n, 3))
    elif kind == "clusters":
        c = rng.random((4, 3)) * 100.0
        x = c[rng.integers(0, 4, n)] + rng.normal(scale=1e-3, size=(n, 3))
    elif kind == "plane":
        x = rng.random((n, 3))
        x[:, 2] = 0.5
    elif kind == "line":
        t = rng.random(n)
        x = np.stack([t, 2 * t, -t], 1)
    elif kind == "dups":
        base = rng.random((max(1, n // 4), 3))
        x = base[rng.integers(0, base.shape[0], n)]
    else:
        x = rng.standard_normal((n, 3)) * 1e4 + 1e5
    return x.astype(np.float32).astype(np.float64)


@settings(max_examples=25, deadline=None, suppress_health_check=[HealthCheck.too_slow], derandomize=True)
@given(kind=st.sampled_from(["cube", "clusters", "plane", "line", "dups", "far"]),
       n=st.integers(2, 700), ncrit=st.integers(1, 40), theta=st.sampled_from([0.3, 0.4, 0.5]),
       seed=st.integers(0, 10 ** 6), lists=st.sampled_from([0, 1]))
def test_pairs_partition_all_interactions(kind, n, ncrit, theta, seed, lists):
    x = _cloud(kind, n, seed)
    pl = oracle.Plan(x, ncrit, theta, lists)
    c = pl.cells()
    m2l, p2p = pl.pairs()
    cov = np.zeros((n, n), np.int16)
    for a, b in np.concatenate([m2l, p2p]):
        cov[c["start"][a]:c["start"][a] + c["count"][a], c["start"][b]:c["start"][b] + c["count"][b]] += 1
    assert cov.min() == 1 and cov.max() == 1
    # leaves hold at most ncrit bodies unless they sit at the deepest level
    leaf = c["leaf"] == 1
    assert np.all((c["count"][leaf] <= ncrit) | (c["level"][leaf] == 21))
    # children partition their parent's range
    for i in range(pl.ncells):
        ch = np.nonzero(c["parent"] == i)[0]
        if ch.size:
            assert c["count"][ch].sum() == c["count"][i]


@settings(max_examples=12, deadline=None, derandomize=True)
@given(kind=st.sampled_from(["cube", "clusters", "plane", "dups"]), n=st.integers(50, 900),
       seed=st.integers(0, 10 ** 6))
def test_fmm_close_to_direct(kind, n, seed):
    """The truncation error falls like (sqrt(3) theta)^p (0.69 per order at theta = 0.4) with a
    cloud-dependent constant: a duplicate-heavy cloud (420 points, 104 distinct) has a 2.3e-4
    gradient error at p = 8 and 1.2e-5 at p = 12.  p = 12 keeps every cloud below 1e-4, and
    the error must shrink from p = 6 to p = 12 at no worse than that rate."""
    x = _cloud(kind, n, seed)
    q = np.random.default_rng(seed + 1).uniform(-1, 1, n)
    pl = oracle.Plan(x, 16, 0.4)
    ref, gref = oracle.direct(x, q)
    err = {}
    for p in (6, 12):
        phi, grad, _ = pl.eval(q, p)
        err[p] = (np.linalg.norm(phi - ref) / np.linalg.norm(ref), np.linalg.norm(grad - gref) / np.linalg.norm(gref))
    assert max(err[12]) <= 1e-4
    rate = (np.sqrt(3) * 0.4) ** 6
    for i in range(2):
        assert err[12][i] <= 2 * rate * err[6][i] + 1e-12


def test_partition_and_accuracy_fresh_examples(capsys):
    """The two checks above on examples drawn afresh at every run (not derandomized).
    The seed is printed; FMM_FUZZ_SEED=<seed> replays a run."""
    s = int(os.environ.get("FMM_FUZZ_SEED", secrets.randbits(32)))
    with capsys.disabled():
        print(f"\n[fuzz] hypothesis seed {s} (replay: FMM_FUZZ_SEED={s})")

    @seed(s)
    @settings(max_examples=8, deadline=None, database=None, suppress_health_check=[HealthCheck.too_slow])
    @given(kind=st.sampled_from(["cube", "clusters", "plane", "line", "dups", "far"]),
           n=st.integers(2, 500), ncrit=st.integers(1, 40), theta=st.sampled_from([0.3, 0.4, 0.5]),
           cseed=st.integers(0, 10 ** 6), lists=st.sampled_from([0, 1]))
    def partition(kind, n, ncrit, theta, cseed, lists):
        test_pairs_partition_all_interactions.hypothesis.inner_test(kind, n, ncrit, theta, cseed, lists)

    @seed(s + 1)
    @settings(max_examples=4, deadline=None, database=None)
    @given(kind=st.sampled_from(["cube", "clusters", "plane", "dups"]), n=st.integers(50, 600),
           cseed=st.integers(0, 10 ** 6))
    def accuracy(kind, n, cseed):
        test_fmm_close_to_direct.hypothesis.inner_test(kind, n, cseed)

    partition()
    accuracy()


def test_inputs_are_seeded_and_shaped():
    a = inputs.workload("uniform-4k")
    b = inputs.workload("uniform-4k")
    assert np.array_equal(a[0], b[0]) and a[0].dtype == np.float32 and a[0].shape == (4096, 3)
    x, q = inputs.make("plummer", 20000, 3)
    r = np.linalg.norm(x.astype(np.float64), axis=1)
    assert r.max() <= 10.0 + 1e-5 and np.all(q > 0) and np.all(q <= 1)
    # half-mass radius of a Plummer sphere (scale 1) is about 1.305 (truncation at r = 10 shifts it slightly)
    assert 1.2 < np.median(r) < 1.4
    x, q = inputs.make("sphere", 5000, 4)
    assert np.allclose(np.linalg.norm(x.astype(np.float64), axis=1), 1.0, atol=1e-6)
    x, q = inputs.make("cube", 5000, 5)
    assert x.min() >= 0 and x.max() < 1 and q.min() >= -1 and q.max() <= 1
    idx, ax = inputs.fd_coordinates(1000)
    assert idx.shape == (64,) and set(np.unique(ax)) <= {0, 1, 2}
