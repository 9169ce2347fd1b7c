"""Shared helpers of the GPU tests: plan comparison and error norms."""
import numpy as np


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def cell_ids(level, prefix):
    """Unique 64-bit identity of (level, Morton prefix): a leading 1 bit above the prefix."""
    level = np.asarray(level, np.uint64)
    return (np.uint64(1) << (np.uint64(3) * level)) | np.asarray(prefix, np.uint64)


def compare_plans(gpu, ora_plan, keep=None):
    """Assert the GPU plan (export dict) and the oracle plan hold identical cells, order and
    lists (with `keep`, only the oracle pairs for which keep(pairs) is True)."""
    oc = ora_plan.cells()
    om2l, op2p = ora_plan.pairs()
    if keep is not None:
        om2l, op2p = om2l[keep(om2l)], op2p[keep(op2p)]
    oorder, _ = ora_plan.order()
    assert np.array_equal(gpu["order"], oorder), "sorted order differs"
    gid = cell_ids(gpu["level"], gpu["prefix"])
    oid = cell_ids(oc["level"], oc["prefix"])
    gs = np.argsort(gid)
    os_ = np.argsort(oid)
    assert np.array_equal(gid[gs], oid[os_]), "cell sets differ"
    for f in ("start", "count", "leaf"):
        assert np.array_equal(np.asarray(gpu[f])[gs].astype(np.int64), np.asarray(oc[f])[os_].astype(np.int64)), f

    def pair_ids(ids, pairs):
        if len(pairs) == 0:
            return np.zeros((0, 2), np.uint64)
        p = np.stack([ids[pairs[:, 0]], ids[pairs[:, 1]]], 1)
        o = np.lexsort((p[:, 1], p[:, 0]))
        return p[o]

    for name, gp, opr in (("m2l", gpu["m2l"], om2l), ("p2p", gpu["p2p"], op2p)):
        a, b = pair_ids(gid, gp), pair_ids(oid, opr)
        assert a.shape == b.shape, f"{name} pair counts differ: {a.shape[0]} vs {b.shape[0]}"
        assert np.array_equal(a, b), f"{name} pair sets differ"
