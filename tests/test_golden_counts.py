"""The stored interaction-list counts are reproducible from committed code.

tests/golden/count_lists.py derives them by integer counting from the MAC and the
dual-traversal rule; here they are regenerated and compared with the stored files,
pinned to the classical list of Sec. 2.2 (189 = 6^3 - 3^3 sources per box at
theta = 1/2), and the level-by-level counting is checked against brute force over
every cell pair of small complete octrees.
"""
import itertools

import numpy as np
import pytest

from golden import count_lists as cl


def test_stored_files_are_what_the_script_writes():
    for name, text in (("interaction_list_counts.txt", cl.interior_text()),
                       ("complete_tree_counts.txt", cl.complete_text())):
        with open(f"{cl.HERE}/{name}") as f:
            assert f.read() == text


def test_classical_list_of_the_paper():
    m2l, near, keys = cl.interior_box(0.5)
    assert m2l == 6 ** 3 - 3 ** 3 == 189
    assert near == 3 ** 3
    # the 316 offsets are the 7^3 cube of parent-neighbour children minus the 3^3 near cube
    assert keys == 7 ** 3 - 3 ** 3 == 316


def _brute(depth, theta):
    """Dual traversal of a complete octree written out over explicit cell coordinates:
    a pair of level l is considered iff its parent pair was considered and failed."""
    t2 = float(cl.theta_sq(theta))
    considered = np.zeros((1, 1), bool)
    considered[0, 0] = True
    m2l = near = 0
    keys = set()
    for lev in range(depth + 1):
        side = 2 ** lev
        ijk = np.array(list(itertools.product(range(side), repeat=3)))
        d = ijk[None, :, :] - ijk[:, None, :]
        n2 = (d * d).sum(-1)
        acc = (n2 > 0) & (t2 * n2 >= 1)
        if lev > 0:
            par = ijk // 2
            pid = (par[:, 0] * (side // 2) + par[:, 1]) * (side // 2) + par[:, 2]
            considered = prev_failed[pid][:, pid]
        m2l += int((considered & acc).sum())
        for v in np.unique(d[considered & acc].reshape(-1, 3), axis=0):
            keys.add(tuple(v))
        prev_failed = considered & ~acc
        if lev == depth:
            near = int(prev_failed.sum())
    return sum(8 ** l for l in range(depth + 1)), m2l, near, len(keys)


@pytest.mark.parametrize("depth", [1, 2, 3])
@pytest.mark.parametrize("theta", [0.5, 0.4, 0.3])
def test_level_recursion_equals_brute_force(depth, theta):
    assert cl.complete_tree(depth, theta) == _brute(depth, theta)


def test_pairs_of_a_complete_tree_are_all_pairs():
    # every ordered pair of leaves of a complete tree is covered once: by a near pair or
    # by an M2L pair of ancestors (each M2L pair at level l covers 8^(depth-l) squared)
    depth, theta = 4, 0.4
    t2 = cl.theta_sq(theta)
    mult = {-1: 1, 0: 2, 1: 1}
    level = {(0, 0, 0): 1}
    covered = 0
    for lev in range(depth + 1):
        nxt = {}
        for d, c in level.items():
            if cl.accepts(d, t2):
                covered += c * 64 ** (depth - lev)
            elif lev == depth:
                covered += c
            else:
                for s in itertools.product((-1, 0, 1), repeat=3):
                    k = (2 * d[0] + s[0], 2 * d[1] + s[1], 2 * d[2] + s[2])
                    nxt[k] = nxt.get(k, 0) + c * mult[s[0]] * mult[s[1]] * mult[s[2]]
        level = nxt
    assert covered == (8 ** depth) ** 2
