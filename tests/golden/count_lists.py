"""Interaction-list counts of uniform octrees, by integer counting alone.

Writes (with --write) or prints the expected values that the tests compare against:

* interaction_list_counts.txt -- per interior box of a deep uniform octree: the number of
  M2L sources, of near boxes (self included) and of distinct same-level offsets taken
  over the eight child positions (Sec. 2.2 gives 189 = 6^3 - 3^3 for the classical list);
* complete_tree_counts.txt -- totals of a complete octree whose leaves all sit at one
  depth: cells, M2L pairs, near (P2P) leaf pairs and distinct offsets.

Nothing here runs an FMM or a tree builder.  The counts follow from three facts:
the MAC theta |c_A - c_B| >= R_A + R_B with R the half side, which for two cells of one
level and integer offset d (in cell sides) reads theta^2 |d|^2 >= 1 (never for d = 0);
the dual traversal of a complete tree, where a same-level pair that fails the MAC is
replaced by its 64 child pairs (a leaf pair that fails is a near pair); and the
child-pair offsets of a parent pair with offset D, which are 2D + (b - a) for the child
positions a, b in {0,1}^3, so along one axis the child offset 2D arises in two ways and
2D - 1, 2D + 1 in one way each.  theta is taken as the FP32 value the library receives,
compared exactly with rational arithmetic.
"""
import argparse
import itertools
import os
from collections import defaultdict
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
THETAS = (0.5, 0.4)


def theta_sq(theta):
    """theta^2 as an exact rational of the FP32 value."""
    t = Fraction(float(np.float32(theta)))
    return t * t


def accepts(d, t2):
    """MAC between two cells of one level at integer offset d (in cell sides)."""
    n2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
    return n2 > 0 and t2 * n2 >= 1


def interior_box(theta):
    """(M2L sources, near boxes, distinct offsets) of an interior box: the children of
    the parent's failing neighbours (offsets D, self included) that pass the MAC, over
    every child position a of the target in its parent."""
    t2 = theta_sq(theta)
    r = int((1 / t2) ** 0.5) + 2
    fail = [D for D in itertools.product(range(-r, r + 1), repeat=3) if not accepts(D, t2)]
    bits = list(itertools.product((0, 1), repeat=3))
    per_pos, offsets = [], set()
    for a in bits:
        m2l = near = 0
        for D in fail:
            for b in bits:
                d = tuple(2 * D[i] + b[i] - a[i] for i in range(3))
                if accepts(d, t2):
                    m2l += 1
                    offsets.add(d)
                else:
                    near += 1
        per_pos.append((m2l, near))
    assert len(set(per_pos)) == 1, "every child position has the same list sizes"
    return per_pos[0][0], per_pos[0][1], len(offsets)


def complete_tree(depth, theta):
    """(cells, M2L pairs, near leaf pairs, distinct offsets) of the dual traversal of a
    complete octree with every leaf at `depth`: the number of considered pairs per
    offset is carried from level to level."""
    t2 = theta_sq(theta)
    mult = {-1: 1, 0: 2, 1: 1}
    level = {(0, 0, 0): 1}            # the pair (root, root)
    m2l = near = 0
    keys = set()
    for lev in range(depth + 1):
        failed = {}
        for d, c in level.items():
            if accepts(d, t2):
                m2l += c
                keys.add(d)
            else:
                failed[d] = c
        if lev == depth:
            near = sum(failed.values())
            break
        nxt = defaultdict(int)
        for D, c in failed.items():
            for s in itertools.product((-1, 0, 1), repeat=3):
                w = mult[s[0]] * mult[s[1]] * mult[s[2]]
                nxt[(2 * D[0] + s[0], 2 * D[1] + s[1], 2 * D[2] + s[2])] += c * w
        level = nxt
    cells = sum(8 ** l for l in range(depth + 1))
    return cells, m2l, near, len(keys)


def interior_text():
    rows = ["# Steady-state interaction-list sizes of an interior box in a uniform octree.",
            "#",
            "# Sec. 2.2 gives 189 = 6^3 - 3^3 source boxes per target box for the classical list",
            "# (theta = 1/2 under the MAC theta |dc| >= R_A + R_B).  Written by",
            "# tests/golden/count_lists.py (integer counting:",
            "# children of the parent's failing neighbours that pass the MAC; offsets over the",
            "# eight child positions).",
            "# theta  m2l_per_interior_box  near_per_interior_box  distinct_offsets"]
    for th in THETAS:
        m, nb, k = interior_box(th)
        rows.append(f"{th} {m} {nb} {k}")
    return "\n".join(rows) + "\n"


def complete_text(depths=(5,)):
    rows = ["# Dual-traversal totals of a complete octree, every leaf at one depth (the uniform",
            "# 2^20-point cube at ncrit 64 has all leaves at depth 5).  Written by",
            "# tests/golden/count_lists.py from the MAC and the child-pair offsets alone.",
            "# depth  theta  cells  m2l_pairs  near_leaf_pairs  distinct_offsets"]
    for dep in depths:
        for th in THETAS:
            c, m, nn, k = complete_tree(dep, th)
            rows.append(f"{dep} {th} {c} {m} {nn} {k}")
    return "\n".join(rows) + "\n"


def read_table(name):
    """Rows of a golden file as tuples of numbers (comments skipped)."""
    out = []
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                out.append(tuple(float(v) if "." in v else int(v) for v in line.split()))
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--write", action="store_true", help="rewrite the two golden files")
    a = ap.parse_args()
    texts = {"interaction_list_counts.txt": interior_text(), "complete_tree_counts.txt": complete_text()}
    for name, text in texts.items():
        if a.write:
            with open(os.path.join(HERE, name), "w") as f:
                f.write(text)
        print(text, end="")
