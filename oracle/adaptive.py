"""TEST INFRASTRUCTURE ONLY: the oracle's own adaptive octree builder.

Sec. 2.4: every node of the octree carries one 8x8x8 sub-grid and is either a
leaf or refined into 8 children, and the sub-grids are properly nested: across
any sub-grid boundary (faces, edges and corners) the refinement level changes
by at most one.  Refinement here follows the density criterion used for the
binary runs (Sec. 2.7) in a fixed-threshold form: a node at level l < max_level
is refined when the maximum density over its cube exceeds the threshold; nodes
are then refined further until the nesting rule holds.  The balanced tree is
the smallest one containing the density refinement, so it does not depend on
the order in which violations are repaired.

Plain Python sets; meant for trees of up to some tens of thousands of nodes.
"""
from __future__ import annotations

import itertools

import numpy as np

_DIRS = [d for d in itertools.product((-1, 0, 1), repeat=3) if d != (0, 0, 0)]


def _cube(level, nodes):
    w = 1.0 / (1 << level)
    a = np.asarray(nodes, dtype=np.float64).reshape(-1, 3)
    lo = a * w - 0.5
    return lo, lo + w


def build_adaptive_leaves(boxmax, max_level: int, threshold: float) -> np.ndarray:
    """Leaf list (level, nx, ny, nz), sorted by level then index.

    boxmax(lo, hi) -> max density over each box (arrays n x 3)."""
    interior = [set() for _ in range(max_level + 1)]
    # density criterion, level by level
    current = [(0, 0, 0)]
    for lev in range(max_level):
        if not current:
            break
        lo, hi = _cube(lev, current)
        bm = np.asarray(boxmax(lo, hi), dtype=np.float64)
        refine = [n for n, v in zip(current, bm) if v > threshold]
        interior[lev].update(refine)
        current = [(2 * x + a, 2 * y + b, 2 * z + c) for (x, y, z) in refine
                   for a in (0, 1) for b in (0, 1) for c in (0, 1)]

    def exists(lev, n):
        if lev == 0:
            return n == (0, 0, 0)
        m = 1 << lev
        if not all(0 <= v < m for v in n):
            return False
        return (n[0] >> 1, n[1] >> 1, n[2] >> 1) in interior[lev - 1]

    # proper nesting: a leaf may not touch an interior node one level finer
    changed = True
    while changed:
        changed = False
        for lev in range(max_level - 1, -1, -1):
            finer = interior[lev + 1] if lev + 1 <= max_level else set()
            if not finer:
                continue
            # candidate leaves at lev: parents of finer-interior nodes' neighbours
            cands = set()
            for (x, y, z) in finer:
                for dx, dy, dz in _DIRS + [(0, 0, 0)]:
                    cands.add(((x + dx) >> 1, (y + dy) >> 1, (z + dz) >> 1))
            for n in cands:
                if n in interior[lev] or not exists(lev, n):
                    continue
                bx, by, bz = 2 * n[0], 2 * n[1], 2 * n[2]
                bad = False
                for mx in range(bx - 1, bx + 3):
                    for my in range(by - 1, by + 3):
                        for mz in range(bz - 1, bz + 3):
                            if bx <= mx <= bx + 1 and by <= my <= by + 1 and bz <= mz <= bz + 1:
                                continue
                            if (mx, my, mz) in finer:
                                bad = True
                                break
                        if bad:
                            break
                    if bad:
                        break
                if bad:
                    interior[lev].add(n)
                    changed = True
    leaves = []
    for lev in range(max_level + 1):
        if lev == 0:
            nodes = [(0, 0, 0)]
        else:
            nodes = [(2 * x + a, 2 * y + b, 2 * z + c) for (x, y, z) in interior[lev - 1]
                     for a in (0, 1) for b in (0, 1) for c in (0, 1)]
        for n in nodes:
            if n not in interior[lev]:
                leaves.append((lev,) + tuple(n))
    leaves.sort()
    return np.asarray(leaves, dtype=np.int32).reshape(-1, 4)


def is_balanced(leaves) -> bool:
    """True if no two touching leaves differ by more than one level (checked
    on the finest grid by brute force; for small trees)."""
    leaves = np.asarray(leaves).reshape(-1, 4)
    top = int(leaves[:, 0].max())
    n = 1 << top
    lvl = -np.ones((n, n, n), dtype=np.int32)
    for l, x, y, z in leaves:
        s = 1 << (top - l)
        lvl[x * s:(x + 1) * s, y * s:(y + 1) * s, z * s:(z + 1) * s] = l
    if (lvl < 0).any():
        return False
    for dx, dy, dz in _DIRS:
        a = lvl[max(dx, 0):n + min(dx, 0), max(dy, 0):n + min(dy, 0), max(dz, 0):n + min(dz, 0)]
        b = lvl[max(-dx, 0):n + min(-dx, 0), max(-dy, 0):n + min(-dy, 0), max(-dz, 0):n + min(-dz, 0)]
        if (np.abs(a - b) > 1).any():
            return False
    return True
