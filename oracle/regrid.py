"""TEST INFRASTRUCTURE ONLY: one regrid of the octree by the density criterion
of Sec. 2.7 ("Refinement Criteria"), with the dynamic cut-off rho_r and 2:1
balance, written from the paper's description in plain Python over a dict of
nodes.

Readings where the printed text is garbled or silent (also listed in the
design notes):

* the criterion: a cell of level l is flagged when rho > 8^(l + 1 - l_max) rho_r,
  i.e. when the largest level L with rho > 8^(L - l_max) rho_r exceeds l.  With
  the exponent as printed (l_max - L) the inequality holds at l_max whenever it
  holds anywhere, so the level-dependent factor would never matter; with it
  reversed the wanted level rises by one for every factor of 8 in density
  (refinement at constant cell mass);
* refinement and de-refinement move one level per regrid: a leaf with a
  flagged cell (and level < l_max) gets 8 children; an interior node whose 8
  children are leaves is de-refined when none of its cells (averages of the
  children's cells) and none of its children's cells are flagged;
* 2:1 balance (26 neighbours): a refined leaf makes every leaf of the coarser
  level next to it refine as well, to a fixed point; a de-refinement is
  dropped when a child of the node is refined, or when a node two levels finer
  than the de-refined node would touch it (a child of a same-level neighbour,
  touching the node, that is interior or refined);
* the window of two cells and the regrid cadence (time stepping) are not used;
* densities move with the cells: a new child's cell takes the density of the
  parent cell containing it; a de-refined node's cell the mean of its 8 child
  cells (summed in child-cell order a, b, c, then divided by 8); both keep
  the mass sum(rho h^3);
* after the regrid rho_r -> (N_grids / N_target)^2 rho_r with N_grids the number
  of sub-grids of the new tree, leaves and interior nodes.

Leaves are (level, ix, iy, iz); densities (n, 512) with the cells (x, y, z) of a
sub-grid in the order z fastest.
"""
from __future__ import annotations

import itertools
from typing import Dict, Tuple

import numpy as np

Key = Tuple[int, int, int, int]
DIRS = [d for d in itertools.product((-1, 0, 1), repeat=3) if d != (0, 0, 0)]


def threshold(level: int, l_max: int, rho_r: float) -> float:
    """Density above which a cell of `level` is flagged (exact: a power of 8)."""
    return rho_r * 8.0 ** (level + 1 - l_max)


def _children(k: Key):
    l, x, y, z = k
    return [(l + 1, 2 * x + a, 2 * y + b, 2 * z + c) for a in (0, 1) for b in (0, 1) for c in (0, 1)]


def _parent_mean(child_rho):
    """The 512 cells of a node from its 8 children's cells (child order
    a*4 + b*2 + c); cell (x, y, z) is the mean of the child cells under it."""
    out = np.empty((8, 8, 8))
    ch = [c.reshape(8, 8, 8) for c in child_rho]
    for x in range(8):
        for y in range(8):
            for z in range(8):
                kid = ch[(x >> 2) * 4 + (y >> 2) * 2 + (z >> 2)]
                bx, by, bz = 2 * (x & 3), 2 * (y & 3), 2 * (z & 3)
                s = 0.0
                for a in (0, 1):
                    for b in (0, 1):
                        for c in (0, 1):
                            s += kid[bx + a, by + b, bz + c]
                out[x, y, z] = s / 8.0
    return out.ravel()


def _child_inject(parent_rho, a, b, c):
    p = parent_rho.reshape(8, 8, 8)
    x = np.arange(8)
    # child cell x lies in parent cell 4a + x // 2 along each axis
    return p[np.ix_(4 * a + (x >> 1), 4 * b + (x >> 1), 4 * c + (x >> 1))].ravel()


def regrid(leaves, rho, l_max: int, rho_r: float, n_target: int = 0):
    """One regrid.  Returns (new_leaves (m, 4) int32 sorted by (level, ix, iy,
    iz), new_rho (m, 512), rho_r_next, info dict)."""
    leaves = np.asarray(leaves, dtype=np.int64).reshape(-1, 4)
    rho = np.asarray(rho, dtype=np.float64).reshape(-1, 512)
    leaf: Dict[Key, np.ndarray] = {tuple(int(v) for v in k): r for k, r in zip(leaves, rho)}
    nodes = set(leaf)
    for k in list(leaf):
        l, x, y, z = k
        while l > 0:
            l, x, y, z = l - 1, x >> 1, y >> 1, z >> 1
            nodes.add((l, x, y, z))
    interior = nodes - set(leaf)

    def inside(l, x, y, z):
        n = 1 << l
        return 0 <= x < n and 0 <= y < n and 0 <= z < n

    # criterion on leaves
    refine = {k for k, r in leaf.items() if k[0] < l_max and r.max() > threshold(k[0], l_max, rho_r)}
    criterion = set(refine)
    # de-refinement candidates: interior nodes whose children are all leaves
    mean = {}
    deref = set()
    for p in interior:
        kids = _children(p)
        if not all(c in leaf for c in kids):
            continue
        lv = p[0]
        kid_flag = lv + 1 < l_max and any(leaf[c].max() > threshold(lv + 1, l_max, rho_r) for c in kids)
        m = _parent_mean([leaf[c] for c in kids])
        mean[p] = m
        if not kid_flag and not m.max() > threshold(lv, l_max, rho_r):
            deref.add(p)
    # 2:1 balance of refinements, to a fixed point
    todo = list(refine)
    while todo:
        l, x, y, z = todo.pop()
        for dx, dy, dz in DIRS:
            q = (l, x + dx, y + dy, z + dz)
            if not inside(*q) or q in nodes:
                continue
            cov = (l - 1, q[1] >> 1, q[2] >> 1, q[3] >> 1)
            assert cov in leaf, "input tree not 2:1 balanced"
            if cov not in refine:
                refine.add(cov)
                todo.append(cov)
    # de-refinements that would break the balance
    kept = set()
    for p in deref:
        if any(c in refine for c in _children(p)):
            continue
        l, x, y, z = p
        bad = False
        for dx, dy, dz in DIRS:
            qn = (l, x + dx, y + dy, z + dz)
            if qn not in interior:
                continue
            for c in _children(qn):
                touch = all(2 * pc - 1 <= cc <= 2 * pc + 2 for cc, pc in zip(c[1:], p[1:]))
                if touch and (c in interior or c in refine):
                    bad = True
        if not bad:
            kept.add(p)
    # the new leaves and their densities
    new = {}
    for k, r in leaf.items():
        par = (k[0] - 1, k[1] >> 1, k[2] >> 1, k[3] >> 1)
        if k[0] > 0 and par in kept:
            continue
        if k in refine:
            for i, c in enumerate(_children(k)):
                new[c] = _child_inject(r, (i >> 2) & 1, (i >> 1) & 1, i & 1)
        else:
            new[k] = r
    for p in kept:
        new[p] = mean[p]
    keys = sorted(new)
    new_leaves = np.array(keys, dtype=np.int32).reshape(-1, 4)
    new_rho = np.stack([new[k] for k in keys]) if keys else np.zeros((0, 512))
    all_nodes = set(keys)
    for k in keys:
        l, x, y, z = k
        while l > 0:
            l, x, y, z = l - 1, x >> 1, y >> 1, z >> 1
            all_nodes.add((l, x, y, z))
    n_grids = len(all_nodes)
    rho_next = rho_r * (n_grids / n_target) ** 2 if n_target > 0 else rho_r
    info = dict(refined=len(criterion), balance_refined=len(refine) - len(criterion), derefined=len(kept),
                n_leaves=len(keys), n_grids=n_grids)
    return new_leaves, new_rho, rho_next, info
