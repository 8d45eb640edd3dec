"""Pins of the regrid oracle (density criterion, dynamic cut-off and 2:1
balance of Sec. 2.7) against closed forms and brute force.

* a uniform density refines a uniform tree level by level and stops at the
  level the criterion gives in closed form, then stays; too fine a tree
  coarsens back to it;
* a single dense cell: repeated regrids refine its sub-grid to the closed-form
  level, nothing else refines beyond what balance forces;
* every output tiles the unit box and is 2:1 balanced over faces, edges and
  corners (brute force over all pairs of leaves);
* mass sum(rho h^3) is kept (injection and 8-cell means);
* a de-refinement next to a neighbour's refined child is dropped (hand-built
  tree);
* the cut-off feedback: (N_grids / N_target)^2 with N_grids counted here.
"""
from __future__ import annotations

import itertools

import numpy as np
import pytest

import workloads as w
from oracle import regrid as R


def mass(leaves, rho):
    h = 1.0 / (8 << np.asarray(leaves)[:, 0])
    return float(np.sum(rho.sum(axis=1) * h ** 3))


def check_tiling_and_balance(leaves):
    lv = np.asarray(leaves, dtype=np.int64)
    # volume tiles the box
    vol = np.sum(8.0 ** (-lv[:, 0]))
    assert abs(vol - 1.0) < 1e-12
    # boxes in units of the finest level
    L = int(lv[:, 0].max())
    lo = lv[:, 1:] << (L - lv[:, :1])
    size = (1 << (L - lv[:, 0]))[:, None]
    hi = lo + size
    for i in range(len(lv)):
        # overlap with any other leaf
        ov = np.all((lo < hi[i]) & (hi > lo[i]), axis=1)
        ov[i] = False
        assert not ov.any()
        # touching (faces, edges, corners) leaves differ by at most one level
        touch = np.all((lo <= hi[i]) & (hi >= lo[i]), axis=1)
        touch[i] = False
        assert np.all(np.abs(lv[touch, 0] - lv[i, 0]) <= 1), (lv[i], lv[touch][np.abs(lv[touch, 0] - lv[i, 0]) > 1])


def count_nodes(leaves):
    nodes = set()
    for l, x, y, z in np.asarray(leaves, dtype=np.int64):
        while True:
            nodes.add((l, x, y, z))
            if l == 0:
                break
            l, x, y, z = l - 1, x >> 1, y >> 1, z >> 1
    return len(nodes)


def uniform(level, value):
    lv = w.uniform_leaves(level)
    return lv, np.full((len(lv), 512), value)


# rho_r = 1: a cell of level l is flagged when value > 8^(l + 1 - l_max), so the
# tree refines until the first level where it is not, or l_max:
# 0.5 > 8^(l-2) for l <= 1 (ends at 2); 1e-2 > 8^(l-3) for l = 0 (ends at 1);
# 1e-5 > 8^(l-3) never (stays at 0); 3 > 8^(l-1) up to l_max = 2
@pytest.mark.parametrize("value,l_max,expect", [(0.5, 3, 2), (1e-2, 4, 1), (1e-5, 4, 0), (3.0, 2, 2)])
def test_uniform_density_closed_form(value, l_max, expect):
    lv, rho = uniform(0, value)
    for step in range(l_max + 2):
        lv2, rho2, _, info = R.regrid(lv, rho, l_max, 1.0)
        want = min(step + 1, expect)
        assert set(lv2[:, 0]) == {want}, (step, set(lv2[:, 0]))
        assert np.all(rho2 == value)
        lv, rho = lv2, rho2
    # too fine: coarsens one level per regrid back to the same level
    if expect < 2:
        lv, rho = uniform(expect + 2, value)
        for _ in range(3):
            lv, rho, _, _ = R.regrid(lv, rho, l_max, 1.0)
        assert set(lv[:, 0]) == {expect}


def test_single_dense_cell_reaches_its_level():
    # floor 1e-10 everywhere, one cell of density 0.02: with rho_r = 1 and
    # l_max = 5 its sub-grid is flagged at levels with 0.02 > 8^(l - 4), i.e.
    # l <= 2, so it ends at level 3; every other sub-grid only by balance
    lv, rho = uniform(0, 1e-10)
    rho[0, (3 * 8 + 5) * 8 + 6] = 0.02
    m0 = mass(lv, rho)
    for _ in range(6):
        lv, rho, _, info = R.regrid(lv, rho, 5, 1.0)
        check_tiling_and_balance(lv)
        assert abs(mass(lv, rho) - m0) <= 1e-14 * m0
    k = int(np.argmax(rho.max(axis=1)))
    assert lv[k, 0] == 3 and rho[k].max() == 0.02
    # the dense cell (3, 5, 6) of the level-0 grid, at level 3, lies in sub-grid
    # (3*8 + 5*8... ) // 8 per axis of the 64^3 cell lattice
    assert tuple(lv[k, 1:]) == ((3 * 8) // 8, (5 * 8) // 8, (6 * 8) // 8)
    assert lv[:, 0].max() == 3


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_trees_keep_mass_tiling_and_balance(seed):
    from helpers import random_amr_leaves

    leaves, f = random_amr_leaves(seed, max_level=3, n_stars=2)
    rho = w.leaf_density(f, leaves)
    rng = np.random.default_rng(seed)
    rho = rho * rng.uniform(0.5, 1.5, rho.shape)
    m0 = mass(leaves, rho)
    rho_r = float(np.quantile(rho, 0.9))
    lv = leaves
    for _ in range(3):
        lv, rho, nxt, info = R.regrid(lv, rho, 4, rho_r, n_target=200)
        check_tiling_and_balance(lv)
        assert abs(mass(lv, rho) - m0) <= 1e-13 * m0
        assert info["n_grids"] == count_nodes(lv)
        assert nxt == rho_r * (info["n_grids"] / 200) ** 2


def test_derefinement_dropped_next_to_a_refined_neighbour_child():
    # level-1 tree; node P = (1,0,0,0) refined to level-2 leaves of tiny
    # density (a de-refinement candidate); its neighbour Q = (1,1,0,0) refined
    # too, with its child (2,2,0,0), which touches P, dense enough to refine:
    # P may not coarsen (it would face level-3 leaves)
    leaves = [(1, x, y, z) for x in range(2) for y in range(2) for z in range(2) if (x, y, z) not in ((0, 0, 0), (1, 0, 0))]
    kids_p = [(2, a, b, c) for a in range(2) for b in range(2) for c in range(2)]
    kids_q = [(2, 2 + a, b, c) for a in range(2) for b in range(2) for c in range(2)]
    leaves = leaves + kids_p + kids_q
    rho = np.full((len(leaves), 512), 1e-10)
    rho[leaves.index((2, 2, 0, 0))] = 2.0  # above 8^(2 + 1 - 3) = 1
    lv, _, _, info = R.regrid(leaves, rho, 3, 1.0)
    check_tiling_and_balance(lv)
    keys = {tuple(k) for k in lv}
    assert (3, 4, 0, 0) in keys            # Q's child refined
    assert (1, 0, 0, 0) not in keys        # P kept its children
    assert (2, 0, 0, 0) in keys
    # without the dense child P coarsens
    rho[leaves.index((2, 2, 0, 0))] = 1e-10
    lv, _, _, info = R.regrid(leaves, rho, 3, 1.0)
    keys = {tuple(k) for k in lv}
    assert (1, 0, 0, 0) in keys and (1, 1, 0, 0) in keys and info["derefined"] == 2


def test_cutoff_feedback_special_cases():
    lv, rho = uniform(1, 1e-3)
    _, _, same, info = R.regrid(lv, rho, 3, 1.0, n_target=0)
    assert same == 1.0
    _, _, nxt, info = R.regrid(lv, rho, 3, 1.0, n_target=info["n_grids"])
    assert nxt == 1.0


def test_derefinement_uses_each_level_threshold():
    # P = (1,0,0,0) with leaf children; one child cell at 0.5: above the
    # level-1 threshold 8^(1 + 1 - 3) = 1/8 but not the level-2 one (1), and
    # the mean over P's cell 0.5/8 is below 1/8: P coarsens, keeping the mass
    leaves = [(1, x, y, z) for x in range(2) for y in range(2) for z in range(2) if (x, y, z) != (0, 0, 0)]
    leaves += [(2, a, b, c) for a in range(2) for b in range(2) for c in range(2)]
    rho = np.full((len(leaves), 512), 1e-10)
    rho[leaves.index((2, 1, 1, 1)), 0] = 0.5
    m0 = mass(leaves, rho)
    lv, rho2, _, info = R.regrid(leaves, rho, 3, 1.0)
    assert info["derefined"] == 1 and len(lv) == 8 and set(lv[:, 0]) == {1}
    assert abs(mass(lv, rho2) - m0) <= 1e-14 * m0
    # the child cell (0,0,0) of child (1,1,1) lies under P's cell (4,4,4),
    # the first of the 8 cells summed there
    k = [tuple(x) for x in lv].index((1, 0, 0, 0))
    s = 0.5
    for _ in range(7):
        s += 1e-10
    assert rho2[k].reshape(8, 8, 8)[4, 4, 4] == s / 8.0
    f = 0.0
    for _ in range(8):
        f += 1e-10
    assert rho2[k].reshape(8, 8, 8)[3, 4, 4] == f / 8.0
