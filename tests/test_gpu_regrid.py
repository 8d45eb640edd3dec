"""GPU parity of the device regrid (octo_regrid, Sec. 2.7) with the oracle's
regrid, and of the regridded tree's device layout with the host builder's.

Bar: bit-exact.  The leaf lists are integer data; the moved densities are
copies (new children) or means of 8 cells summed in the same order on both
sides (de-refined nodes); the statistics are integer counts and one product.
Leaves are compared as sets (the library emits them in its node order), the
densities leaf by leaf.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2101_08226_amd as lib
import workloads as w
from helpers import random_amr_leaves
from oracle import regrid as R

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-regrid]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = lib.Context(0)
    yield c
    c.close()


def sorted_tree(leaves, rho):
    leaves = np.asarray(leaves, dtype=np.int64).reshape(-1, 4)
    rho = np.asarray(rho).reshape(-1, 512)
    order = np.lexsort((leaves[:, 3], leaves[:, 2], leaves[:, 1], leaves[:, 0]))
    return leaves[order], rho[order]


def check_tables(t2):
    """The regridded tree is laid out on the device: its node tables, counts,
    leaf flags and interior-child bits equal the host builder's for its leaf
    list (integer data: exact)."""
    leaves = t2.leaves()
    nl, _ = lib.octo_host_layout(leaves)
    for l in range(nl):
        d = t2.level_tables(l)
        h = lib.octo_host_level_tables(leaves, l)
        for k in ("n_nodes", "n_int", "n_rec"):
            assert d[k] == h[k], (l, k, d[k], h[k])
        for k in ("nbr", "child", "parent", "coord", "out_base", "flags", "int_child"):
            assert np.array_equal(d[k], h[k]), (l, k)
    with pytest.raises(lib.OctoError):
        t2.level_tables(nl)


def gpu_regrid(ctx, tree, l_max, rho_r, n_target):
    t2, st = tree.regrid(l_max, rho_r, n_target)
    check_tables(t2)
    lv, rho = sorted_tree(t2.leaves(), t2.density())
    return t2, lv, rho, st


def compare(lv_g, rho_g, st_g, lv_o, rho_o, nxt_o, info_o):
    assert lv_g.shape == lv_o.shape and np.array_equal(lv_g, lv_o)
    assert np.array_equal(rho_g, rho_o)
    for k in ("refined", "balance_refined", "derefined", "n_leaves", "n_grids"):
        assert st_g[k] == info_o[k], (k, st_g[k], info_o[k])
    assert st_g["rho_r_next"] == nxt_o


@pytest.mark.parametrize("seed,l_max,q", [(1, 4, 0.9), (2, 4, 0.5), (3, 5, 0.99), (4, 3, 0.2)])
def test_regrid_random_trees(ctx, seed, l_max, q):
    leaves, f = random_amr_leaves(seed, max_level=3, n_stars=2)
    rng = np.random.default_rng(seed)
    rho = w.leaf_density(f, leaves) * rng.uniform(0.5, 1.5, (len(leaves), 512))
    rho_r = float(np.quantile(rho, q))
    say(f"seed={seed} leaves={len(leaves)} l_max={l_max} rho_r={rho_r:.3e}")
    tree = ctx.tree(leaves, rho)
    t2, lv_g, rho_g, st = gpu_regrid(ctx, tree, l_max, rho_r, 300)
    tree.destroy()
    t2.destroy()
    lv_o, rho_o, nxt, info = R.regrid(leaves, rho, l_max, rho_r, n_target=300)
    say(f"  {info}")
    compare(lv_g, rho_g, st, lv_o, rho_o, nxt, info)


def test_regrid_chain_from_the_root(ctx):
    # five regrids in a row from a single sub-grid holding the binary (each
    # side regrids its own previous output)
    f = w.binary_polytrope_128()
    lv_o = w.uniform_leaves(0)
    rho_o = w.leaf_density(f, lv_o)
    tree = ctx.tree(lv_o, rho_o)
    rho_r = 1e-3
    for step in range(5):
        t2, lv_g, rho_g, st = gpu_regrid(ctx, tree, 6, rho_r, 500)
        lv_o, rho_o, nxt, info = R.regrid(lv_o, rho_o, 6, rho_r, n_target=500)
        say(f"step {step}: {info}")
        compare(lv_g, rho_g, st, lv_o, rho_o, nxt, info)
        tree.destroy()
        tree = t2
        rho_r = nxt
    tree.destroy()


def test_regrid_uniform_grid_layout(ctx):
    # a tree on the uniform grid layout (caller strides n^2, n, 1)
    rho = w.uniform_grid(w.binary_polytrope_128(), 3)
    tree = ctx.uniform_tree(rho)
    t2, lv_g, rho_g, st = gpu_regrid(ctx, tree, 5, 1e-2, 0)
    tree.destroy()
    t2.destroy()
    lv_o, rho_o, nxt, info = R.regrid(w.uniform_leaves(3), w.grid_to_leaves(rho), 5, 1e-2)
    say(f"uniform 64^3: {info}")
    assert info["refined"] > 0 and info["derefined"] > 0
    compare(lv_g, rho_g, st, lv_o, rho_o, nxt, info)


def test_regrid_full_size_adaptive(ctx):
    # the adaptive binary to level 6 (3.96M leaf cells), leaf list from the
    # oracle's builder; a cut-off that both refines and coarsens
    f = w.binary_polytrope_128()
    leaves = oracle.build_adaptive_leaves(f.boxmax, 6, 1e-4)
    rho = w.leaf_density(f, leaves)
    tree = ctx.tree(leaves, rho)
    say(f"full size: {len(leaves)} leaves")
    t2, lv_g, rho_g, st = gpu_regrid(ctx, tree, 7, 0.1, 4000)
    tree.destroy()
    lv_o, rho_o, nxt, info = R.regrid(leaves, rho, 7, 0.1, n_target=4000)
    say(f"  {info}")
    assert info["refined"] > 0 and info["derefined"] > 0
    compare(lv_g, rho_g, st, lv_o, rho_o, nxt, info)
    # the new tree solves, bitwise as the same leaves laid out on the host;
    # its mass is the old one's
    phi2, g2, s2 = ctx.solve(t2, theta=0.5)
    t3 = ctx.tree(t2.leaves(), t2.density())
    phi3, g3, _ = ctx.solve(t3, theta=0.5)
    assert np.array_equal(phi2.cpu().numpy(), phi3.cpu().numpy())
    assert np.array_equal(g2.cpu().numpy(), g3.cpu().numpy())
    t3.destroy()
    t2.destroy()
    h = 1.0 / (8 << leaves[:, 0])
    m = float(np.sum(rho.sum(axis=1) * h ** 3))
    assert abs(s2["total_mass"] - m) <= 1e-13 * m


def test_regrid_edge_cases(ctx):
    lv = w.uniform_leaves(1)
    rho = np.full((len(lv), 512), 1e-3)
    tree = ctx.tree(lv, rho)
    # a cut-off that coarsens the level-1 leaves into the root (l_max 1) or
    # keeps them (l_max 3)
    for l_max, rho_r in ((1, 1.0), (3, 1.0)):
        t2, lv_g, rho_g, st = gpu_regrid(ctx, tree, l_max, rho_r, 0)
        t2.destroy()
        lv_o, rho_o, nxt, info = R.regrid(lv, rho, l_max, rho_r)
        compare(lv_g, rho_g, st, lv_o, rho_o, nxt, info)
    # every leaf refines (tiny cut-off)
    t2, lv_g, rho_g, st = gpu_regrid(ctx, tree, 2, 1e-12, 0)
    t2.destroy()
    assert st["refined"] == 8 and st["n_leaves"] == 64
    # errors
    for l_max, rho_r in ((-1, 1.0), (10, 1.0), (3, 0.0), (3, float("nan"))):
        with pytest.raises(lib.OctoError) as e:
            tree.regrid(l_max, rho_r)
        assert e.value.status == lib.OCTO_E_INVALID
    tree.destroy()
