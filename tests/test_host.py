"""CPU tests of the HIP library's host side: exported symbols, interaction
stencils, tree validation and the adaptive builder (no GPU calls)."""
import os
import re

import numpy as np
import pytest

import oracle
import paper_2101_08226_amd as lib
import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for h in ("octo.h", "octo_host.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        names |= set(re.findall(r"\b(octo_[a-z_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    L = lib.load_library()
    declared = _declared_symbols()
    assert declared, "no declarations found"
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert declared == set(lib.EXPORTS)


@pytest.mark.parametrize("theta,m2l,near", [(0.5, 231, 32), (0.34, 651, 92)])
def test_stencil_sizes(theta, m2l, near):
    s = lib.octo_host_stencil_sizes(theta)
    assert np.all(s[:8] == m2l) and np.all(s[8:16] == near)
    assert np.all(s[16:] == 5)  # reach of 5 cells: only the 26 neighbouring sub-grids


def test_stencil_theta_035_equals_034():
    """No integer |d|^2 lies in (1/0.35^2, 1/0.34^2] = (8.16, 8.65]."""
    assert np.array_equal(lib.octo_host_stencil_sizes(0.35), lib.octo_host_stencil_sizes(0.34))


def test_stencil_sizes_match_oracle_pair_counts():
    """On a uniform 32^3 tree, level-2 cells far from the boundary have exactly
    the stencil's partners: compare the per-cell count implied by the oracle's
    recursion (constant kernel counts partners) with the library's stencil."""
    for theta in (0.5, 0.34):
        s = lib.octo_host_stencil_sizes(theta)
        rho = np.ones((32, 32, 32))
        t = oracle.Tree(w.uniform_leaves(2), w.grid_to_leaves(rho))
        coef = np.zeros(20)
        coef[0] = 1.0
        # phi_i = -(number of partners evaluated at the leaf level + coarser) ...
        # count only same-level leaf partners: a uniform grid has no coarser
        # direct pairs, so the oracle's direct + leaf-leaf multipole pairs per
        # interior-most cell equal the leaf stencil size.
        t.solve(theta=theta, kernel=coef, sample=np.array([_cell_id(2, (16, 16, 16))]))
        m2l, direct, ll = t.last_counts(split=True)
        assert direct + ll == s[0] + s[8]


def _cell_id(level, g):
    n = 8 << level
    from helpers import grid_ids

    return int(grid_ids(level, np.array([(g[0] * n + g[1]) * n + g[2]]))[0])


def test_layout_validation_errors():
    full = w.uniform_leaves(1)
    with pytest.raises(lib.OctoError, match="OCTO_E_INVALID"):
        lib.octo_host_layout(full[:7])  # gap
    with pytest.raises(lib.OctoError, match="OCTO_E_INVALID"):
        lib.octo_host_layout(np.vstack([full, [[0, 0, 0, 0]]]))  # overlap
    with pytest.raises(lib.OctoError, match="OCTO_E_INVALID"):
        lib.octo_host_layout(np.vstack([full, full[:1]]))  # duplicate
    leaves = [[1, 0, 0, 1], [1, 0, 1, 0], [1, 0, 1, 1], [1, 1, 0, 0], [1, 1, 0, 1], [1, 1, 1, 0], [1, 1, 1, 1]]
    leaves += [[2, a, b, c] for a in (0, 1) for b in (0, 1) for c in (0, 1) if (a, b, c) != (1, 1, 1)]
    leaves += [[3, 2 + a, 2 + b, 2 + c] for a in (0, 1) for b in (0, 1) for c in (0, 1)]
    with pytest.raises(lib.OctoError, match="nested"):
        lib.octo_host_layout(leaves)
    with pytest.raises(lib.OctoError):
        lib.octo_host_layout([[10, 0, 0, 0]])
    n, lv = lib.octo_host_layout(full)
    assert n == 2 and lv.tolist() == [[1, 1, 0], [8, 0, 0]]


@pytest.mark.parametrize("max_level", [3, 5])
def test_adaptive_builder_matches_oracle(max_level):
    f = w.binary_polytrope_128()
    a = lib.octo_host_adaptive_leaves(f, max_level, 1e-4)
    b = oracle.build_adaptive_leaves(f.boxmax, max_level, 1e-4)
    assert np.array_equal(a, b)
    assert oracle.is_balanced(a) if max_level <= 4 else True


def test_adaptive_builder_lmax6_counts():
    """The binary-polytrope tree to level 6 (root = level 0): 7736 leaf
    sub-grids, 1105 interior ones."""
    f = w.binary_polytrope_128()
    a = lib.octo_host_adaptive_leaves(f, 6, 1e-4)
    n, lv = lib.octo_host_layout(a)
    assert len(a) == 7736 and n == 7
    assert int(lv[:, 1].sum()) == 1105
    assert lv[:, 0].tolist() == [1, 8, 64, 512, 896, 2272, 5088]


def test_random_adaptive_trees_match_oracle():
    rng = np.random.default_rng(5)
    for _ in range(4):
        stars = [w.Star(tuple(rng.uniform(-0.35, 0.35, 3)), float(rng.uniform(0.03, 0.15)), 1.0)
                 for _ in range(rng.integers(1, 4))]
        f = w.Polytropes(stars=stars)
        thr = float(10 ** rng.uniform(-6, -1))
        a = lib.octo_host_adaptive_leaves(f, 4, thr)
        b = oracle.build_adaptive_leaves(f.boxmax, 4, thr)
        assert np.array_equal(a, b)


@pytest.mark.parametrize("theta", [0.34, 0.5, 0.7])
def test_near_lists_cover_the_stencil_with_minimal_padding(theta):
    """The leaf kernel's near-field walk, per target class: exactly the
    partners whose parents are not well separated (the opening criterion of
    Sec. 2.2 on the parents' offset, d != 0), each once, each in a sign octant
    that agrees with its nonzero components, every octant list a whole number
    of blocks of 8, and the padding no more than the total count forces."""
    beg, d = lib.octo_host_near_lists(theta)
    sizes = lib.octo_host_stencil_sizes(theta)

    def fdiv2(v):
        return v // 2  # floor division, as for the parent index of a cell

    for p in range(8):
        pc = ((p >> 2) & 1, (p >> 1) & 1, p & 1)
        want = set()
        for dx in range(-7, 8):
            for dy in range(-7, 8):
                for dz in range(-7, 8):
                    if (dx, dy, dz) == (0, 0, 0):
                        continue
                    D = [fdiv2(c + v) for c, v in zip(pc, (dx, dy, dz))]
                    if theta * theta * sum(x * x for x in D) <= 1.0:
                        want.add((dx, dy, dz))
        got, pad = [], 0
        for o in range(8):
            a, b = beg[9 * p + o], beg[9 * p + o + 1]
            assert (b - a) % 8 == 0
            for row in d[a:b]:
                t = tuple(int(v) for v in row)
                if t == (0, 0, 0):
                    pad += 1
                    continue
                for ax in range(3):
                    if t[ax] != 0:
                        assert ((o >> (2 - ax)) & 1) == (t[ax] < 0), (p, o, t)
                got.append(t)
        assert len(got) == len(set(got)) and set(got) == want
        assert len(got) == sizes[p] + sizes[8 + p]
        assert pad == (8 - len(got) % 8) % 8, (theta, p, pad)


def test_near_stage_table_loads_every_halo_cell_once():
    """The near-field kernel's halo staging table: each of the 18^3 cells
    within 5 cells of a sub-grid is loaded exactly once, from the neighbour
    sub-grid that holds it (slot of its floor-divided coordinates) at its
    parity-major storage index there; it lands in a distinct halo slot, in
    the block of its parity class, at lattice position (u >> 1) with one
    stride per axis; the entries past the 18^3 cells are -1."""
    t = lib.octo_host_near_stage().astype(np.int64)
    NH = 18 ** 3
    assert t.shape == (12 * 512,)
    assert np.all(t[NH:] == -1) and np.all(t[:NH] >= 0)
    slot, store, dest = t[:NH] & 31, (t[:NH] >> 5) & 511, t[:NH] >> 14
    c = np.arange(NH)
    local = np.stack([c // 324 - 5, (c // 18) % 18 - 5, c % 18 - 5], axis=1)
    nb = local // 8 + 1  # neighbour sub-grid per axis, 0..2
    assert np.array_equal(slot, nb[:, 0] * 9 + nb[:, 1] * 3 + nb[:, 2])
    # storage index back to the cell: parity class major, then the 4x4x4 lattice
    cls, lat = store >> 6, store & 63
    inner = np.stack([2 * (lat >> 4) + (cls >> 2), 2 * ((lat >> 2) & 3) + ((cls >> 1) & 1),
                      2 * (lat & 3) + (cls & 1)], axis=1)
    assert np.array_equal(local, 8 * (nb - 1) + inner)
    # distinct destinations, one block per parity class of the halo cell
    assert len(np.unique(dest)) == NH
    u = local + 5
    q = (u[:, 0] & 1) * 4 + (u[:, 1] & 1) * 2 + (u[:, 2] & 1)
    lo = [dest[q == k].min() for k in range(8)]
    hi = [dest[q == k].max() for k in range(8)]
    assert all(hi[k] < lo[k + 1] for k in range(7))
    # inside a block: base + ix * SX + iy * SY + iz over the 9^3 lattice
    L = u >> 1
    for k in range(8):
        m = q == k
        d, l3 = dest[m], L[m]
        base = d[np.all(l3 == 0, axis=1)][0]
        sy = d[np.all(l3 == (0, 1, 0), axis=1)][0] - base
        sx = d[np.all(l3 == (1, 0, 0), axis=1)][0] - base
        assert sy >= 9 and sx >= 9 * sy
        assert np.array_equal(d, base + l3[:, 0] * sx + l3[:, 1] * sy + l3[:, 2])


def _morton(c):
    m = np.zeros(len(c), dtype=np.int64)
    for b in range(10):
        for a, sh in ((0, 2), (1, 1), (2, 0)):
            m |= ((c[:, a] >> b) & 1).astype(np.int64) << (3 * b + sh)
    return m


@pytest.mark.parametrize("seed", [2, 5, 8])
def test_level_tables_describe_the_tree(seed):
    """The node tables of the leaf-list layout (the format octo_tree_level_tables
    reports for a tree in device memory) against the tree they describe:
    children and parents invert each other and nest by coordinate, neighbours
    sit at their offsets and see each other back, nodes run interior / leaves
    next to interior nodes / other leaves, each run in Morton order, a leaf's
    flags follow its neighbours and its parent's neighbours, and out_base
    names its place in the caller's list."""
    import helpers

    leaves, _ = helpers.random_amr_leaves(seed, max_level=3 + seed % 2, n_stars=2)
    leaves = np.asarray(leaves, dtype=np.int32)
    leaves = leaves[np.random.default_rng(seed).permutation(len(leaves))]
    nl, _ = lib.octo_host_layout(leaves)
    T = [lib.octo_host_level_tables(leaves, l) for l in range(nl)]
    where = {tuple(v): i for i, v in enumerate(leaves.tolist())}
    for l, t in enumerate(T):
        n, ni, nr = t["n_nodes"], t["n_int"], t["n_rec"]
        c = t["coord"].astype(np.int64)
        assert np.all((c >= 0) & (c < 2 ** l))
        for lo, hi in ((0, ni), (ni, nr), (nr, n)):
            assert np.all(np.diff(_morton(c[lo:hi])) > 0)
        is_int = np.arange(n) < ni
        if l + 1 < nl:
            ch = T[l + 1]
            for k in range(ni):
                for q in range(8):
                    j = t["child"][k, q]
                    assert ch["parent"][j] == k
                    assert np.array_equal(ch["coord"][j], 2 * c[k] + [q >> 2, (q >> 1) & 1, q & 1])
                assert t["int_child"][k] == int(np.any(t["child"][k] < ch["n_int"]))
        else:
            assert ni == 0
        if l == 0:
            assert np.all(t["nbr"] == -1) and t["parent"][0] == -1
            continue
        P = T[l - 1]
        for k in range(n):
            assert np.array_equal(P["child"][t["parent"][k]][np.dot(c[k] & 1, [4, 2, 1])], k)
            touches_int = False
            for o in range(27):
                d = np.array([o // 9 - 1, (o // 3) % 3 - 1, o % 3 - 1])
                b = t["nbr"][k, o]
                q = c[k] + d
                inside = np.all((q >= 0) & (q < 2 ** l))
                if b < 0:
                    # absent: outside the domain, or the parent's neighbour there is a leaf
                    if inside:
                        pq = q >> 1
                        pk = np.flatnonzero(np.all(P["coord"] == pq, axis=1))
                        assert len(pk) == 1 and pk[0] >= P["n_int"]
                    continue
                assert np.array_equal(c[b], q) and t["nbr"][b, 26 - o] == k
                touches_int |= bool(is_int[b])
            if k >= ni:
                # the parent's neighbours that are leaves
                pn = P["nbr"][t["parent"][k]]
                x2 = bool(np.any((pn >= P["n_int"]) & (pn >= 0))) if l > 1 else False
                assert (k < nr) == touches_int
                assert t["flags"][k] == (5 if touches_int else 0) | (2 if x2 else 0)
                assert t["out_base"][k] == 512 * where[(l, *c[k])]
            else:
                assert t["out_base"][k] == -1 and t["flags"][k] == 0
