"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test is chosen so that a plausible mistake in the oracle (a dropped term,
a wrong sign or index, a transposed operand, a missed or doubled pair) fails
at least one of them:

* derivative tensors against finite differences and harmonicity;
* a cubic polynomial kernel, for which a third-order expansion is exact, so
  the whole tree machinery (upward, interaction lists, downward, AMR
  boundaries) must equal brute force;
* the constant kernel K = 1: every pair is counted exactly once;
* a single 8^3 leaf: all pairs are direct and must equal the N^2 sum;
* two-cell invariants of the angular-momentum correction;
* zero net force and torque of whole solves (Sec. 2.2 conservation claims);
* closed forms (point mass, uniform sphere) and the paper's residual table.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as w
from helpers import MONOMIALS, poly_direct, random_amr_leaves, rel_err_g, rel_err_phi, zero_block_density

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------
# derivative tensors
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kernel", ["newton", "cubic"])
def test_dtensors_finite_differences(kernel):
    rng = np.random.default_rng(1)
    coef = rng.standard_normal(20) if kernel == "cubic" else None
    for _ in range(5):
        R = rng.uniform(-1, 1, 3)
        R *= rng.uniform(0.3, 2.0) / np.linalg.norm(R)
        D = oracle.dtensors(R, coef)
        if kernel == "newton":
            assert D[0] == pytest.approx(1.0 / np.linalg.norm(R), rel=1e-15)
        else:
            k = sum(c * R[0] ** p[0] * R[1] ** p[1] * R[2] ** p[2] for c, p in zip(coef, MONOMIALS))
            assert D[0] == pytest.approx(k, rel=1e-13, abs=1e-13)
        eps = 1e-5 * np.linalg.norm(R)
        for k in range(4):
            fd = np.empty(D[k + 1].shape)
            for e in range(3):
                dR = np.zeros(3)
                dR[e] = eps
                fd[..., e] = (np.asarray(oracle.dtensors(R + dR, coef)[k]) -
                              np.asarray(oracle.dtensors(R - dR, coef)[k])) / (2 * eps)
            scale = np.max(np.abs(D[k + 1])) + 1e-30
            assert np.max(np.abs(fd - D[k + 1])) / scale < 1e-7, (kernel, k)
        # full symmetry of every tensor
        for k in range(2, 5):
            T = D[k]
            for perm in [(1, 0) + tuple(range(2, k)), tuple(range(1, k)) + (0,)]:
                assert np.allclose(T, np.transpose(T, perm), rtol=0, atol=1e-12 * np.max(np.abs(T)))
        if kernel == "newton":
            # 1/|R| is harmonic: every trace of D^(k), k >= 2, vanishes
            s2, s3, s4 = np.max(np.abs(D[2])), np.max(np.abs(D[3])), np.max(np.abs(D[4]))
            assert abs(np.trace(D[2])) < 1e-13 * s2
            assert np.max(np.abs(np.einsum("aab->b", D[3]))) < 1e-13 * s3
            assert np.max(np.abs(np.einsum("aabc->bc", D[4]))) < 1e-13 * s4


def test_direct_matches_numpy():
    rng = np.random.default_rng(2)
    n = 300
    x = rng.uniform(-0.5, 0.5, (3, n))
    m = rng.uniform(0.1, 1.0, n)
    phi, g = oracle.direct(x, m, G=1.0)
    R = x[:, :, None] - x[:, None, :]
    r = np.sqrt((R * R).sum(0))
    np.fill_diagonal(r, np.inf)
    phi_ref = -(m[None, :] / r).sum(1)
    g_ref = -(m[None, None, :] * R / r[None] ** 3).sum(2)
    assert rel_err_phi(phi, phi_ref) < 1e-13
    assert rel_err_g(g, g_ref) < 1e-13
    pt, gt = oracle.direct_points(x, m, x[:, 10:20])
    assert np.array_equal(pt, phi[10:20]) or rel_err_phi(pt, phi[10:20]) < 1e-15


# --------------------------------------------------------------------------
# exactness for polynomial kernels, completeness
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [3, 4])
def test_cubic_kernel_is_exact(seed):
    leaves, _ = random_amr_leaves(seed, max_level=2, n_stars=2)
    assert len(np.unique(leaves[:, 0])) >= 2, "want an adaptive tree"
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.1, 1.0, (len(leaves), 512))
    t = oracle.Tree(leaves, rho)
    coef = rng.standard_normal(20)
    for theta in ((0.5, 0.34) if seed == 3 else (0.6,)):
        phi, g = t.solve(theta=theta, kernel=coef)
        x, m = t.leaf_cells()
        pr, gr = poly_direct(coef, x, m)
        assert np.max(np.abs(phi - pr)) / np.max(np.abs(pr)) < 1e-11
        assert rel_err_g(g, gr) < 1e-11


def test_constant_kernel_counts_every_pair_once():
    leaves, _ = random_amr_leaves(7, max_level=2, n_stars=1)
    rng = np.random.default_rng(7)
    rho = rng.uniform(0.1, 1.0, (len(leaves), 512))
    t = oracle.Tree(leaves, rho)
    coef = np.zeros(20)
    coef[0] = 1.0
    x, m = t.leaf_cells()
    for theta in (0.5, 0.34, 0.9):
        phi, g = t.solve(theta=theta, kernel=coef)
        expect = -(m.sum() - m)
        assert np.max(np.abs(phi - expect)) < 1e-12 * m.sum()
        assert np.max(np.abs(g)) == 0.0


def test_massless_cells():
    """Reading R11: an interior cell whose children have no mass takes its
    geometric centre as expansion centre, has all moments zero and skips the
    correction as a target; massless cells remain targets.  Constant kernel:
    every target sees exactly the mass of all other cells; cubic kernel:
    brute force; Newton: zero net force and torque."""
    rho = zero_block_density(5)
    t = oracle.Tree(w.uniform_leaves(2), w.grid_to_leaves(rho))
    x, m = t.leaf_cells()
    assert np.sum(m == 0.0) == 3 * 64 + 8
    coef = np.zeros(20)
    coef[0] = 1.0
    for theta in (0.5, 0.34):
        phi, g = t.solve(theta=theta, kernel=coef)
        assert np.max(np.abs(phi + (m.sum() - m))) < 1e-12 * m.sum()
        assert np.max(np.abs(g)) == 0.0
    rng = np.random.default_rng(5)
    coef = rng.standard_normal(20)
    phi, g = t.solve(theta=0.5, kernel=coef)
    pr, gr = poly_direct(coef, x, m)
    assert np.max(np.abs(phi - pr)) / np.max(np.abs(pr)) < 1e-11
    assert rel_err_g(g, gr) < 1e-11
    # the massless cells: root cell (0,0,0) and its level-1 cells, and one level-1 cell
    for level, gi in ((0, (0, 0, 0)), (1, (1, 0, 1)), (0, (3, 4, 2)), (1, (3, 3, 13))):
        c = t.cell_moments(level, *gi)
        h = 1.0 / (8 << level)
        assert c["m"] == 0.0
        assert np.array_equal(c["z"], (np.array(gi) + 0.5) * h - 0.5)
        assert np.all(c["M2"] == 0.0) and np.all(c["M3"] == 0.0)
    phi, g = t.solve(theta=0.5)
    assert np.all(np.isfinite(phi)) and np.all(np.isfinite(g)) and np.all(phi < 0)
    st = oracle.stats(x, m, g)
    assert st["force"] < 1e-14 and st["torque"] < 1e-13
    pd, gd = oracle.direct(x, m)
    assert rel_err_phi(phi, pd) < 1e-2  # truncation level against the N^2 sum


def test_corner_neighbours_above_inverse_sqrt3():
    """The printed opening test on integer offsets: cells touching at a
    corner (|d|^2 = 3) become well separated once theta exceeds 1/sqrt(3).
    Their expansions then reach masses next to the shared corner, outside the
    region where they converge, and the method loses its accuracy on an
    adaptive tree (errors of order one, potentials near zero or positive,
    where the N^2 sum is -4.7e-3), while up to 0.57 it stays at the truncation
    level of a few per cent at worst.  The paper runs only theta = 0.5 and
    0.34; the library accepts [0.34, 1) as the text allows."""
    leaves, f = random_amr_leaves(22, max_level=3, n_stars=2)
    t = oracle.Tree(leaves, w.leaf_density(f, leaves))
    x, m = t.leaf_cells()
    rng = np.random.default_rng(22)
    ids = np.unique(np.concatenate([rng.choice(t.n_cells, 3000, replace=False), [66004, 69998, 33015]]))
    pd, _ = oracle.direct_points(x, m, x[:, ids])
    worst = {}
    for theta in (0.5, 0.57, 0.578):
        phi, _ = t.solve(theta=theta, sample=ids)
        worst[theta] = float(np.max(np.abs(phi - pd) / np.abs(pd)))
    assert worst[0.5] < 5e-2 and worst[0.57] < 5e-2
    assert worst[0.578] > 0.5


def test_single_leaf_equals_direct_sum():
    rng = np.random.default_rng(8)
    rho = rng.uniform(0.5, 2.0, (1, 512))
    t = oracle.Tree([[0, 0, 0, 0]], rho)
    phi, g = t.solve()
    x, m = t.leaf_cells()
    pd, gd = oracle.direct(x, m)
    assert rel_err_phi(phi, pd) < 1e-13
    assert rel_err_g(g, gd) < 1e-13


# --------------------------------------------------------------------------
# upward pass
# --------------------------------------------------------------------------

def test_moments_equal_direct_sums():
    leaves, f = random_amr_leaves(9, max_level=2, n_stars=1)
    rho = w.leaf_density(f, leaves)
    t = oracle.Tree(leaves, rho)
    t.solve()
    x, m = t.leaf_cells()
    rng = np.random.default_rng(9)
    checked = 0
    for level in (0, 1):
        n = 8 << level
        for _ in range(20):
            gi = rng.integers(0, n, 3)
            try:
                c = t.cell_moments(level, *gi)
            except KeyError:
                continue
            h = 1.0 / n
            lo = gi * h - 0.5
            inside = np.all((x >= lo[:, None]) & (x < lo[:, None] + h), axis=0)
            if c["m"] == 0 or inside.sum() == 0:
                continue
            mm = m[inside]
            xx = x[:, inside]
            M = mm.sum()
            z = (mm * xx).sum(1) / M
            r = xx - z[:, None]
            M2 = np.einsum("n,an,bn->ab", mm, r, r)
            M3 = np.einsum("n,an,bn,cn->abc", mm, r, r, r)
            assert c["m"] == pytest.approx(M, rel=1e-14)
            assert np.max(np.abs(c["z"] - z)) < 1e-15
            assert np.max(np.abs(c["M2"] - M2)) <= 1e-13 * M * h ** 2
            assert np.max(np.abs(c["M3"] - M3)) <= 1e-13 * M * h ** 3
            checked += 1
    assert checked >= 10


# --------------------------------------------------------------------------
# angular-momentum correction, two cells
# --------------------------------------------------------------------------

def _cluster(rng, centre, size, n=40):
    pts = centre[:, None] + rng.uniform(-size / 2, size / 2, (3, n))
    m = rng.uniform(0.2, 1.0, n)
    M = m.sum()
    z = (m * pts).sum(1) / M
    r = pts - z[:, None]
    return pts, m, dict(m=M, z=z, M2=np.einsum("n,an,bn->ab", m, r, r), M3=np.einsum("n,an,bn,cn->abc", m, r, r, r))


def _eval_local(loc, z, pts):
    """phi and g = -grad phi of the local polynomial about z at points."""
    r = pts - z[:, None]
    phi = (loc["L0"] + loc["L1"] @ r + 0.5 * np.einsum("ab,an,bn->n", loc["L2"], r, r) +
           np.einsum("abc,an,bn,cn->n", loc["L3"], r, r, r) / 6.0)
    grad = (loc["L1"][:, None] + loc["L2"] @ r + 0.5 * np.einsum("abc,bn,cn->an", loc["L3"], r, r))
    return phi, -grad + loc["C"][:, None]


def test_two_cell_correction_invariants():
    rng = np.random.default_rng(10)
    pa, ma, A = _cluster(rng, np.array([0.0, 0.0, 0.0]), 0.1)
    pb, mb, B = _cluster(rng, np.array([0.25, 0.12, -0.07]), 0.1)
    res = {}
    for amc in (False, True):
        la = oracle.m2l_pair(A, B, amc=amc)
        lb = oracle.m2l_pair(B, A, amc=amc)
        _, ga = _eval_local(la, A["z"], pa)
        _, gb = _eval_local(lb, B["z"], pb)
        Fa = (ma * ga).sum(1)
        Fb = (mb * gb).sum(1)
        T = np.cross(pa.T, (ma * ga).T).sum(0) + np.cross(pb.T, (mb * gb).T).sum(0)
        scale = np.linalg.norm(Fa) * np.linalg.norm(B["z"] - A["z"])
        assert np.linalg.norm(Fa + Fb) < 1e-14 * np.linalg.norm(Fa)  # linear momentum
        res[amc] = np.linalg.norm(T) / scale
    assert res[True] < 1e-13  # the correction removes the pair torque
    assert res[False] > 1e-6  # ... which is there without it


def test_expansion_order_three():
    """The potential error of one expansion falls as (size/distance)^4."""
    rng = np.random.default_rng(11)
    pa, ma, A = _cluster(rng, np.zeros(3), 0.1, n=30)
    errs = []
    dists = [0.4, 0.8, 1.6]
    u = np.array([0.6, 0.64, 0.48])
    for d in dists:
        pb, mb, B = _cluster(np.random.default_rng(12), d * u, 0.1, n=30)
        loc = oracle.m2l_pair(A, B, amc=False)
        phi, _ = _eval_local(loc, A["z"], pa)
        R = pa[:, :, None] - pb[:, None, :]
        exact = -(mb[None, :] / np.sqrt((R * R).sum(0))).sum(1)
        errs.append(np.max(np.abs(phi - exact) / np.abs(exact)))
    slopes = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    for s in slopes:
        assert 3.5 < s < 4.6, slopes


# --------------------------------------------------------------------------
# whole solves
# --------------------------------------------------------------------------

def test_net_force_and_torque_adaptive():
    leaves, f = random_amr_leaves(13, max_level=2, n_stars=2)
    rho = w.leaf_density(f, leaves)
    t = oracle.Tree(leaves, rho)
    x, m = t.leaf_cells()
    _, g1 = t.solve(amc=True)
    _, g0 = t.solve(amc=False)
    s1 = oracle.stats(x, m, g1)
    s0 = oracle.stats(x, m, g0)
    assert s1["force"] < 1e-14 and s0["force"] < 1e-14
    assert s1["torque"] < 1e-13
    assert s0["torque"] > 1e-9


def test_point_mass():
    """A single heavy cell in a near-empty box: phi = -M/r and g = -M R/r^3 up to
    the truncation of the targets' local expansions (phi ~1e-3; the force is
    consistent to second order, so up to a few per cent at theta = 0.5)."""
    rho = np.full((16, 16, 16), 1e-10)
    rho[5, 9, 6] = 1e6
    t = oracle.Tree(w.uniform_leaves(1), w.grid_to_leaves(rho))
    phi, g = t.solve()
    x, m = t.leaf_cells()
    src = w.cell_centres(1)[[5, 9, 6]]
    R = x - src[:, None]
    r = np.sqrt((R * R).sum(0))
    far = r > 0
    M = 1e6 / 16 ** 3
    e = np.abs(phi[far] + M / r[far]) / (M / r[far])
    assert e.max() < 5e-3 and e.mean() < 5e-4
    g_ref = -M * R[:, far] / r[far] ** 3
    eg = np.linalg.norm(g[:, far] - g_ref, axis=0) / np.linalg.norm(g_ref, axis=0)
    assert eg.max() < 0.1 and eg.mean() < 1e-2
    # direct (near) neighbours are exact point-mass sums
    near = far & (r < 2.5 / 16)
    assert np.max(np.abs(phi[near] + M / r[near]) / (M / r[near])) < 1e-12


def test_exact_scaling_and_thread_independence():
    leaves, f = random_amr_leaves(14, max_level=2, n_stars=1)
    rho = w.leaf_density(f, leaves)
    p1, g1 = oracle.Tree(leaves, rho).solve(threads=1)
    p4, g4 = oracle.Tree(leaves, 4.0 * rho).solve(threads=4)
    assert np.array_equal(4.0 * p1, p4) and np.array_equal(4.0 * g1, g4)
    t = oracle.Tree(leaves, rho)
    sample = np.random.default_rng(14).choice(len(leaves) * 512, 50, replace=False)
    ps, gs = t.solve(sample=sample)
    assert np.array_equal(ps, p1[sample]) and np.array_equal(gs, g1[:, sample])


def test_mirror_symmetry():
    rho = w.noisy_sphere_16(seed=99)
    mir = rho[::-1].copy()
    p, g = oracle.Tree(w.uniform_leaves(1), w.grid_to_leaves(rho)).solve()
    pm, gm = oracle.Tree(w.uniform_leaves(1), w.grid_to_leaves(mir)).solve()
    P, Pm = w.leaves_to_grid(p, 1), w.leaves_to_grid(pm, 1)[::-1]
    assert rel_err_phi(Pm, P) < 1e-13
    for a, sgn in ((0, -1.0), (1, 1.0), (2, 1.0)):
        Ga = w.leaves_to_grid(g[a], 1)
        Gm = sgn * w.leaves_to_grid(gm[a], 1)[::-1]
        assert np.max(np.abs(Gm - Ga)) < 1e-13 * np.max(np.abs(Ga))


def test_c1_noisy_sphere_against_direct():
    """16^3 grid, 2x2x2 sub-grids: FMM within truncation of the N^2 sum,
    conserving force and torque to machine precision."""
    t = oracle.Tree(w.uniform_leaves(1), w.grid_to_leaves(w.noisy_sphere_16()))
    phi, g = t.solve(theta=0.5)
    x, m = t.leaf_cells()
    pd, gd = oracle.direct(x, m)
    e = np.abs(phi - pd) / np.abs(pd)
    assert 1e-6 < e.mean() < 1e-4 and 1e-5 < e.max() < 1e-2
    assert 1e-5 < rel_err_g(g, gd) < 3e-2
    s = oracle.stats(x, m, g)
    assert s["force"] < 1e-14 and s["torque"] < 1e-13


def _paper_pair_counts(theta):
    """Ordered-pair counts on the 16^3 two-level grid by the paper's literal
    opening criterion on geometric cell centres: A, B are well separated iff
    dx/|x_A - x_B| < theta; multipole pairs are well separated with parents that
    are not (every distinct root pair is a candidate); the remaining leaf pairs
    whose parents are not well separated are direct."""
    def ws(c_a, c_b, h):
        d = np.sqrt(((c_a[:, None, :] - c_b[None, :, :]) ** 2).sum(-1))
        with np.errstate(divide="ignore"):
            return h / d < theta
    c0 = w.cell_centres(0)
    c1 = w.cell_centres(1)
    g0 = np.stack(np.meshgrid(c0, c0, c0, indexing="ij"), -1).reshape(-1, 3)
    g1 = np.stack(np.meshgrid(c1, c1, c1, indexing="ij"), -1).reshape(-1, 3)
    i1 = np.stack(np.meshgrid(*(np.arange(16),) * 3, indexing="ij"), -1).reshape(-1, 3)
    par = (i1[:, 0] // 2) * 64 + (i1[:, 1] // 2) * 8 + i1[:, 2] // 2
    ws0 = ws(g0, g0, 1.0 / 8)
    np.fill_diagonal(ws0, False)
    m2l = int(ws0.sum())
    direct = 0
    for s0 in range(0, 4096, 512):
        w1 = ws(g1[s0:s0 + 512], g1, 1.0 / 16)
        parent_ws = ws0[par[s0:s0 + 512]][:, par]
        same = np.arange(s0, s0 + 512)[:, None] == np.arange(4096)[None, :]
        m2l += int((w1 & ~parent_ws).sum())
        direct += int((~w1 & ~parent_ws & ~same).sum())
    return m2l, direct


@pytest.mark.parametrize("theta", [0.5, 0.34])
def test_interaction_counts_follow_the_opening_criterion(theta):
    t = oracle.Tree(w.uniform_leaves(1), w.grid_to_leaves(w.noisy_sphere_16()))
    t.solve(theta=theta)
    assert t.last_counts() == _paper_pair_counts(theta)


# --------------------------------------------------------------------------
# tree validation and the adaptive builder
# --------------------------------------------------------------------------

def test_tree_validation():
    rho1 = np.ones((1, 512))
    with pytest.raises(ValueError):
        oracle.Tree([[1, 0, 0, 0]], rho1)  # gap
    full = w.uniform_leaves(1)
    with pytest.raises(ValueError):
        oracle.Tree(np.vstack([full, [[0, 0, 0, 0]]]), np.ones((9, 512)))  # overlap
    with pytest.raises(ValueError):
        oracle.Tree(np.vstack([full, full[:1]]), np.ones((9, 512)))  # duplicate
    # a level-1 leaf touching level-3 leaves violates proper nesting
    leaves = [[1, 0, 0, 1], [1, 0, 1, 0], [1, 0, 1, 1], [1, 1, 0, 0], [1, 1, 0, 1], [1, 1, 1, 0], [1, 1, 1, 1]]
    leaves += [[2, a, b, c] for a in (0, 1) for b in (0, 1) for c in (0, 1) if (a, b, c) != (1, 1, 1)]
    leaves += [[3, 2 + a, 2 + b, 2 + c] for a in (0, 1) for b in (0, 1) for c in (0, 1)]
    with pytest.raises(ValueError, match="balance"):
        oracle.Tree(leaves, np.ones((len(leaves), 512)))
    bad = np.ones((8, 512))
    bad[3, 7] = -1.0
    with pytest.raises(ValueError):
        oracle.Tree(full, bad)
    bad[3, 7] = np.nan
    with pytest.raises(ValueError):
        oracle.Tree(full, bad)


def test_adaptive_builder_properties():
    f = w.binary_polytrope_128()
    leaves = oracle.build_adaptive_leaves(f.boxmax, 3, 1e-4)
    assert oracle.is_balanced(leaves)
    lo = leaves[:, 1:4] / (1 << leaves[:, 0:1]) - 0.5
    hi = lo + 1.0 / (1 << leaves[:, 0:1])
    bm = f.boxmax(lo, hi)
    coarse = leaves[:, 0] < 3
    assert np.all(bm[coarse] <= 1e-4)  # unrefined leaves satisfy the criterion
    assert np.any(leaves[:, 0] == 3) and np.any(leaves[:, 0] < 3)
    # tiling: volumes add up to the unit box
    assert np.isclose(np.sum(8.0 ** -leaves[:, 0]), 1.0)
    oracle.Tree(leaves, w.leaf_density(f, leaves))  # the oracle tree accepts it


# --------------------------------------------------------------------------
# the paper's static-sphere residuals
# --------------------------------------------------------------------------

@pytest.mark.slow
def test_uniform_sphere_residuals_against_paper_table():
    """Sec. 3.4: sphere of radius 0.25 and mass 1 on a 64^3 grid.

    Reading: the paper's grid voxelisation is unspecified, so the density is
    sampled at cell centres and renormalised to total mass 1.  The mean residual
    of the FMM against the discrete N^2 sum (its truncation error) is compared
    with the paper's converged means, and the residual against the closed form
    with the paper's 64^3 row, each within a factor 3."""
    table = json.load(open(os.path.join(HERE, "golden", "sphere_residuals.json")))["rows"]
    paper = {(int(r[0]), float(r[1])): r for r in table}
    lev = 3
    n = 8 << lev
    f = w.UniformSphere()
    g0 = w.uniform_grid(f, lev)
    inside = g0 > 1e-9
    rho = np.where(inside, g0 / (g0[inside].sum() / n ** 3), g0)
    t = oracle.Tree(w.uniform_leaves(lev), w.grid_to_leaves(rho))
    x, m = t.leaf_cells()
    from helpers import grid_ids

    G = np.arange(n ** 3).reshape(n, n, n)
    ids = grid_ids(lev, G[:, :, n // 2].ravel())
    pdir, _ = oracle.direct_points(x, m, x[:, ids])
    c = w.cell_centres(lev)
    X, Y = np.meshgrid(c, c, indexing="ij")
    pan = f.potential(X, Y, c[n // 2] + 0 * X).ravel()
    means = {}
    for theta in (0.5, 0.35):
        phi, _ = t.solve(theta=theta, sample=ids)
        e_fmm = np.abs((phi - pdir) / pdir)
        means[theta] = e_fmm.mean()
        conv = paper[(512, 0.5)] if theta == 0.5 else paper[(256, 0.35)]
        assert conv[3] / 3 < e_fmm.mean() < 3 * conv[3], (theta, e_fmm.mean())
        if theta == 0.5:
            e_an = np.abs((phi - pan) / pan)
            assert paper[(64, 0.5)][3] / 3 < e_an.mean() < 3 * paper[(64, 0.5)][3]
            # most common residual about 1e-4 (histogram peak)
            hist, edges = np.histogram(np.log10(e_fmm), bins=np.arange(-8, 0, 0.5))
            peak = 10 ** edges[np.argmax(hist)]
            assert 1e-5 <= peak <= 1e-3
    assert means[0.35] < means[0.5]


def _sphere_plane(lev):
    """Sec. 3.4 sphere on the uniform grid of `lev` (cell-centre sampling,
    renormalised to mass 1): the oracle tree, target ids on the equatorial
    plane (every corner of the square enclosing the sphere within 3 cells,
    the central 8 x 8 block, and every 4th cell of the plane) and the exact
    N^2 potential there."""
    from helpers import grid_ids

    n = 8 << lev
    f = w.UniformSphere()
    g0 = w.uniform_grid(f, lev)
    inside = g0 > 1e-9
    rho = np.where(inside, g0 / (g0[inside].sum() / n ** 3), g0)
    t = oracle.Tree(w.uniform_leaves(lev), w.grid_to_leaves(rho))
    c = w.cell_centres(lev)
    sel = np.zeros((n, n), dtype=bool)
    sel[::4, ::4] = True
    sel[n // 2 - 4:n // 2 + 4, n // 2 - 4:n // 2 + 4] = True
    lo, hi = n // 4 - 3, n // 4 + 3  # cells within 3 of x = -0.25 (index n/4 - 1/2)
    for a in (slice(lo, hi), slice(n - hi, n - lo)):
        for b in (slice(lo, hi), slice(n - hi, n - lo)):
            sel[a, b] = True
    ii, jj = np.nonzero(sel)
    G = np.arange(n ** 3).reshape(n, n, n)
    ids = grid_ids(lev, G[ii, jj, n // 2])
    x, m = t.leaf_cells()
    pdir, _ = oracle.direct_points(x, m, x[:, ids])
    return t, ids, pdir, c[ii], c[jj], 1.0 / n


@pytest.mark.slow
def test_uniform_sphere_maxima_sec34():
    """Sec. 3.4, the maxima of the static-sphere residuals: the largest
    residual sits at the corners of the square that encloses the sphere, does
    not fall with resolution (coarse levels interact the same way at every
    resolution) and falls with theta.

    The printed opening test is strict (cells |d| = 2 widths apart are not
    well separated at theta = 0.5); the table's behaviour matches the
    non-strict test (theta' <= theta), obtained here with theta = 0.5 + 1e-9
    (the same test with |d| = 2 admitted).  Under both tests the maximum does
    not fall from 64^3 to 128^3; under the non-strict one it sits at a corner
    of that square and shrinks by more than 3x at theta = 0.35 (the table:
    4x).  The magnitudes stay below the table's (3.7e-3 / 4.4e-3 against
    2.66e-2 / 3.23e-2); the design notes discuss the gap."""
    NONSTRICT = 0.5 + 1e-9
    res = {}
    for lev in (3, 4):
        t, ids, pdir, X, Y, h = _sphere_plane(lev)
        for theta in (0.5, NONSTRICT, 0.35):
            phi, _ = t.solve(theta=theta, sample=ids)
            e = np.abs((phi - pdir) / pdir)
            k = int(np.argmax(e))
            res[lev, theta] = (float(e.max()), float(X[k]), float(Y[k]), h, float(e.mean()))
            print(f"sphere {8 << lev}^3 theta={theta:.10f}: max {e.max():.3e} at ({X[k]:+.4f}, {Y[k]:+.4f})")
    for theta in (0.5, NONSTRICT, 0.35):
        assert res[4, theta][0] >= 0.9 * res[3, theta][0], theta  # not falling with resolution
    for lev in (3, 4):
        for theta in (NONSTRICT, 0.35):
            mx, x, y, h, _ = res[lev, theta]
            # at a corner of the square enclosing the sphere (|x|, |y| = 0.25)
            assert abs(abs(x) - 0.25) <= 2 * h and abs(abs(y) - 0.25) <= 2 * h, (lev, theta, x, y)
        assert res[lev, 0.35][0] < res[lev, NONSTRICT][0] / 3.0
        # the FMM error of every reading stays at truncation level
        assert res[lev, NONSTRICT][0] < 1e-2 and res[lev, 0.5][0] < 2e-3


# --------------------------------------------------------------------------
# coupling to the hydrodynamic update (Sec. 2.3)
# --------------------------------------------------------------------------

def test_coupling_sources_cancel_globally():
    """With phi, dphi/dt and g from a symmetric pair sum (the direct N^2 sum),
    the source terms integrate to zero: sum rho g = 0 (action = reaction),
    sum (phi drho/dt - rho dphi/dt) = 0 (K_ij = K_ji), and
    sum rho Omega.(x cross g) = Omega . (net torque) = 0 (central forces).
    A sign error in any of the terms breaks one of these."""
    rng = np.random.default_rng(41)
    leaves, f = random_amr_leaves(41, max_level=2, n_stars=1)
    rho = w.leaf_density(f, leaves).ravel()
    drho = rng.standard_normal(rho.size) * rho
    t = oracle.Tree(leaves, rho.reshape(-1, 512))
    x, m = t.leaf_cells()
    vol = m / rho
    phi, g = oracle.direct(x, m)
    dphi, _ = oracle.direct(x, drho * vol)
    omega = np.array([0.3, -0.2, 1.1])
    s = rng.standard_normal((3, rho.size))
    S_s, S_E = oracle.coupling.gravity_sources(omega, x, rho, s, phi, g, drho, dphi)
    S_s0, S_E0 = oracle.coupling.gravity_sources(np.zeros(3), x, rho, np.zeros_like(s), phi, g, drho, dphi)
    scale_f = np.sum(vol * rho * np.linalg.norm(g, axis=0))
    assert np.linalg.norm((vol * S_s0).sum(1)) < 1e-13 * scale_f
    scale_e = np.sum(vol * (np.abs(phi * drho) + np.abs(rho * dphi)))
    assert abs((vol * S_E0).sum()) < 1e-13 * scale_e
    rot = (vol * (S_E - S_E0)).sum()
    scale_r = np.linalg.norm(omega) * np.sum(vol * rho * np.linalg.norm(x, axis=0) * np.linalg.norm(g, axis=0))
    assert abs(rot) < 1e-13 * scale_r
    # the rotation term of the momentum source is Omega x s exactly
    assert np.allclose(S_s - S_s0, np.cross(omega[:, None], s, axis=0), rtol=0, atol=1e-15 * np.abs(s).max())
    # with the multipole solve the same cancellations hold to rounding (momentum and torque conserved)
    p_f, g_f = t.solve()
    S_sf, S_Ef = oracle.coupling.gravity_sources(omega, x, rho, np.zeros_like(s), p_f, g_f)
    assert np.linalg.norm((vol * S_sf).sum(1)) < 1e-13 * scale_f
    assert abs((vol * S_Ef).sum()) < 1e-13 * scale_r


def test_energy_update_conserves_total_energy():
    """E + 1/2 rho phi is unchanged by a potential update (Sec. 2.3)."""
    rng = np.random.default_rng(42)
    rho = rng.uniform(0.1, 1.0, 1000)
    E = rng.uniform(1.0, 2.0, 1000)
    pb, pa = -rng.uniform(1, 2, 1000), -rng.uniform(1, 2, 1000)
    E2 = oracle.coupling.energy_update(E, rho, pb, pa)
    assert np.allclose(E2 + 0.5 * rho * pa, E + 0.5 * rho * pb, rtol=1e-15, atol=0)


def test_coupling_rotation_term_is_power_of_the_torque():
    """The rotation part of the energy source integrates to Omega . T with T the
    gravitational torque diagnostic sum x cross rho g (Sec. 4); with the
    correction off T != 0, which fixes the term's sign and orientation."""
    leaves, f = random_amr_leaves(44, max_level=2, n_stars=2)
    rho = w.leaf_density(f, leaves).ravel()
    t = oracle.Tree(leaves, rho.reshape(-1, 512))
    x, m = t.leaf_cells()
    vol = m / rho
    phi, g = t.solve(amc=False)
    omega = np.array([0.4, -0.7, 0.2])
    _, S_E = oracle.coupling.gravity_sources(omega, x, rho, np.zeros_like(g), phi, g)
    st = oracle.stats(x, m, g)
    T = st["T"]
    tol = 1e-13 * np.linalg.norm(omega) * st["ST"]  # rounding of two sums with heavy cancellation
    assert abs(omega @ T) > 1e4 * tol  # the uncorrected torque is resolved
    assert abs((vol * S_E).sum() - omega @ T) < tol


# --------------------------------------------------------------------------
# time derivative of the potential (Sec. 2.1: the FMM applied to the density
# rate, expanded about the density's centres of mass)
# --------------------------------------------------------------------------

def _source_case(seed, max_level=2, n_stars=2):
    leaves, f = random_amr_leaves(seed, max_level=max_level, n_stars=n_stars)
    rng = np.random.default_rng(seed)
    rho = w.leaf_density(f, leaves) + 1e-3 * rng.uniform(size=(len(leaves), 512))
    src = rng.standard_normal(rho.shape) * rho  # a signed density rate
    return leaves, rho, src


def test_source_solve_cubic_kernel_is_exact():
    """For a cubic kernel a third-order expansion of the signed source about
    the density's centres (where its dipole does not vanish) is exact, so the
    result equals brute force; a dropped or mis-signed dipole term in the
    upward shift or in the multipole-to-local step fails this."""
    leaves, rho, src = _source_case(51)
    t = oracle.Tree(leaves, rho)
    rng = np.random.default_rng(51)
    coef = rng.standard_normal(20)
    x, m = t.leaf_cells()
    vol = m / rho.ravel()
    for theta in (0.5, 0.34):
        dphi = t.solve_source(src, theta=theta, kernel=coef)
        pr, _ = poly_direct(coef, x, src.ravel() * vol)
        assert np.max(np.abs(dphi - pr)) / np.max(np.abs(pr)) < 1e-11
    # the expansion centres are the density's: interior cells carry a dipole
    dip = [t.cell_moments(0, i, j, k) for i in range(8) for j in range(8) for k in range(8)]
    m_max = max(abs(mo["m"]) for mo in dip)
    assert max(np.linalg.norm(mo["M1"]) for mo in dip) > 1e-3 * m_max / 8


def test_source_solve_energy_terms_cancel():
    """sum_i (phi_i mdot_i - m_i dphi_i) = 0: the density and its rate go
    through the same symmetric discrete operator (Sec. 2.1), although each
    solve differs from the exact N^2 sum at truncation level."""
    leaves, rho, src = _source_case(52)
    t = oracle.Tree(leaves, rho)
    x, m = t.leaf_cells()
    md = src.ravel() * (m / rho.ravel())
    for theta in (0.5, 0.34):
        phi, _ = t.solve(theta=theta)
        dphi = t.solve_source(src, theta=theta)
        scale = np.sum(np.abs(phi * md)) + np.sum(np.abs(m * dphi))
        assert abs(np.dot(phi, md) - np.dot(m, dphi)) < 1e-14 * scale
        dd, _ = oracle.direct(x, md)
        trunc = np.max(np.abs(dphi - dd)) / np.max(np.abs(dd))
        assert 1e-9 < trunc < 1e-2  # not a direct sum in disguise


def test_source_solve_special_cases():
    """src = rho gives phi; the constant kernel counts every pair once; a
    power-of-two scaling is exact; a sampled solve equals the full one."""
    leaves, rho, src = _source_case(53, n_stars=1)
    t = oracle.Tree(leaves, rho)
    phi, _ = t.solve()
    same = t.solve_source(rho)
    assert np.max(np.abs(same - phi)) < 1e-13 * np.max(np.abs(phi))
    coef = np.zeros(20)
    coef[0] = 1.0
    x, m = t.leaf_cells()
    md = src.ravel() * (m / rho.ravel())
    for theta in (0.5, 0.9):
        c = t.solve_source(src, theta=theta, kernel=coef)
        assert np.max(np.abs(c + (md.sum() - md))) < 1e-12 * np.abs(md).sum()
    d1 = t.solve_source(src)
    assert np.array_equal(t.solve_source(4.0 * src), 4.0 * d1)
    sample = np.random.default_rng(5).choice(d1.size, 300, replace=False)
    assert np.array_equal(t.solve_source(src, sample=sample), d1[sample])
