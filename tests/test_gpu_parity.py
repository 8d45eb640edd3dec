"""GPU parity of the HIP library against the CPU oracle (FP64).

Bar (FP64): e_phi = max_i |dphi_i| / |phi_i| <= 1e-12 (phi < 0 everywhere)
and e_g = max_i |dg_i| / max_i |g_i| <= 1e-12 (normwise, g -> 0 near centres).
Pair counts are integers and must match the oracle's recursion exactly.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2101_08226_amd as lib
import workloads as w
from helpers import random_amr_leaves, zero_block_density

pytestmark = pytest.mark.gpu
TOL = 1e-12
# batch-fitted work shapes against each tree's own plan: the same FP64 sums
# taken in another order; a few thousand terms per target bound the relative
# change by about n * 2^-53 ~ 1e-13
FITTED_TOL = 1e-13


def say(*a):
    print("[gpu-parity]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = lib.Context(0)
    yield c
    c.close()


def errs(phi, g, phi_ref, g_ref):
    e_phi = float(np.max(np.abs(phi - phi_ref) / np.abs(phi_ref)))
    e_g = float(np.max(np.abs(g - g_ref)) / np.max(np.abs(g_ref)))
    return e_phi, e_g


def gpu_solve(ctx, tree, **kw):
    phi, g, st = ctx.solve(tree, **kw)
    return phi.cpu().numpy(), g.cpu().numpy(), st


def check_counts(st, t_orc):
    m2l, direct, ll = t_orc.last_counts(split=True)
    assert st["m2l_pairs"] == m2l - ll
    assert st["direct_pairs"] == direct + ll


def uniform_case(ctx, rho, theta, amc=True, counts=True):
    n = rho.shape[0]
    level = int(np.log2(n // 8))
    say(f"uniform n={n} theta={theta} amc={amc}")
    tree = ctx.uniform_tree(rho)
    phi, g, st = gpu_solve(ctx, tree, theta=theta, amc=amc)
    tree.destroy()
    t = oracle.Tree(w.uniform_leaves(level), w.grid_to_leaves(rho))
    p_ref, g_ref = t.solve(theta=theta, amc=amc)
    phi_l = w.grid_to_leaves(phi.reshape(n, n, n)).ravel()
    g_l = np.stack([w.grid_to_leaves(g[a].reshape(n, n, n)).ravel() for a in range(3)])
    e = errs(phi_l, g_l, p_ref, g_ref)
    say(f"  e_phi={e[0]:.2e} e_g={e[1]:.2e} torque={st['torque']:.2e} force={st['force']:.2e}")
    if counts:
        check_counts(st, t)
    return e, st


def test_single_leaf(ctx):
    rho = np.random.default_rng(1).uniform(0.5, 2.0, (8, 8, 8))
    e, st = uniform_case(ctx, rho, 0.5)
    assert e[0] <= TOL and e[1] <= TOL


@pytest.mark.parametrize("theta", [0.5, 0.34])
def test_c1_noisy_sphere_16(ctx, theta):
    e, st = uniform_case(ctx, w.noisy_sphere_16(), theta)
    assert e[0] <= TOL and e[1] <= TOL
    assert st["torque"] < 1e-13 and st["force"] < 1e-13


@pytest.mark.parametrize("amc", [True, False])
def test_uniform_32_random(ctx, amc):
    rho = np.random.default_rng(2).uniform(0.0, 1.0, (32, 32, 32))
    e, st = uniform_case(ctx, rho, 0.5, amc=amc)
    assert e[0] <= TOL and e[1] <= TOL
    if amc:
        assert st["torque"] < 1e-13
    else:
        assert st["torque"] > 1e-10


def test_uniform_64_binary_polytrope(ctx):
    rho = w.uniform_grid(w.binary_polytrope(0.12, 0.10, 0.35, 0.7), 3)
    e, st = uniform_case(ctx, rho, 0.5)
    assert e[0] <= TOL and e[1] <= TOL
    assert st["torque"] < 1e-13


@pytest.mark.parametrize("seed,max_level", [(21, 2), (22, 3), (23, 3)])
def test_adaptive_random(ctx, seed, max_level):
    leaves, f = random_amr_leaves(seed, max_level=max_level, n_stars=2)
    say(f"adaptive seed={seed} max_level={max_level} leaves={len(leaves)}")
    tree = ctx.adaptive_tree(f, max_level, 1e-4)
    assert np.array_equal(tree.leaves(), leaves)
    for theta in (0.5, 0.34):
        phi, g, st = gpu_solve(ctx, tree, theta=theta)
        t = oracle.Tree(leaves, w.leaf_density(f, leaves))
        p_ref, g_ref = t.solve(theta=theta)
        e = errs(phi, g, p_ref, g_ref)
        say(f"  theta={theta} e_phi={e[0]:.2e} e_g={e[1]:.2e} torque={st['torque']:.2e}")
        assert e[0] <= TOL and e[1] <= TOL
        check_counts(st, t)
        assert st["torque"] < 1e-13 and st["force"] < 1e-13
    tree.destroy()


@pytest.mark.parametrize("theta", [0.5, 0.34])
def test_massless_cells(ctx, theta):
    """Reading R11: root and level-1 cells without mass (all their leaf
    cells at density 0) expand about their geometric centres, carry no
    moments and skip the correction as targets; massless leaf cells are still
    targets."""
    rho = zero_block_density(5)
    e, st = uniform_case(ctx, rho, theta)
    assert e[0] <= TOL and e[1] <= TOL
    assert st["torque"] < 1e-13 and st["force"] < 1e-13


@pytest.mark.parametrize("theta", [0.7, 0.5 + 1e-9])
def test_other_opening_angles(ctx, theta):
    """Opening angles beyond the two of the paper's runs: 0.7 (fewer
    multipole pairs, more direct ones) and 0.5 + 1e-9, the non-strict
    reading of the opening test at 0.5 (cells two widths apart become well
    separated), on a uniform and an adaptive tree."""
    e, st = uniform_case(ctx, w.uniform_grid(w.binary_polytrope(0.12, 0.10, 0.35, 0.7), 2), theta)
    assert e[0] <= TOL and e[1] <= TOL
    assert st["torque"] < 1e-13 and st["force"] < 1e-13
    leaves, f = random_amr_leaves(22, max_level=3, n_stars=2)
    tree = ctx.adaptive_tree(f, 3, 1e-4)
    phi, g, st = gpu_solve(ctx, tree, theta=theta)
    tree.destroy()
    t = oracle.Tree(leaves, w.leaf_density(f, leaves))
    p_ref, g_ref = t.solve(theta=theta)
    e = errs(phi, g, p_ref, g_ref)
    # above 1/sqrt(3) cells touching at a corner are well separated and the
    # method's own result can come out near zero (even positive) at cells
    # next to concentrated mass (oracle pin test_corner_neighbours_above_
    # inverse_sqrt3): phi is no longer of one sign, so it is compared
    # normwise there, like g
    e_phi_norm = float(np.max(np.abs(phi - p_ref)) / np.max(np.abs(p_ref)))
    say(f"  adaptive theta={theta} e_phi={e[0]:.2e} (normwise {e_phi_norm:.2e}) e_g={e[1]:.2e} "
        f"torque={st['torque']:.2e}")
    assert (e_phi_norm if theta > 3 ** -0.5 else e[0]) <= TOL and e[1] <= TOL
    check_counts(st, t)
    assert st["torque"] < 1e-13 and st["force"] < 1e-13


# Mixed precision (FP32 near field and FP32 bulk of the LDS-staged multipole
# work, accumulated in FP32; FP64 moments, the root's and level 1's
# per-wavefront multipole work, the correction's accumulation and the final
# accumulation): each bound is 4x the largest error measured on the GPU over
# the mixed cases of this file (e_phi 2.67e-7 on the sampled level-6 tree,
# e_g 4.54e-7 on the sampled level-7 tree), and the torque bound 4x the
# largest relative torque (3.21e-9, sampled level-6 tree).
MIXED_PHI = 1.1e-6
MIXED_G = 1.9e-6
MIXED_TORQUE = 1.3e-8


@pytest.mark.parametrize("case", ["c1", "poly64", "amr"])
def test_mixed_precision_bounds(ctx, case):
    if case == "c1":
        rho = w.noisy_sphere_16()
    elif case == "poly64":
        rho = w.uniform_grid(w.binary_polytrope(0.12, 0.10, 0.35, 0.7), 3)
    if case in ("c1", "poly64"):
        n = rho.shape[0]
        level = int(np.log2(n // 8))
        tree = ctx.uniform_tree(rho)
        t = oracle.Tree(w.uniform_leaves(level), w.grid_to_leaves(rho))
        to_leaf = lambda a: w.grid_to_leaves(a.reshape(n, n, n)).ravel()  # noqa: E731
    else:
        leaves, f = random_amr_leaves(22, max_level=3, n_stars=2)
        tree = ctx.adaptive_tree(f, 3, 1e-4)
        t = oracle.Tree(leaves, w.leaf_density(f, leaves))
        to_leaf = lambda a: a  # noqa: E731
    say(f"mixed {case}")
    phi, g, st = gpu_solve(ctx, tree, theta=0.5, precision=lib.OCTO_MIXED)
    p64, g64, st64 = gpu_solve(ctx, tree, theta=0.5, precision=lib.OCTO_FP64)
    tree.destroy()
    p_ref, g_ref = t.solve(theta=0.5)
    phi_l = to_leaf(phi)
    g_l = np.stack([to_leaf(g[a]) for a in range(3)])
    e = errs(phi_l, g_l, p_ref, g_ref)
    say(f"  mixed e_phi={e[0]:.2e} e_g={e[1]:.2e} torque={st['torque']:.2e} (fp64 torque {st64['torque']:.2e})")
    assert e[0] <= MIXED_PHI and e[1] <= MIXED_G
    assert st["torque"] < MIXED_TORQUE and st["force"] < MIXED_TORQUE
    assert st["m2l_pairs"] == st64["m2l_pairs"] and st["direct_pairs"] == st64["direct_pairs"]


def test_explicit_leaf_order(ctx):
    """octo_tree_build keeps the caller's leaf order (shuffled here)."""
    leaves, f = random_amr_leaves(31, max_level=2, n_stars=1)
    perm = np.random.default_rng(31).permutation(len(leaves))
    lv = leaves[perm]
    rho = w.leaf_density(f, lv)
    say(f"explicit leaves={len(lv)}")
    tree = ctx.tree(lv, rho)
    phi, g, st = gpu_solve(ctx, tree)
    tree.destroy()
    p_ref, g_ref = oracle.Tree(lv, rho).solve()
    e = errs(phi, g, p_ref, g_ref)
    assert e[0] <= TOL and e[1] <= TOL


def test_batch_and_async_equal_single(ctx):
    rng = np.random.default_rng(4)
    grids = [rng.uniform(0.1, 1.0, (n, n, n)) for n in (16, 32, 16)]
    trees = [ctx.uniform_tree(r) for r in grids]
    say("batch of 3 trees")
    single = [gpu_solve(ctx, t)[:2] for t in trees]
    outs, sts = ctx.solve_batch(trees)
    for (p, g), (ps, gs) in zip(outs, single):
        assert np.array_equal(p.cpu().numpy(), ps) and np.array_equal(g.cpu().numpy(), gs)
    outs2, _ = ctx.solve_batch(trees)  # graph replay
    for (p, g), (ps, gs) in zip(outs2, single):
        assert np.array_equal(p.cpu().numpy(), ps) and np.array_equal(g.cpu().numpy(), gs)
    say("async requests")
    import torch

    res = []
    for t in trees + trees[:1]:
        phi = torch.empty(t.n_leaf_cells, dtype=torch.float64, device="cuda")
        g = torch.empty((3, t.n_leaf_cells), dtype=torch.float64, device="cuda")
        tk = lib.octo_submit(ctx.handle, t.handle, lib.make_opts(), phi.data_ptr(), g.data_ptr())
        res.append((tk, phi, g))
    for i, (tk, phi, g) in enumerate(res):
        st = lib.octo_wait(ctx.handle, tk)
        ps, gs = single[i % 3]
        assert np.array_equal(phi.cpu().numpy(), ps) and np.array_equal(g.cpu().numpy(), gs)
        assert st.n_leaf_cells == phi.numel()
    for t in trees:
        t.destroy()


def test_served_stream_equals_single():
    """The request server (parallel tree builds, budget admission, requests
    merged into launch waves) returns for every request exactly what a solve
    of that tree alone returns, in both precisions."""
    from paper_2101_08226_amd import serve

    c = lib.Context(0, hbm_budget=160 << 20)  # a few trees at a time: admission waits
    try:
        stream = w.mixes.served_stream(14, 200.0, seed=77, min_cells=4096, max_cells=1 << 17,
                                       count_leaves=lambda f, lv: 512 * len(lib.octo_host_adaptive_leaves(f, lv, 1e-4)))
        payloads = []
        for r in stream:
            lv = lib.octo_host_adaptive_leaves(r.field, r.max_level, 1e-4)
            payloads.append(serve.Payload(r.index, r.arrival, lv, w.leaf_density(r.field, lv), r.precision))
        say(f"served stream: {len(payloads)} requests, {sum(p.leaves.shape[0] for p in payloads) * 512} cells")
        rec, outs, wall = serve.serve(c, payloads, keep_outputs=True, builders=4, lookahead=6, time_limit=60.0)
        assert sorted(r.index for r in rec) == list(range(len(payloads)))
        for p in payloads:
            t = c.tree(p.leaves, p.rho)
            phi, g, _ = c.solve(t, precision=p.precision)
            assert np.array_equal(outs[p.index][0], phi.cpu().numpy()), p.index
            assert np.array_equal(outs[p.index][1], g.cpu().numpy()), p.index
            t.destroy()
        say(f"  wall {wall * 1e3:.1f} ms, p50 {serve.summary(rec, wall)['p50_ms']:.2f} ms")
    finally:
        c.close()


def test_served_tight_budget():
    """Admission with a budget just above the largest tree (plus its work
    plan): trees built ahead and launch waves compete for the memory, waves
    shrink to what fits, and every request still completes with the result
    of its solve alone."""
    from paper_2101_08226_amd import serve

    stream = w.mixes.served_stream(10, 400.0, seed=78, min_cells=4096, max_cells=1 << 16,
                                   count_leaves=lambda f, lv: 512 * len(lib.octo_host_adaptive_leaves(f, lv, 1e-4)))
    payloads = []
    for r in stream:
        lv = lib.octo_host_adaptive_leaves(r.field, r.max_level, 1e-4)
        payloads.append(serve.Payload(r.index, r.arrival, lv, w.leaf_density(r.field, lv), r.precision))
    probe = lib.Context(0)
    try:
        sizes, single = [], {}
        for p in payloads:
            t = probe.tree(p.leaves, p.rho)
            sizes.append(t.bytes)
            phi, g, _ = probe.solve(t, precision=p.precision)
            single[p.index] = (phi.cpu().numpy(), g.cpu().numpy())
            t.destroy()
    finally:
        probe.close()
    budget = int(max(sizes) * 1.3)
    say(f"tight budget: {budget} bytes, trees {min(sizes)}..{max(sizes)} bytes")
    c = lib.Context(0, hbm_budget=budget)
    try:
        rec, outs, wall = serve.serve(c, payloads, keep_outputs=True, builders=4, lookahead=6, time_limit=60.0)
        used, _ = c.memory()
    finally:
        c.close()
    assert sorted(r.index for r in rec) == list(range(len(payloads)))
    for p in payloads:
        assert np.array_equal(outs[p.index][0], single[p.index][0]), p.index
        assert np.array_equal(outs[p.index][1], single[p.index][1]), p.index
    assert used == 0


def test_errors(ctx):
    rho = np.ones((16, 16, 16))
    tree = ctx.uniform_tree(rho)
    with pytest.raises(lib.OctoError, match="UNSUPPORTED"):
        ctx.solve(tree, theta=0.2)
    with pytest.raises(lib.OctoError, match="UNSUPPORTED"):
        ctx.solve(tree, theta=1.0)
    tree.destroy()
    bad = rho.copy()
    bad[1, 2, 3] = -1.0
    with pytest.raises(lib.OctoError, match="INVALID"):
        ctx.uniform_tree(bad)
    with pytest.raises(lib.OctoError, match="INVALID"):
        ctx.tree(w.uniform_leaves(1)[:7], np.ones((7, 512)))


def test_budget_admission():
    c = lib.Context(0, hbm_budget=64 << 20)
    try:
        t = c.uniform_tree(np.ones((32, 32, 32)))
        with pytest.raises(lib.OctoError, match="BUDGET"):
            c.uniform_tree(np.ones((128, 128, 128)))
        used, budget = c.memory()
        assert used <= budget
        t.destroy()
    finally:
        c.close()


def test_c2_full_size_sampled(ctx):
    """128^3 binary polytrope (16^3 sub-grids), the benchmark's workload:
    every output against the oracle's sampled solve at 400 cells, plus the
    invariants over all cells."""
    rho = w.uniform_grid(w.binary_polytrope_128(), 4)
    say("c2 128^3 full solve")
    tree = ctx.uniform_tree(rho)
    phi, g, st = gpu_solve(ctx, tree, theta=0.5)
    tree.destroy()
    n = 128
    rng = np.random.default_rng(7)
    sel = rng.choice(n ** 3, 400, replace=False)
    from helpers import grid_ids

    ids = grid_ids(4, sel)
    t = oracle.Tree(w.uniform_leaves(4), w.grid_to_leaves(rho))
    p_ref, g_ref = t.solve(theta=0.5, sample=ids)
    e_phi = float(np.max(np.abs(phi[sel] - p_ref) / np.abs(p_ref)))
    e_g = float(np.max(np.abs(g[:, sel] - g_ref)) / np.max(np.abs(g_ref)))
    say(f"  e_phi={e_phi:.2e} e_g={e_g:.2e} torque={st['torque']:.2e} pairs={st['m2l_pairs']} {st['direct_pairs']}")
    assert e_phi <= TOL and e_g <= TOL
    assert st["torque"] < 1e-13 and st["force"] < 1e-13
    assert st["m2l_pairs"] == 64121280 and st["direct_pairs"] == 534396416
    assert 0 < st["m2l_lds_pairs"] < st["m2l_pairs"]


@pytest.mark.parametrize("max_level", [6, 7])
def test_c3_adaptive_full_size_sampled(ctx, max_level):
    """The c2 field refined adaptively to level 6 (7736 leaf sub-grids, 3.96M
    leaf cells) and to level 7 (39,012 leaf sub-grids, 20.0M leaf cells, the
    config's level 7 counted from the root sub-grid as level 0): sampled cells
    against the oracle, leaf list identical to the oracle's builder,
    invariants over all cells."""
    f = w.binary_polytrope_128()
    say(f"c3 adaptive level {max_level} build")
    tree = ctx.adaptive_tree(f, max_level, 1e-4)
    lv = tree.leaves()
    assert np.array_equal(lv, oracle.build_adaptive_leaves(f.boxmax, max_level, 1e-4))
    say(f"c3 solve leaves={len(lv)}")
    for prec in (lib.OCTO_FP64, lib.OCTO_MIXED):
        phi, g, st = gpu_solve(ctx, tree, theta=0.5, precision=prec)
        rng = np.random.default_rng(8)
        # half the samples in the stars (the two finest levels), half anywhere
        fine = np.nonzero(np.repeat(lv[:, 0] >= max_level - 1, 512))[0]
        sel = np.concatenate([rng.choice(fine, 200, replace=False), rng.choice(tree.n_leaf_cells, 200, replace=False)])
        if prec == lib.OCTO_FP64:
            t = oracle.Tree(lv, w.leaf_density(f, lv))
            p_ref, g_ref = t.solve(theta=0.5, sample=sel)
        e_phi = float(np.max(np.abs(phi[sel] - p_ref) / np.abs(p_ref)))
        e_g = float(np.max(np.abs(g[:, sel] - g_ref)) / np.max(np.abs(g_ref)))
        say(f"  prec={prec} e_phi={e_phi:.2e} e_g={e_g:.2e} torque={st['torque']:.2e} force={st['force']:.2e}")
        if prec == lib.OCTO_FP64:
            assert e_phi <= TOL and e_g <= TOL
            assert st["torque"] < 1e-13 and st["force"] < 1e-13
        else:
            assert e_phi <= MIXED_PHI and e_g <= MIXED_G
            assert st["torque"] < MIXED_TORQUE
    tree.destroy()


def test_c4_batched_mix(ctx):
    """The benchmark's batched workload itself: 256 uniform trees of 16^3,
    32^3 and 64^3 cells, each a seeded single or binary polytrope, solved in
    one batch: every tree bitwise equal to its own solve, in both precisions,
    and three trees (the largest of each size) against the oracle on sampled
    cells."""
    import torch

    mix = w.mixes.batched_mix(256)
    trees = [ctx.uniform_tree(w.uniform_grid(b.field, b.level)) for b in mix]
    say(f"c4 mix: {len(trees)} trees, {sum(t.n_leaf_cells for t in trees)} cells")
    for prec in (lib.OCTO_FP64, lib.OCTO_MIXED):
        outs, sts = ctx.solve_batch(trees, precision=prec)
        torch.cuda.synchronize()
        for i, t in enumerate(trees):
            p1, g1, st1 = gpu_solve(ctx, t, precision=prec)
            assert np.array_equal(outs[i][0].cpu().numpy(), p1) and np.array_equal(outs[i][1].cpu().numpy(), g1), i
            assert sts[i]["m2l_pairs"] == st1["m2l_pairs"] and sts[i]["direct_pairs"] == st1["direct_pairs"]
        say(f"  prec={prec}: batch == single for all trees, worst torque {max(s['torque'] for s in sts):.2e}")
        if prec == lib.OCTO_FP64:
            assert max(s["torque"] for s in sts) < 1e-13
        else:
            # 4x the worst mixed torque measured over the 256 trees (2.40e-8)
            assert max(s["torque"] for s in sts) < 1e-7
        # work shapes fitted to the batch: the same sums in another order
        ctx.set_batch_shapes(1)
        try:
            outs_f, sts_f = ctx.solve_batch(trees, precision=prec)
            torch.cuda.synchronize()
        finally:
            ctx.set_batch_shapes(0)
        worst = 0.0
        # mixed precision: the fitted shapes move level 1 from the FP64
        # per-wavefront kernel to the FP32 LDS-staged one, so the two results
        # are two mixed solves, each within MIXED_G of the oracle
        tol = FITTED_TOL if prec == lib.OCTO_FP64 else 2 * MIXED_G
        for i in range(len(trees)):
            e = errs(outs_f[i][0].cpu().numpy(), outs_f[i][1].cpu().numpy(), outs[i][0].cpu().numpy(),
                     outs[i][1].cpu().numpy())
            worst = max(worst, e[0], e[1])
            assert sts_f[i]["m2l_pairs"] == sts[i]["m2l_pairs"] and sts_f[i]["direct_pairs"] == sts[i]["direct_pairs"]
        say(f"  prec={prec}: fitted shapes vs own plans: worst relative difference {worst:.2e}")
        assert worst <= tol
        if prec == lib.OCTO_FP64:
            assert max(s["torque"] for s in sts_f) < 1e-13
            fp64 = outs_f  # the oracle check below takes the fitted-shape results
        else:
            assert max(s["torque"] for s in sts_f) < 1e-7
    from helpers import grid_ids

    rng = np.random.default_rng(10)
    for lev in (1, 2, 3):
        i = max((k for k, b in enumerate(mix) if b.level == lev), key=lambda k: trees[k].n_leaf_cells)
        n = 8 << lev
        rho = w.uniform_grid(mix[i].field, lev)
        sel = rng.choice(n ** 3, 200, replace=False)
        t = oracle.Tree(w.uniform_leaves(lev), w.grid_to_leaves(rho))
        p_ref, g_ref = t.solve(theta=0.5, sample=grid_ids(lev, sel))
        phi = fp64[i][0].cpu().numpy()[sel]
        g = fp64[i][1].cpu().numpy()[:, sel]
        e_phi = float(np.max(np.abs(phi - p_ref) / np.abs(p_ref)))
        e_g = float(np.max(np.abs(g - g_ref)) / np.max(np.abs(g_ref)))
        say(f"  tree {i} ({n}^3): e_phi={e_phi:.2e} e_g={e_g:.2e}")
        assert e_phi <= TOL and e_g <= TOL
    for t in trees:
        t.destroy()


def test_batch_per_tree_status(ctx):
    """octo_solve_batch reports each tree's outcome: refused entries (a NULL
    tree, a NULL output, a tree listed twice) get their own status and are
    skipped; the others are solved together, bitwise as alone."""
    import torch

    rng = np.random.default_rng(12)
    trees = [ctx.uniform_tree(rng.uniform(0.1, 1.0, (n, n, n))) for n in (16, 32)]
    single = [gpu_solve(ctx, t)[:2] for t in trees]
    outs = [(torch.empty(t.n_leaf_cells, dtype=torch.float64, device="cuda"),
             torch.empty((3, t.n_leaf_cells), dtype=torch.float64, device="cuda")) for t in trees]
    handles = [trees[0].handle, 0, trees[1].handle, trees[0].handle, trees[1].handle]
    phis = [outs[0][0].data_ptr(), outs[0][0].data_ptr(), outs[1][0].data_ptr(), outs[0][0].data_ptr(), 0]
    gs = [outs[0][1].data_ptr(), outs[0][1].data_ptr(), outs[1][1].data_ptr(), outs[0][1].data_ptr(),
          outs[1][1].data_ptr()]
    status = []
    say("batch with refused entries")
    sts = lib.octo_solve_batch(ctx.handle, handles, lib.make_opts(), phis, gs, True, status_out=status)
    torch.cuda.synchronize()
    assert status == [lib.OCTO_OK, lib.OCTO_E_INVALID, lib.OCTO_OK, lib.OCTO_E_INVALID, lib.OCTO_E_INVALID]
    for k, i in ((0, 0), (2, 1)):
        assert sts[k].n_leaf_cells == trees[i].n_leaf_cells
        assert np.array_equal(outs[i][0].cpu().numpy(), single[i][0])
        assert np.array_equal(outs[i][1].cpu().numpy(), single[i][1])
    # every entry refused: the call fails with the first entry's status
    status = []
    lib.octo_solve_batch(ctx.handle, [0, 0], lib.make_opts(), [0, 0], [0, 0], True, status_out=status)
    assert status == [lib.OCTO_E_INVALID, lib.OCTO_E_INVALID]
    with pytest.raises(lib.OctoError):
        lib.octo_solve_batch(ctx.handle, [trees[0].handle, trees[0].handle], lib.make_opts(), phis[:2], gs[:2], True)
    # bad options fail the whole call, for every tree
    status = []
    lib.octo_solve_batch(ctx.handle, [t.handle for t in trees], lib.make_opts(theta=0.2), phis[::2][:2], gs[::2][:2],
                         True, status_out=status)
    assert status == [lib.OCTO_E_UNSUPPORTED, lib.OCTO_E_UNSUPPORTED]
    for t in trees:
        t.destroy()


def test_device_stats(ctx):
    """octo_solve_device_stats: the same potential and acceleration as
    octo_solve, bit for bit, and the 9 reduction results in device memory
    equal to the host statistics of a solve that counts pairs (the counting
    pass changes no sum)."""
    import torch

    rho = w.uniform_grid(w.binary_polytrope(0.12, 0.10, 0.35, 0.7), 3)
    tree = ctx.uniform_tree(rho)
    for prec in (lib.OCTO_FP64, lib.OCTO_MIXED):
        phi, g, st = gpu_solve(ctx, tree, precision=prec)
        opts = lib.make_opts(0.5, 1.0, prec, True)
        d_phi = torch.empty(tree.n_leaf_cells, dtype=torch.float64, device="cuda")
        d_g = torch.empty((3, tree.n_leaf_cells), dtype=torch.float64, device="cuda")
        d_st = torch.full((9,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()  # the fill (torch's stream) before the library's stream writes
        for _ in range(2):  # capture, then graph replay
            lib.octo_solve_device_stats(ctx.handle, tree.handle, opts, d_phi.data_ptr(), d_g.data_ptr(),
                                        d_st.data_ptr())
            ctx.stream.synchronize()
            assert np.array_equal(d_phi.cpu().numpy(), phi) and np.array_equal(d_g.cpu().numpy(), g)
            v = d_st.cpu().numpy()
            host = np.array([st["total_mass"], *st["net_force"], *st["net_torque"], st["force_scale"],
                             st["torque_scale"]])
            assert np.array_equal(v, host), (v, host)
    tree.destroy()


def test_batch_mixed_sizes_and_precision(ctx):
    """Trees of different depths in one batch (levels 0-3 and adaptive): every
    result bitwise equal to its single solve, in both precisions; with work
    shapes fitted to the batch, equal to it to within rounding of the
    summation order, on graph replay too."""
    rng = np.random.default_rng(9)
    trees = [ctx.uniform_tree(rng.uniform(0.1, 1.0, (n, n, n))) for n in (8, 64, 16)]
    leaves, f = random_amr_leaves(24, max_level=3, n_stars=1)
    trees.append(ctx.adaptive_tree(f, 3, 1e-4))
    for prec in (lib.OCTO_FP64, lib.OCTO_MIXED):
        say(f"batch sizes prec={prec}")
        single = [gpu_solve(ctx, t, precision=prec)[:2] for t in trees]
        outs, sts = ctx.solve_batch(trees, precision=prec)
        for (p, g), (ps, gs) in zip(outs, single):
            assert np.array_equal(p.cpu().numpy(), ps) and np.array_equal(g.cpu().numpy(), gs)
        ctx.set_batch_shapes(1)
        try:
            first = None
            for _ in range(2):  # capture, then replay
                outs_f, sts_f = ctx.solve_batch(trees, precision=prec)
                got = [(p.cpu().numpy(), g.cpu().numpy()) for p, g in outs_f]
                tol = FITTED_TOL if prec == lib.OCTO_FP64 else 2 * MIXED_G  # see test_c4_batched_mix
                for (p, g), (ps, gs) in zip(got, single):
                    e = errs(p, g, ps, gs)
                    assert e[0] <= tol and e[1] <= tol, e
                if first is not None:
                    for (p, g), (p0, g0) in zip(got, first):
                        assert np.array_equal(p, p0) and np.array_equal(g, g0)
                first = got
            for a_, b_ in zip(sts_f, sts):
                assert a_["m2l_pairs"] == b_["m2l_pairs"] and a_["direct_pairs"] == b_["direct_pairs"]
        finally:
            ctx.set_batch_shapes(0)
    for t in trees:
        t.destroy()


def test_autotune_keeps_parity(ctx):
    """The autotuner changes only the work shape: results stay at parity."""
    rho = w.uniform_grid(w.binary_polytrope(0.12, 0.10, 0.35, 0.7), 3)
    tree = ctx.uniform_tree(rho)
    say("autotune 64^3")
    choice = tree.autotune(theta=0.5)
    say(f"  choice per level: {choice}")
    assert len(choice) == 4 and choice[-1] == -1 and all(c != -1 for c in choice[:-1])
    phi, g, st = gpu_solve(ctx, tree, theta=0.5)
    tree.destroy()
    t = oracle.Tree(w.uniform_leaves(3), w.grid_to_leaves(rho))
    p_ref, g_ref = t.solve(theta=0.5)
    phi_l = w.grid_to_leaves(phi.reshape(64, 64, 64)).ravel()
    g_l = np.stack([w.grid_to_leaves(g[a].reshape(64, 64, 64)).ravel() for a in range(3)])
    e = errs(phi_l, g_l, p_ref, g_ref)
    assert e[0] <= TOL and e[1] <= TOL
    check_counts(st, t)


def test_coupling_kernels(ctx):
    """Gravity source terms and energy update on the device equal the oracle's
    definitions (elementwise, FP64)."""
    import torch

    leaves, f = random_amr_leaves(43, max_level=3, n_stars=2)
    tree = ctx.adaptive_tree(f, 3, 1e-4)
    lv = tree.leaves()
    rho_h = w.leaf_density(f, lv).ravel()
    rng = np.random.default_rng(43)
    n = rho_h.size
    s_h = rng.standard_normal((3, n))
    drho_h = rng.standard_normal(n)
    dphi_h = rng.standard_normal(n)
    say("coupling kernels")
    phi, g, _ = ctx.solve(tree)
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    rho, s, drho, dphi = dev(rho_h), dev(s_h), dev(drho_h), dev(dphi_h)
    omega = np.array([0.1, 0.2, 0.9])
    src_s, src_e = ctx.gravity_sources(tree, omega, rho, s, phi, g, drho, dphi)
    x, _ = oracle.Tree(lv, rho_h.reshape(-1, 512)).leaf_cells()
    ref_s, ref_e = oracle.coupling.gravity_sources(omega, x, rho_h, s_h, phi.cpu().numpy(), g.cpu().numpy(), drho_h,
                                                   dphi_h)
    assert np.max(np.abs(src_s.cpu().numpy() - ref_s)) <= 1e-14 * np.max(np.abs(ref_s))
    assert np.max(np.abs(src_e.cpu().numpy() - ref_e)) <= 1e-14 * np.max(np.abs(ref_e))
    src_s0, src_e0 = ctx.gravity_sources(tree, omega, rho, s, phi, g)  # NULL time derivatives
    ref_s0, ref_e0 = oracle.coupling.gravity_sources(omega, x, rho_h, s_h, phi.cpu().numpy(), g.cpu().numpy())
    assert np.max(np.abs(src_e0.cpu().numpy() - ref_e0)) <= 1e-14 * np.max(np.abs(ref_e0))
    E = dev(rng.uniform(1, 2, n))
    E_h = E.cpu().numpy()
    pb = dev(-rng.uniform(1, 2, n))
    ctx.energy_update(tree, rho, pb, phi, E)
    ref = oracle.coupling.energy_update(E_h, rho_h, pb.cpu().numpy(), phi.cpu().numpy())
    assert np.max(np.abs(E.cpu().numpy() - ref)) <= 1e-15 * np.max(np.abs(ref))
    tree.destroy()


# --------------------------------------------------------------------------
# dphi/dt: the density rate as a second source (Sec. 2.1)
# Bar (FP64): max_i |d_i| / max_i |ref_i| <= 1e-12 (normwise: the rate and its
# potential change sign).  Mixed: MIXED_DPHI, 4x the largest error measured
# (5.74e-7, orbital rate on the adaptive level-3 tree at theta 0.34).
# --------------------------------------------------------------------------

MIXED_DPHI = 2.3e-6


def _dev(a):
    import torch

    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("seed,max_level,rate", [(21, 2, "noisy"), (22, 3, "orbital"), (23, 3, "noisy")])
def test_dphidt_parity(ctx, seed, max_level, rate):
    leaves, f = random_amr_leaves(seed, max_level=max_level, n_stars=2)
    say(f"dphidt seed={seed} max_level={max_level} rate={rate} leaves={len(leaves)}")
    tree = ctx.adaptive_tree(f, max_level, 1e-4)
    lv = tree.leaves()
    rho = w.leaf_density(f, lv)
    src = w.noisy_rate(rho, seed) if rate == "noisy" else w.leaf_density(w.OrbitalRate(f, 1.0, 1e-3), lv)
    t = oracle.Tree(lv, rho)
    x, m = t.leaf_cells()
    md = src.ravel() * (m / rho.ravel())
    drho = _dev(src.ravel())
    for theta in (0.5, 0.34):
        ref = t.solve_source(src, theta=theta)
        d64 = ctx.solve_dphidt(tree, drho, theta=theta).cpu().numpy()
        e = float(np.max(np.abs(d64 - ref)) / np.max(np.abs(ref)))
        phi, _, _ = gpu_solve(ctx, tree, theta=theta)
        scale = np.sum(np.abs(phi * md)) + np.sum(np.abs(m * d64))
        cancel = abs(np.dot(phi, md) - np.dot(m, d64)) / scale
        d32 = ctx.solve_dphidt(tree, drho, theta=theta, precision=lib.OCTO_MIXED).cpu().numpy()
        e32 = float(np.max(np.abs(d32 - ref)) / np.max(np.abs(ref)))
        say(f"  theta={theta} e={e:.2e} cancel={cancel:.2e} mixed e={e32:.2e}")
        assert e <= TOL
        assert cancel < 1e-13
        assert e32 <= MIXED_DPHI
    # the solve of the density itself is unaffected by an interleaved rate solve
    phi2, g2, _ = gpu_solve(ctx, tree, theta=0.5)
    p_ref, g_ref = t.solve(theta=0.5)
    e2 = errs(phi2, g2, p_ref, g_ref)
    assert e2[0] <= TOL and e2[1] <= TOL
    tree.destroy()


def test_dphidt_uniform_and_full_size(ctx):
    """32^3 random density with a noisy rate (every cell), then the 128^3
    binary with its orbital rate (sampled cells against the oracle, the
    cancellation over all cells)."""
    rng = np.random.default_rng(33)
    rho = rng.uniform(0.1, 1.0, (32, 32, 32))
    src = w.noisy_rate(rho, 33)
    say("dphidt uniform 32")
    tree = ctx.uniform_tree(rho)
    d = ctx.solve_dphidt(tree, _dev(src.ravel())).cpu().numpy()
    tree.destroy()
    t = oracle.Tree(w.uniform_leaves(2), w.grid_to_leaves(rho))
    ref = t.solve_source(w.grid_to_leaves(src))
    d_l = w.grid_to_leaves(d.reshape(32, 32, 32)).ravel()
    e = float(np.max(np.abs(d_l - ref)) / np.max(np.abs(ref)))
    say(f"  e={e:.2e}")
    assert e <= TOL

    f = w.binary_polytrope_128()
    rho = w.uniform_grid(f, 4)
    src = w.uniform_grid(w.OrbitalRate(f, 1.0, 1e-3), 4)
    say("dphidt c2 128^3")
    tree = ctx.uniform_tree(rho)
    d = ctx.solve_dphidt(tree, _dev(src.ravel())).cpu().numpy()
    phi, _, _ = gpu_solve(ctx, tree, theta=0.5)
    tree.destroy()
    vol = (1.0 / 128) ** 3
    m, md = rho.ravel() * vol, src.ravel() * vol
    scale = np.sum(np.abs(phi * md)) + np.sum(np.abs(m * d))
    cancel = abs(np.dot(phi, md) - np.dot(m, d)) / scale
    from helpers import grid_ids

    sel = np.random.default_rng(7).choice(128 ** 3, 300, replace=False)
    # the stars, where the rate lives
    star = np.nonzero(np.abs(src.ravel()) > 1e-3 * np.abs(src).max())[0]
    sel = np.concatenate([sel, np.random.default_rng(8).choice(star, 300, replace=False)])
    t = oracle.Tree(w.uniform_leaves(4), w.grid_to_leaves(rho))
    ref = t.solve_source(w.grid_to_leaves(src), sample=grid_ids(4, sel))
    e = float(np.max(np.abs(d[sel] - ref)) / np.max(np.abs(ref)))
    say(f"  e={e:.2e} cancel={cancel:.2e}")
    assert e <= TOL
    assert cancel < 1e-13


def test_profiling_modes(ctx):
    """Profiling (kernels one by one) gives the graph solve's results bit for
    bit; mode 1 keeps the statistics, mode 2 (timing only) zeroes them and
    still times every phase (64^3: the LDS-staged multipole kernel runs)."""
    rho = w.uniform_grid(w.binary_polytrope_128(), 3)
    tree = ctx.uniform_tree(rho)
    p0, g0, st0 = gpu_solve(ctx, tree)
    for mode in (1, 2):
        ctx.set_profiling(mode)
        try:
            p, g, st = gpu_solve(ctx, tree)
        finally:
            ctx.set_profiling(0)
        say(f"profiling {mode}: phases {[round(x, 4) for x in st['phase_ms']]}")
        assert np.array_equal(p, p0) and np.array_equal(g, g0)
        assert all(x > 0 for i, x in enumerate(st["phase_ms"]) if i != 6)  # [6]: statistics
        if mode == 1:
            assert st["m2l_pairs"] == st0["m2l_pairs"] and st["total_mass"] == st0["total_mass"]
        else:
            assert st["m2l_pairs"] == 0 and st["total_mass"] == 0.0 and st["n_leaf_cells"] == st0["n_leaf_cells"]
    for bad in (-1, 3):
        with pytest.raises(lib.OctoError, match="INVALID"):
            ctx.set_profiling(bad)
    tree.destroy()
