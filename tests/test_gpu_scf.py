"""GPU parity of the self-consistent-field iteration (Sec. 4.1) with the
oracle's SCF.

Bars.  One step (octo_scf_step) gets the same density and potential as the
oracle step: the centre and L1 cells must be identical, the scalars and the
new density agree to 1e-12 (relative, normwise for the density); both sides
round the same expressions in the same order, only the sums' order and pow's
last bit differ.  A whole run (octo_scf_run) solves for the potential with the
multipole method on each side (FP64 parity 1e-12); the iteration turns that
into differences of the constants of ~10 |phi| / |C - phi_c| times it and of
the density of n times that, so runs of a few iterations are held to 1e-9
(scalars relative, density and potential normwise) with identical cells.
Full sizes (the 128^3 grid of the benchmark and a 256^3 grid): the step
against the oracle step on oracle-made inputs; one iteration of the run
against the oracle's; longer runs by properties: the run's final potential is
the library's own solve of the returned density bit for bit, the stars' masses,
and the hydrostatic relation near the fixed point.
"""
import sys

import numpy as np
import pytest

import paper_2101_08226_amd as lib
import workloads as w
from helpers import fft_poisson
from oracle import scf as S

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-scf]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = lib.Context(0)
    yield c
    c.close()


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).to("cuda:0")


def _params(p: S.SCFParams, x_L1=0.0):
    return lib.make_scf_params(p.M1, p.M2, p.n, p.a0, p.f, p.K0, p.floor, p.G, x_L1)


def _model(level, M2=0.7, a0=0.4, R1=0.12, R2=0.1, f=0.9):
    # the stars' axis lies off the cell faces (y, z offsets unlike any
    # multiple of h/2 on these grids): each maximum the iteration takes then
    # has one clear winner, instead of cells that tie up to rounding, where
    # the two sides may legitimately pick different cells
    p = S.SCFParams(M1=1.0, M2=M2, a0=a0, f=f)
    rho0, p.K0 = w.scf_initial_binary(level, 1.0, M2, a0, R1, R2, yz=(0.0123, 0.0071))
    return p, rho0


SCALARS = ("omega", "K", "C1", "C2", "x_L1", "a", "mass1", "mass2")


def _cmp_state(sg: dict, so: S.SCFState, tol):
    assert (sg["c1"], sg["c2"], sg["l1"]) == (so.c1, so.c2, so.l1)
    for k in SCALARS:
        a, b = sg[k], getattr(so, k)
        assert abs(a - b) <= tol * abs(b), (k, a, b)


def _step_case(ctx, level, x_L1, phi_fn):
    p, rho0 = _model(level)
    rho = S.normalise(rho0, level, p, x_L1)
    phi = phi_fn(rho)
    K = p.K0
    J0 = S.initial_angular_momentum(p)
    out_o, st_o = S.scf_step(rho, phi, level, p, K, x_L1, J0)
    out_g, st_g = ctx.scf_step(level, _dev(rho), _dev(phi), K, x_L1, _params(p))
    out_g = out_g.cpu().numpy().reshape(rho.shape)
    e = float(np.abs(out_g - out_o).max() / out_o.max())
    say(f"step level={level} x_L1={x_L1} e_rho={e:.2e} c=({st_g['c1']},{st_g['c2']}) l1={st_g['l1']}")
    _cmp_state(st_g, st_o, 1e-12)
    assert e <= 1e-12


@pytest.mark.parametrize("level,x_L1", [(1, 0.0), (2, 0.0), (2, -3.0 / 64), (3, -3.0 / 128)])
def test_step_matches_oracle_step(ctx, level, x_L1):
    _step_case(ctx, level, x_L1, fft_poisson(level))


def test_step_full_size_128(ctx):
    # the benchmark's grid; inputs from the oracle side (normalised initial
    # model, FFT potential)
    _step_case(ctx, 4, 0.0, fft_poisson(4))


def test_step_256(ctx):
    # a 256^3 grid with an analytic potential (two softened point masses)
    level = 5
    n = 8 << level
    c = (np.arange(n) + 0.5) / n - 0.5
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")

    def phi_fn(rho):
        r1 = np.sqrt((X + 0.165) ** 2 + Y * Y + Z * Z + 1e-3)
        r2 = np.sqrt((X - 0.235) ** 2 + Y * Y + Z * Z + 1e-3)
        return -1.0 / r1 - 0.7 / r2

    _step_case(ctx, level, 0.0, phi_fn)


def _run_case(ctx, level, iters, R1=0.12, R2=0.1):
    p, rho0 = _model(level, R1=R1, R2=R2)
    say(f"run level={level} iterations={iters}")
    tree = ctx.uniform_tree(rho0)
    rho_g, phi_g, hist_g = ctx.scf_run(tree, _params(p), iters)
    tree.destroy()
    rho_o, phi_o, hist_o = S.run(rho0, level, p, iters, S.oracle_solver(level, theta=0.5))
    n = rho0.shape[0]
    rho_g = rho_g.cpu().numpy().reshape(n, n, n)
    phi_g = phi_g.cpu().numpy().reshape(n, n, n)
    for sg, so in zip(hist_g, hist_o):
        _cmp_state(sg, so, 1e-9)
    e_rho = float(np.abs(rho_g - rho_o).max() / rho_o.max())
    e_phi = float(np.abs(phi_g - phi_o).max() / np.abs(phi_o).max())
    say(f"  e_rho={e_rho:.2e} e_phi={e_phi:.2e}")
    assert len(hist_g) == iters
    assert e_rho <= 1e-9 and e_phi <= 1e-9


@pytest.mark.parametrize("level,iters", [(1, 3), (2, 6), (3, 2), (1, 0)])
def test_run_matches_oracle_run(ctx, level, iters):
    # on the 16^3 grid the stars take 2-3 cells per radius: larger stars
    _run_case(ctx, level, iters, *((0.15, 0.13) if level == 1 else (0.12, 0.1)))


def _mirrors(c, n):
    """The cell c and its mirror images in y and z (the grid's centre planes
    y = 0 and z = 0 are cell faces)."""
    ix, iy, iz = np.unravel_index(c, (n, n, n))
    return {int(np.ravel_multi_index((ix, jy, jz), (n, n, n))) for jy in (iy, n - 1 - iy) for jz in (iz, n - 1 - iz)}


def test_step_on_axis(ctx):
    """The paper's symmetric set-up, the stars' axis on the grid's centre
    line: with the same inputs on both sides, the mirror-image cells tie
    exactly and both take the smallest index; the step matches at 1e-12."""
    level = 2
    p = S.SCFParams(M1=1.0, M2=0.7, a0=0.4, f=0.9)
    rho0, p.K0 = w.scf_initial_binary(level, 1.0, 0.7, 0.4, 0.12, 0.10, yz=(0.0, 0.0))
    rho = S.normalise(rho0, level, p, 0.0)
    phi = fft_poisson(level)(rho)
    # symmetric inputs: the potential averaged over its mirror images
    phi = 0.25 * (phi + phi[:, ::-1, :] + phi[:, :, ::-1] + phi[:, ::-1, ::-1])
    out_o, st_o = S.scf_step(rho, phi, level, p, p.K0, 0.0, S.initial_angular_momentum(p))
    out_g, st_g = ctx.scf_step(level, _dev(rho), _dev(phi), p.K0, 0.0, _params(p))
    out_g = out_g.cpu().numpy().reshape(rho.shape)
    say(f"on-axis step c=({st_g['c1']},{st_g['c2']}) l1={st_g['l1']}")
    _cmp_state(st_g, st_o, 1e-12)
    assert float(np.abs(out_g - out_o).max() / out_o.max()) <= 1e-12


def test_run_on_axis_ties(ctx):
    """Runs with the stars' axis on the grid's centre line.  The densest
    cells come in mirror-image sets whose densities agree only up to the
    rounding of the two sides' potential solves, so each side may take a
    different cell of a set, and the result depends on the choice (the star
    lobes are balls about the centre cells).  Accepted: every centre and L1
    cell of the device is a mirror image of the oracle's, and the scalars,
    density and potential differ from the oracle's by at most 4x the spread
    between two oracle runs that break every near-tie (1e-12) differently
    (smallest index, largest index)."""
    level, iters = 2, 6
    p = S.SCFParams(M1=1.0, M2=0.7, a0=0.4, f=0.9)
    rho0, p.K0 = w.scf_initial_binary(level, 1.0, 0.7, 0.4, 0.12, 0.10, yz=(0.0, 0.0))
    n = rho0.shape[0]
    solve = S.oracle_solver(level, theta=0.5)
    rho_a, phi_a, hist_a = S.run(rho0, level, p, iters, solve)
    try:
        S.TIE_LAST, S.TIE_RTOL = True, 1e-12
        rho_b, phi_b, hist_b = S.run(rho0, level, p, iters, solve)
    finally:
        S.TIE_LAST, S.TIE_RTOL = False, 0.0
    tree = ctx.uniform_tree(rho0)
    rho_g, phi_g, hist_g = ctx.scf_run(tree, _params(p), iters)
    tree.destroy()
    rho_g = rho_g.cpu().numpy().reshape(n, n, n)
    phi_g = phi_g.cpu().numpy().reshape(n, n, n)
    spread = {k: max(abs(getattr(a, k) - getattr(b, k)) / abs(getattr(a, k)) for a, b in zip(hist_a, hist_b))
              for k in SCALARS}
    for sg, so in zip(hist_g, hist_a):
        for k in ("c1", "c2", "l1"):
            assert sg[k] in _mirrors(getattr(so, k), n), (k, sg[k], getattr(so, k))
        for k in SCALARS:
            assert abs(sg[k] - getattr(so, k)) <= 4 * spread[k] * abs(getattr(so, k)) + 1e-12 * abs(getattr(so, k))
    e_rho = float(np.abs(rho_g - rho_a).max() / rho_a.max())
    e_phi = float(np.abs(phi_g - phi_a).max() / np.abs(phi_a).max())
    s_rho = float(np.abs(rho_b - rho_a).max() / rho_a.max())
    s_phi = float(np.abs(phi_b - phi_a).max() / np.abs(phi_a).max())
    say(f"on-axis run: e_rho={e_rho:.2e} (spread {s_rho:.2e}) e_phi={e_phi:.2e} (spread {s_phi:.2e}); "
        f"cells {[(h['c1'], h['c2']) for h in hist_g]} vs {[(h.c1, h.c2) for h in hist_a]}")
    assert e_rho <= 4 * s_rho + 1e-9 and e_phi <= 4 * s_phi + 1e-9


def test_run_full_size_one_iteration(ctx):
    # the benchmark's 128^3 grid: one iteration and the final solve against
    # the oracle's (two oracle solves of 2M cells)
    _run_case(ctx, 4, 1)


@pytest.mark.parametrize("level,iters", [(4, 12), (5, 4)])
def test_run_full_size_properties(ctx, level, iters):
    import torch

    p, rho0 = _model(level)
    n = rho0.shape[0]
    say(f"run full size level={level} n={n} iterations={iters}")
    tree = ctx.uniform_tree(rho0)
    rho_g, phi_g, hist = ctx.scf_run(tree, _params(p), iters)
    # the tree now holds the returned density: the run's last potential is
    # the library's solve of it, bit for bit
    phi2, _, _ = ctx.solve(tree, theta=0.5)
    tree.destroy()
    assert torch.equal(phi_g, phi2)
    rho = rho_g.cpu().numpy().reshape(n, n, n)
    phi = phi_g.cpu().numpy().reshape(n, n, n)
    # the stars hold M1 + M2, every other cell the floor (the box has volume 1)
    total = rho.sum() / rho.size
    assert abs(total - (p.M1 + p.M2)) <= p.floor + 1e-12
    assert np.all(np.isfinite([h[k] for h in hist for k in SCALARS]))
    s = hist[-1]
    assert s["K"] > 0.0
    # near the fixed point each star is hydrostatic in the rotating frame
    c = (np.arange(n) + 0.5) / n - 0.5
    X, Y, _ = np.meshgrid(c, c, c, indexing="ij")
    m = rho / rho.size
    xc, yc = (m * X).sum() / m.sum(), (m * Y).sum() / m.sum()
    pe = phi - 0.5 * s["omega"] ** 2 * ((X - xc) ** 2 + (Y - yc) ** 2)
    lhs = s["K"] * (p.n + 1.0) * rho ** (1.0 / p.n) + pe
    dense = rho > 1e-2 * rho.max()
    worst = 0.0
    for C, side, ci in ((s["C1"], X < s["x_L1"], s["c1"]), (s["C2"], X >= s["x_L1"], s["c2"])):
        sel = dense & side
        assert sel.sum() > 50
        worst = max(worst, float(np.abs(lhs[sel] - C).max() / abs(C - pe.ravel()[ci])))
    say(f"  total={total:.15f} K={s['K']:.6f} omega={s['omega']:.6f} hydrostatic residual={worst:.2e}")
    assert worst <= 3e-2


def test_run_repeats_bit_for_bit(ctx):
    import torch

    p, rho0 = _model(3)
    out = []
    for _ in range(2):
        tree = ctx.uniform_tree(rho0)
        out.append(ctx.scf_run(tree, _params(p), 3))
        tree.destroy()
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]


def test_scf_errors(ctx):
    p, rho0 = _model(1)
    tree = ctx.uniform_tree(rho0)
    with pytest.raises(lib.OctoError) as e:
        ctx.scf_run(tree, _params(p, x_L1=0.01), 1)  # neither a cell centre nor a face
    assert e.value.status == lib.OCTO_E_INVALID
    with pytest.raises(lib.OctoError) as e:
        ctx.scf_run(tree, _params(p), -1)
    assert e.value.status == lib.OCTO_E_INVALID
    bad = _params(p)
    bad.M2 = 0.0
    with pytest.raises(lib.OctoError) as e:
        ctx.scf_run(tree, bad, 1)
    assert e.value.status == lib.OCTO_E_INVALID
    tree.destroy()
    # a tree on the leaf layout (not the uniform grid layout) is refused
    lt = ctx.tree(w.uniform_leaves(1), w.grid_to_leaves(rho0))
    with pytest.raises(lib.OctoError) as e:
        ctx.scf_run(lt, _params(p), 1)
    assert e.value.status == lib.OCTO_E_INVALID
    lt.destroy()
