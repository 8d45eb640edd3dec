"""TEST INFRASTRUCTURE ONLY: the self-consistent-field (SCF) iteration for a
synchronously rotating binary of two polytropes, written from the paper's
description of its initial model (Sec. 4.1, "The Initial Stellar Model"), on a
uniform grid, with the oracle's own multipole solve for the potential.

Readings where the printed text is garbled or silent (also listed in the
design notes):

* the effective potential is phi_eff = phi - Omega^2 ((x - x_c)^2 + (y - y_c)^2) / 2
  about the rotation axis through the centre of mass (x_c, y_c); the grid is not
  advected (step 2), the axis follows the centre of mass instead;
* step 5: K = (C2 - phi_C) / ((n + 1) rho_2^(1/n)), the hydrostatic relation
  K (1 + n) rho^(1/n) + phi_eff = C at the donor's centre;
* step 6: rho = ((C - phi_eff) / (K (n + 1)))^n where C - phi_eff > 0, the sign
  the hydrostatic relation fixes;
* step 7 solves for the density after the mass normalisation of step 1 (the
  normalisation is applied before each solve), so that the potential used in
  steps 2-6 is the one of the density they use; taken literally (solve, then
  rescale the masses) the iteration diverges;
* the stars: the accretor (mass M1) lies at x < x_L1, the donor (M2) at x > x_L1;
  a star's cells are those on its side of x_L1 within distance |x_L1 - x_i| of
  its centre cell (the densest cell of that side); every other cell holds the
  floor density;
* L1 is the cell of largest phi_eff on the grid row (iy, iz of the accretor's
  centre) strictly between the two centre cells; ties of any maximum go to the
  smallest flat index;
* a star's centre for the separation a is its centre of mass; Omega follows
  step 3 with J0 = M1 M2 / (M1 + M2) a0^2 Omega_K(a0), Omega_K^2 = G (M1 + M2) / a0^3;
* C1 uses the K of the previous iteration (step 4 precedes step 5), starting
  from K0 given with the initial model.

Every step runs in FP64 in the order of the paper's list; the functions are
plain numpy over a (n, n, n) grid indexed [ix, iy, iz].
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np


@dataclass
class SCFParams:
    M1: float              # accretor mass
    M2: float              # donor mass
    n: float = 1.5         # polytropic index
    a0: float = 0.35       # initial separation (fixes J0)
    f: float = 0.9         # Roche filling factor of the donor
    K0: float = 0.1        # polytropic constant before the first update
    floor: float = 1e-10   # density outside the stars
    G: float = 1.0
    theta: float = 0.5     # opening angle of the potential solve


@dataclass
class SCFState:
    omega: float
    K: float
    C1: float
    C2: float
    x_L1: float
    a: float
    mass1: float
    mass2: float
    c1: int                # flat index of the accretor's centre cell
    c2: int
    l1: int


def _centres(level: int):
    n = 8 << level
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h - 0.5
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    return X, Y, Z, h


# Tie rule of every maximum: the smallest flat index among the cells holding
# the largest value.  Tests may switch it to the largest index among the cells
# within TIE_RTOL of the largest value, to measure how much a result depends
# on which of several cells that tie up to rounding is taken.
TIE_LAST = False
TIE_RTOL = 0.0


def _argmax(values: np.ndarray, mask: np.ndarray) -> int:
    """Flat index of the largest value where mask holds; ties to the smallest index."""
    v = np.where(mask, values, -np.inf).ravel()
    if TIE_LAST:
        return int(np.flatnonzero(v >= v.max() - TIE_RTOL * abs(v.max()))[-1])
    return int(np.flatnonzero(v == v.max())[0])


def _stars(rho: np.ndarray, X, Y, Z, x_L1: float):
    """Centre cells (the densest cell of each side of x_L1) and the cells of
    each star (its side, within |x_L1 - x_centre| of its centre cell)."""
    side1 = X < x_L1
    c1 = _argmax(rho, side1)
    c2 = _argmax(rho, ~side1)
    cen = []
    for c in (c1, c2):
        cen.append((X.ravel()[c], Y.ravel()[c], Z.ravel()[c]))
    r1 = np.sqrt((X - cen[0][0]) ** 2 + (Y - cen[0][1]) ** 2 + (Z - cen[0][2]) ** 2)
    r2 = np.sqrt((X - cen[1][0]) ** 2 + (Y - cen[1][1]) ** 2 + (Z - cen[1][2]) ** 2)
    star1 = side1 & (r1 < abs(x_L1 - cen[0][0]))
    star2 = ~side1 & (r2 < abs(x_L1 - cen[1][0]))
    return c1, c2, star1, star2, r1, r2


def normalise(rho: np.ndarray, level: int, p: SCFParams, x_L1: float):
    """Step 1: each star's density times the factor that gives it its mass."""
    X, Y, Z, h = _centres(level)
    _, _, star1, star2, _, _ = _stars(rho, X, Y, Z, x_L1)
    m1 = float(np.sum(rho[star1]) * h ** 3)
    m2 = float(np.sum(rho[star2]) * h ** 3)
    return np.where(star1, rho * (p.M1 / m1), np.where(star2, rho * (p.M2 / m2), rho))


def scf_step(rho: np.ndarray, phi: np.ndarray, level: int, p: SCFParams, K: float, x_L1: float,
             J0: float) -> (np.ndarray, SCFState):
    """Steps 2-6 of Sec. 4.1 from a density `rho` already normalised (step 1)
    and its potential `phi`; returns the new density and the iteration's
    scalars.  `x_L1` is the L1 position of the previous iteration (it splits
    the grid into the two stars' sides)."""
    X, Y, Z, h = _centres(level)
    vol = h ** 3
    c1, c2, star1, star2, r1, r2 = _stars(rho, X, Y, Z, x_L1)
    xc1, xc2 = X.ravel()[c1], X.ravel()[c2]
    mass = rho * vol
    # (2) centre of mass of the grid: the rotation axis
    M = float(mass.sum())
    xc, yc = float((mass * X).sum() / M), float((mass * Y).sum() / M)
    # (3) separation of the stars' centres of mass, Omega from J0
    cm = []
    for st_ in (star1, star2):
        ms = mass[st_]
        cm.append(np.array([(ms * X[st_]).sum(), (ms * Y[st_]).sum(), (ms * Z[st_]).sum()]) / ms.sum())
    a = float(np.linalg.norm(cm[1] - cm[0]))
    omega = J0 * (p.M1 + p.M2) / (p.M1 * p.M2 * a * a)
    # (4) integration constants
    phi_eff = phi - 0.5 * omega * omega * ((X - xc) ** 2 + (Y - yc) ** 2)
    pe = phi_eff.ravel()
    ix1, iy1, iz1 = np.unravel_index(c1, rho.shape)
    ix2 = np.unravel_index(c2, rho.shape)[0]
    row = np.zeros(rho.shape, dtype=bool)
    lo, hi = min(ix1, ix2), max(ix1, ix2)
    row[lo + 1:hi, iy1, iz1] = True
    l1 = _argmax(phi_eff, row)
    x_new = float(X.ravel()[l1])
    rho1 = float(rho.ravel()[c1])
    rho2 = float(rho.ravel()[c2])
    C1 = K * (1.0 + p.n) * rho1 ** (1.0 / p.n) + pe[c1]
    phi_C = pe[c2]
    C2 = (1.0 - p.f) * phi_C + p.f * pe[l1]
    # (5) new K from the donor's centre
    K_new = (C2 - phi_C) / ((p.n + 1.0) * rho2 ** (1.0 / p.n))
    # (6) new density in each star's lobe about the new L1
    side1 = X < x_new
    lobe1 = side1 & (r1 < abs(x_new - xc1))
    lobe2 = ~side1 & (r2 < abs(x_new - xc2))
    H = np.where(lobe1, C1 - phi_eff, np.where(lobe2, C2 - phi_eff, -1.0))
    out = np.where(H > 0.0, (np.maximum(H, 0.0) / (K_new * (p.n + 1.0))) ** p.n, 0.0)
    out = np.maximum(out, p.floor)
    m1 = float(np.sum(rho[star1]) * vol)
    m2 = float(np.sum(rho[star2]) * vol)
    st = SCFState(omega, K_new, float(C1), float(C2), x_new, a, m1, m2, c1, c2, l1)
    return out, st


def initial_angular_momentum(p: SCFParams) -> float:
    mu = p.M1 * p.M2 / (p.M1 + p.M2)
    return mu * p.a0 * p.a0 * np.sqrt(p.G * (p.M1 + p.M2) / p.a0 ** 3)


def run(rho0: np.ndarray, level: int, p: SCFParams, iterations: int, solve, x_L1: Optional[float] = None):
    """Iterate the SCF from `rho0` (grid [ix, iy, iz]); `solve(rho) -> phi`
    (same layout) is the potential solve of step 7 (and of the set-up).
    Returns (rho, phi, [SCFState per iteration])."""
    J0 = initial_angular_momentum(p)
    rho = np.array(rho0, dtype=np.float64)
    K = p.K0
    x = 0.0 if x_L1 is None else x_L1
    hist: List[SCFState] = []
    for _ in range(iterations):
        rho = normalise(rho, level, p, x)  # (1), then the solve of (7) on it
        phi = solve(rho)
        rho, st = scf_step(rho, phi, level, p, K, x, J0)
        K, x = st.K, st.x_L1
        hist.append(st)
    rho = normalise(rho, level, p, x)
    return rho, solve(rho), hist


def oracle_solver(level: int, theta: float = 0.5, G: float = 1.0):
    """The oracle's multipole solve on the uniform tree of `level` as a
    grid -> grid function."""
    import oracle
    import workloads as w

    leaves = w.uniform_leaves(level)

    def solve(rho):
        t = oracle.Tree(leaves, w.grid_to_leaves(rho))
        phi, _ = t.solve(theta=theta, G=G)
        return w.leaves_to_grid(phi, level)

    return solve
