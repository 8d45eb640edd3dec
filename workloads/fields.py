"""Seeded synthetic density fields for the gravity solve.

This module holds only input generation: density values at points, the maximum
of a density over a box (used by the refinement criterion) and analytic
potentials for closed-form checks.  It contains none of the multipole method's
arithmetic and is shared by the HIP path, the CPU oracle, the tests and the
benchmark.

Coordinates are the unit box [-1/2, 1/2]^3 with G = 1 (paper Sec. 2.8, code
units).  All evaluations use only +, -, *, / and sqrt so that the same inputs
give bit-identical densities regardless of how the points are batched.

Workload shapes follow the paper's gravity tests:
  * uniform static sphere, radius 0.25, total mass 1, ambient 1e-10
    (Sec. 3.4, "Uniform Static Sphere");
  * n = 3/2 polytropes evaluated per cell from the Lane-Emden solution
    (Sec. 3.5, "Stationary Star", polytropic EoS p = K rho^(1+1/n) of Sec. 2.1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

FLOOR = 1e-10

# ----------------------------------------------------------------------------
# Lane-Emden solution theta(xi) for polytropic index n (fixed-step RK4).
# ----------------------------------------------------------------------------

_LE_CACHE = {}


def _pow_n(th: float, n: float) -> float:
    if th <= 0.0:
        return 0.0
    if n == 1.5:
        return th * math.sqrt(th)
    if n == 1.0:
        return th
    return th ** n


def lane_emden_table(n: float = 1.5, dxi: float = 2.0e-4):
    """Tabulate theta and dtheta/dxi of the Lane-Emden equation
    theta'' + (2/xi) theta' + theta^n = 0 up to its first zero xi_1.

    Returns (dxi, theta[], dtheta[], xi1, dtheta(xi1)).  The integration starts
    from the series theta = 1 - xi^2/6 + n xi^4/120 at a small xi and uses
    classic fourth-order Runge-Kutta with a fixed step.
    """
    key = (n, dxi)
    if key in _LE_CACHE:
        return _LE_CACHE[key]

    def rhs(xi, th, dth):
        return dth, -_pow_n(th, n) - 2.0 * dth / xi

    xi = dxi
    th = 1.0 - xi * xi / 6.0 + n * xi ** 4 / 120.0
    dth = -xi / 3.0 + n * xi ** 3 / 30.0
    ths = [1.0, th]
    dths = [0.0, dth]
    while True:
        k1a, k1b = rhs(xi, th, dth)
        k2a, k2b = rhs(xi + 0.5 * dxi, th + 0.5 * dxi * k1a, dth + 0.5 * dxi * k1b)
        k3a, k3b = rhs(xi + 0.5 * dxi, th + 0.5 * dxi * k2a, dth + 0.5 * dxi * k2b)
        k4a, k4b = rhs(xi + dxi, th + dxi * k3a, dth + dxi * k3b)
        th_new = th + dxi / 6.0 * (k1a + 2 * k2a + 2 * k3a + k4a)
        dth_new = dth + dxi / 6.0 * (k1b + 2 * k2b + 2 * k3b + k4b)
        if th_new <= 0.0:
            # linear root location between xi and xi + dxi
            frac = th / (th - th_new)
            xi1 = xi + frac * dxi
            dth1 = dth + frac * (dth_new - dth)
            break
        xi += dxi
        th, dth = th_new, dth_new
        ths.append(th)
        dths.append(dth)
    out = (dxi, np.asarray(ths), np.asarray(dths), xi1, dth1)
    _LE_CACHE[key] = out
    return out


def lane_emden_theta(xi: np.ndarray, n: float = 1.5) -> np.ndarray:
    """theta(xi) by cubic Hermite interpolation of the table; 0 beyond xi_1."""
    dxi, ths, dths, xi1, _ = lane_emden_table(n)
    xi = np.asarray(xi, dtype=np.float64)
    out = np.zeros_like(xi)
    inside = xi < xi1
    x = xi[inside]
    k = np.floor(x / dxi).astype(np.int64)
    k = np.minimum(k, len(ths) - 2)
    t = (x - k * dxi) / dxi
    t2 = t * t
    t3 = t2 * t
    h00 = 2.0 * t3 - 3.0 * t2 + 1.0
    h10 = t3 - 2.0 * t2 + t
    h01 = -2.0 * t3 + 3.0 * t2
    h11 = t3 - t2
    th = h00 * ths[k] + h10 * dxi * dths[k] + h01 * ths[k + 1] + h11 * dxi * dths[k + 1]
    out[inside] = np.maximum(th, 0.0)
    return out


# ----------------------------------------------------------------------------
# Fields
# ----------------------------------------------------------------------------


class Field:
    """A density defined at any point of the unit box."""

    floor: float = FLOOR

    def density(self, x: np.ndarray, y: np.ndarray, z: np.ndarray) -> np.ndarray:
        raise NotImplementedError

    def boxmax(self, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
        """Maximum of the density over each axis-aligned box (lo, hi: n x 3)."""
        raise NotImplementedError


@dataclass
class Star:
    centre: Tuple[float, float, float]
    radius: float
    rho_c: float
    n: float = 1.5

    def density(self, x, y, z):
        dx = x - self.centre[0]
        dy = y - self.centre[1]
        dz = z - self.centre[2]
        r = np.sqrt(dx * dx + dy * dy + dz * dz)
        _, _, _, xi1, _ = lane_emden_table(self.n)
        th = lane_emden_theta(xi1 * r / self.radius, self.n)
        if self.n == 1.5:
            return self.rho_c * (th * np.sqrt(th))
        return self.rho_c * th ** self.n

    def mass(self) -> float:
        """M = 4 pi R^3 rho_c (-theta'(xi1)/xi1)."""
        _, _, _, xi1, dth1 = lane_emden_table(self.n)
        return 4.0 * math.pi * self.radius ** 3 * self.rho_c * (-dth1 / xi1)


@dataclass
class Polytropes(Field):
    """Sum of non-overlapping polytropic stars plus a density floor."""

    stars: List[Star] = field(default_factory=list)
    floor: float = FLOOR

    def density(self, x, y, z):
        x = np.asarray(x, dtype=np.float64)
        rho = np.zeros(np.broadcast(x, y, z).shape)
        for s in self.stars:
            rho = rho + s.density(x, y, z)
        return np.maximum(rho, self.floor)

    def boxmax(self, lo, hi):
        lo = np.asarray(lo, dtype=np.float64).reshape(-1, 3)
        hi = np.asarray(hi, dtype=np.float64).reshape(-1, 3)
        best = np.full(lo.shape[0], self.floor)
        for s in self.stars:
            c = np.asarray(s.centre)
            p = np.minimum(np.maximum(c[None, :], lo), hi)  # closest point of the box
            best = np.maximum(best, self.density(p[:, 0], p[:, 1], p[:, 2]))
        return best


@dataclass
class UniformSphere(Field):
    """Static sphere of radius a and total mass M centred at the origin
    (Sec. 3.4: a = 0.25, M = 1, ambient density 1e-10)."""

    radius: float = 0.25
    total_mass: float = 1.0
    floor: float = FLOOR

    @property
    def rho_in(self) -> float:
        return self.total_mass / (4.0 / 3.0 * math.pi * self.radius ** 3)

    def density(self, x, y, z):
        r2 = x * x + y * y + z * z
        return np.where(r2 < self.radius * self.radius, self.rho_in, self.floor)

    def boxmax(self, lo, hi):
        lo = np.asarray(lo, dtype=np.float64).reshape(-1, 3)
        hi = np.asarray(hi, dtype=np.float64).reshape(-1, 3)
        p = np.minimum(np.maximum(0.0, lo), hi)
        return self.density(p[:, 0], p[:, 1], p[:, 2])

    def potential(self, x, y, z):
        """Closed form: -M(3a^2 - r^2)/(2a^3) inside, -M/r outside (G = 1)."""
        r = np.sqrt(x * x + y * y + z * z)
        a, m = self.radius, self.total_mass
        return np.where(r < a, -m * (3 * a * a - r * r) / (2 * a ** 3), -m / np.maximum(r, 1e-300))


@dataclass
class OrbitalRate(Field):
    """Density rate (a second, signed source) of a field whose pattern turns
    rigidly about the z axis at angular speed omega, as a binary does on a grid
    that does not co-rotate: the central difference of the base density over
    rotations by -omega*dt and +omega*dt, divided by 2*dt.  (The rotation's
    cosine and sine are computed once, so points are evaluated with the same
    operations as densities.)"""

    base: Field = None
    omega: float = 1.0
    dt: float = 1.0e-3

    def density(self, x, y, z):
        c, s = math.cos(self.omega * self.dt), math.sin(self.omega * self.dt)
        # the pattern at time t is the base density at R(-omega t) x
        later = self.base.density(c * x + s * y, c * y - s * x, z)  # R(-omega dt) x
        earlier = self.base.density(c * x - s * y, c * y + s * x, z)  # R(+omega dt) x
        return (later - earlier) / (2.0 * self.dt)


def noisy_rate(rho: np.ndarray, seed: int) -> np.ndarray:
    """A signed rate with no structure: rho * N(0, 1) per cell (seeded, in
    array order)."""
    rho = np.asarray(rho, dtype=np.float64)
    return rho * np.random.default_rng(seed).standard_normal(rho.shape)


def scf_initial_binary(level: int, M1: float, M2: float, a0: float, R1: float, R2: float, n: float = 1.5,
                       G: float = 1.0, yz=(0.0, 0.0)):
    """Starting model of a binary self-consistent-field iteration: two
    n-polytropes of masses M1 (at x < 0) and M2 with radii R1, R2, centres a0
    apart on the line y, z = `yz` parallel to x, with their centre of mass at
    x = 0, on the uniform grid of `level`; also returns the polytropic
    constant of the first star, K = 4 pi G R1^2 rho_c1^(1-1/n) / ((n+1) xi1^2),
    as the iteration's starting K.  A `yz` off the cell faces makes each
    star's densest cell unique (on the axis the cells around it tie)."""
    _, _, _, xi1, dth1 = lane_emden_table(n)
    x1, x2 = -a0 * M2 / (M1 + M2), a0 * M1 / (M1 + M2)
    rc1 = M1 / (4.0 * math.pi * R1 ** 3 * (-dth1 / xi1))
    rc2 = M2 / (4.0 * math.pi * R2 ** 3 * (-dth1 / xi1))
    f = Polytropes(stars=[Star((x1, yz[0], yz[1]), R1, rc1, n), Star((x2, yz[0], yz[1]), R2, rc2, n)])
    K0 = 4.0 * math.pi * G * R1 * R1 * rc1 ** (1.0 - 1.0 / n) / ((n + 1.0) * xi1 * xi1)
    return uniform_grid(f, level), K0


def binary_polytrope_128() -> Polytropes:
    """Binary n = 3/2 polytropes: radii 0.12 and 0.10, centres 0.35 apart on x
    with the centre of mass at the origin, mass ratio M2/M1 = 0.7, maximum
    density normalised to 1, floor 1e-10."""
    return binary_polytrope(r1=0.12, r2=0.10, sep=0.35, q=0.7)


def binary_polytrope(r1: float, r2: float, sep: float, q: float, n: float = 1.5) -> Polytropes:
    x1 = -sep * q / (1.0 + q)
    x2 = sep / (1.0 + q)
    # equal structure: M ~ rho_c R^3, so rho_c2/rho_c1 = q (R1/R2)^3
    ratio = q * (r1 / r2) ** 3
    rc1, rc2 = (1.0, ratio) if ratio <= 1.0 else (1.0 / ratio, 1.0)
    return Polytropes(stars=[Star((x1, 0.0, 0.0), r1, rc1, n), Star((x2, 0.0, 0.0), r2, rc2, n)])


def single_polytrope(radius: float, centre=(0.0, 0.0, 0.0), n: float = 1.5) -> Polytropes:
    return Polytropes(stars=[Star(tuple(centre), radius, 1.0, n)])


# ----------------------------------------------------------------------------
# Grids
# ----------------------------------------------------------------------------


def cell_centres(level: int) -> np.ndarray:
    """Centres of the n = 8 * 2^level cells per axis: -1/2 + (i + 1/2) h (exact)."""
    n = 8 << level
    h = 1.0 / n
    return (np.arange(n, dtype=np.float64) + 0.5) * h - 0.5


def uniform_grid(f: Field, level: int) -> np.ndarray:
    """Density at the cell centres of a uniform (8*2^level)^3 grid, shape
    (n, n, n) indexed [ix, iy, iz] (iz fastest in memory)."""
    c = cell_centres(level)
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    return np.ascontiguousarray(f.density(X, Y, Z), dtype=np.float64)


def noisy_sphere_16(seed: int = 210108226) -> np.ndarray:
    """16^3 grid: 1.0 * (1 + 0.01 N(0,1)) where |x|^2 < 0.16, 1e-10 elsewhere.
    Noise drawn in index order i*n^2 + j*n + k (i along x)."""
    n = 16
    c = cell_centres(1)
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    noise = np.random.default_rng(seed).standard_normal(n ** 3).reshape(n, n, n)
    inside = (X * X + Y * Y + Z * Z) < 0.16
    rho = np.where(inside, 1.0 * (1.0 + 0.01 * noise), FLOOR)
    return np.ascontiguousarray(rho)


def leaf_density(f: Field, leaves: np.ndarray) -> np.ndarray:
    """Density at the 512 cell centres of each leaf sub-grid.

    leaves: int array (n, 4) of (level, nx, ny, nz).  Returns (n, 512) with the
    cells of each sub-grid in (ix, iy, iz) order, iz fastest."""
    leaves = np.asarray(leaves, dtype=np.int64).reshape(-1, 4)
    out = np.empty((leaves.shape[0], 512), dtype=np.float64)
    loc = np.arange(8, dtype=np.float64)
    for lev in np.unique(leaves[:, 0]):
        sel = np.nonzero(leaves[:, 0] == lev)[0]
        h = 1.0 / (8 << int(lev))
        base = leaves[sel, 1:4].astype(np.float64) * 8.0  # first cell index
        gx = (base[:, 0:1] + loc[None, :] + 0.5) * h - 0.5
        gy = (base[:, 1:2] + loc[None, :] + 0.5) * h - 0.5
        gz = (base[:, 2:3] + loc[None, :] + 0.5) * h - 0.5
        X = np.broadcast_to(gx[:, :, None, None], (len(sel), 8, 8, 8))
        Y = np.broadcast_to(gy[:, None, :, None], (len(sel), 8, 8, 8))
        Z = np.broadcast_to(gz[:, None, None, :], (len(sel), 8, 8, 8))
        out[sel] = f.density(X, Y, Z).reshape(len(sel), 512)
    return out


def uniform_leaves(level: int) -> np.ndarray:
    """Leaf list of a uniform tree: all sub-grids at `level`, nz fastest."""
    m = 1 << level
    idx = np.arange(m)
    NX, NY, NZ = np.meshgrid(idx, idx, idx, indexing="ij")
    out = np.stack([np.full(m ** 3, level), NX.ravel(), NY.ravel(), NZ.ravel()], axis=1)
    return out.astype(np.int32)


def grid_to_leaves(rho: np.ndarray) -> np.ndarray:
    """Reorder a uniform (n, n, n) grid into the per-sub-grid layout of
    uniform_leaves(level): (n_leaves, 512)."""
    n = rho.shape[0]
    m = n // 8
    r = rho.reshape(m, 8, m, 8, m, 8).transpose(0, 2, 4, 1, 3, 5)
    return np.ascontiguousarray(r.reshape(m ** 3, 512))


def leaves_to_grid(vals: np.ndarray, level: int) -> np.ndarray:
    """Inverse of grid_to_leaves."""
    m = 1 << level
    v = np.asarray(vals).reshape(m, m, m, 8, 8, 8).transpose(0, 3, 1, 4, 2, 5)
    return np.ascontiguousarray(v.reshape(8 * m, 8 * m, 8 * m))
