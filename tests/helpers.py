"""Shared helpers for the tests: random trees and independent reference sums.

Nothing here implements the multipole method; the brute-force references are
written independently of the oracle (numpy, different algorithms)."""
from __future__ import annotations

import itertools
from math import comb

import numpy as np

import workloads as w


def random_amr_leaves(seed: int, max_level: int = 2, n_stars: int = 1):
    """A balanced adaptive leaf list refined around random compact stars."""
    import oracle

    rng = np.random.default_rng(seed)
    stars = []
    for _ in range(n_stars):
        c = tuple(rng.uniform(-0.3, 0.3, 3))
        stars.append(w.Star(c, float(rng.uniform(0.04, 0.12)), 1.0))
    f = w.Polytropes(stars=stars)
    return oracle.build_adaptive_leaves(f.boxmax, max_level, 1e-4), f


MONOMIALS = [(bx, by, bz) for bx in range(4) for by in range(4 - bx) for bz in range(4 - bx - by)]


def poly_sum_all(coef_by_pw: dict, x: np.ndarray, m: np.ndarray) -> np.ndarray:
    """S_i = sum_j m_j P(x_i - x_j) over ALL j (self included), for a polynomial
    P = sum c_b R^b, by the binomial expansion of (x_i - x_j)^b in moments of the
    sources: O(N) and independent of any tree."""
    # source moments S_k = sum_j m_j x_j^k for k up to degree 3 per axis
    mom = {}
    for k in itertools.product(range(4), repeat=3):
        if sum(k) <= 3:
            mom[k] = float((m * x[0] ** k[0] * x[1] ** k[1] * x[2] ** k[2]).sum())
    out = np.zeros(x.shape[1])
    for b, c in coef_by_pw.items():
        if c == 0.0:
            continue
        for k in itertools.product(*(range(bi + 1) for bi in b)):
            coeff = c
            for d in range(3):
                coeff *= comb(b[d], k[d]) * (-1) ** k[d]
            out += coeff * x[0] ** (b[0] - k[0]) * x[1] ** (b[1] - k[1]) * x[2] ** (b[2] - k[2]) * mom[k]
    return out


def poly_direct(coef: np.ndarray, x: np.ndarray, m: np.ndarray, G: float = 1.0):
    """phi_i = -G sum_{j != i} m_j K(x_i - x_j), g_i = G sum_{j != i} m_j grad K."""
    K = {pw: float(c) for pw, c in zip(MONOMIALS, coef)}
    k0 = K.get((0, 0, 0), 0.0)
    phi = -G * (poly_sum_all(K, x, m) - m * k0)
    g = np.zeros_like(x)
    for a in range(3):
        grad = {}
        for pw, c in K.items():
            if pw[a] > 0:
                q = list(pw)
                q[a] -= 1
                grad[tuple(q)] = grad.get(tuple(q), 0.0) + c * pw[a]
        g0 = grad.get((0, 0, 0), 0.0)
        g[a] = G * (poly_sum_all(grad, x, m) - m * g0)
    return phi, g


def rel_err_phi(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


def rel_err_g(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def grid_ids(level: int, sel: np.ndarray) -> np.ndarray:
    """Leaf-order ids of uniform-grid cells given as flat grid indices."""
    n = 8 << level
    G = np.arange(n ** 3).reshape(n, n, n)
    L = w.grid_to_leaves(G).ravel()
    inv = np.empty_like(L)
    inv[L] = np.arange(L.size)
    return inv[np.asarray(sel)]


def fft_poisson(level: int, G: float = 1.0):
    """phi_i = -G sum_{j != i} m_j / |x_i - x_j| over the cell centres of the
    uniform grid of `level`, by zero-padded FFT convolution."""
    n = 8 << level
    h = 1.0 / n
    m = 2 * n
    k = np.arange(m)
    k = np.where(k < n, k, k - m) * h
    X, Y, Z = np.meshgrid(k, k, k, indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z)
    g = np.zeros_like(r)
    g[r > 0] = 1.0 / r[r > 0]
    gh = np.fft.rfftn(g)

    def solve(rho):
        pad = np.zeros((m, m, m))
        pad[:n, :n, :n] = rho * h ** 3
        return -G * np.fft.irfftn(np.fft.rfftn(pad) * gh, s=(m, m, m), axes=(0, 1, 2))[:n, :n, :n]

    return solve


def zero_block_density(seed: int) -> np.ndarray:
    """A 32^3 uniform grid (levels 0-2) with massless regions (reading R11):
    the 4^3 leaf cells under three root cells (one at the domain corner, two
    inside), so each such root cell and its eight level-1 cells have no mass,
    and one 2^3 block under a massive root cell (a massless level-1 cell);
    uniform random density elsewhere."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.1, 1.0, (32, 32, 32))
    for a, b, c in ((0, 0, 0), (12, 16, 8), (16, 12, 20)):
        rho[a:a + 4, b:b + 4, c:c + 4] = 0.0
    rho[6:8, 6:8, 26:28] = 0.0
    return rho
