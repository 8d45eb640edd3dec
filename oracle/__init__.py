"""TEST INFRASTRUCTURE ONLY: the plain FP64 CPU oracle for the gravity solve.

Only `tests/`, `__graft_entry__.smoke()` and the benchmark's CPU-baseline leg
may import this package.  It shares no code with the HIP library
(`paper_2101_08226_amd`); the two meet only through the seeded inputs of
`workloads`.

The C part (`octo_oracle.c`) is built with plain `gcc -O2 -fopenmp` by
`oracle.build.build()`; this module wraps it with ctypes.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from .build import LIB_PATH, build  # noqa: F401
from .adaptive import build_adaptive_leaves, is_balanced  # noqa: F401
from . import coupling  # noqa: F401

_lib = None

_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_tree_new.restype = _P
        L.orc_tree_new.argtypes = [ctypes.c_int, _I32, _D]
        L.orc_tree_free.argtypes = [_P]
        L.orc_tree_error.restype = ctypes.c_char_p
        L.orc_tree_error.argtypes = [_P]
        L.orc_tree_nlev.argtypes = [_P]
        L.orc_tree_nnodes.argtypes = [_P]
        L.orc_last_counts.argtypes = [_P, _I64]
        L.orc_solve.restype = ctypes.c_int
        L.orc_solve.argtypes = [_P, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, _D, _I64,
                                ctypes.c_int64, ctypes.c_int, _D, _D]
        L.orc_solve_source.restype = ctypes.c_int
        L.orc_solve_source.argtypes = [_P, ctypes.c_double, ctypes.c_double, ctypes.c_int, _D, _D, _I64,
                                       ctypes.c_int64, ctypes.c_int, _D]
        L.orc_tree_set_centres.restype = ctypes.c_int
        L.orc_tree_set_centres.argtypes = [_P, ctypes.c_int]
        L.orc_cell_moments.restype = ctypes.c_int
        L.orc_cell_moments.argtypes = [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _D]
        L.orc_leaf_cells.argtypes = [_P, _D, _D]
        L.orc_dtensors.argtypes = [_D, ctypes.c_int, _D, _D]
        L.orc_m2l_pair.argtypes = [_D, _D, ctypes.c_double, ctypes.c_int, ctypes.c_int, _D, _D]
        L.orc_direct.argtypes = [ctypes.c_int64, _D, _D, ctypes.c_double, ctypes.c_int, _D, ctypes.c_int64,
                                 ctypes.c_int64, ctypes.c_int, _D, _D]
        L.orc_direct_points.argtypes = [ctypes.c_int64, _D, _D, ctypes.c_int64, _D, ctypes.c_double, ctypes.c_int,
                                        _D, ctypes.c_int, _D, _D]
        _lib = L
    return _lib


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.cast(None, _D)
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _kernel(coef):
    if coef is None:
        return 0, None
    c = np.ascontiguousarray(coef, dtype=np.float64)
    assert c.shape == (20,)
    return 1, c


# the 20 monomials of degree <= 3 in the oracle's order
MONOMIALS = [(bx, by, bz) for bx in range(4) for by in range(4 - bx) for bz in range(4 - bx - by)]


class Tree:
    """Oracle octree built from a leaf list (level, nx, ny, nz) and the density
    of each leaf's 512 cells ((ix, iy, iz) order, iz fastest)."""

    def __init__(self, leaves, rho):
        self.leaves = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32).reshape(-1, 4))
        self.rho = np.ascontiguousarray(np.asarray(rho, dtype=np.float64).reshape(-1, 512))
        assert self.rho.shape[0] == self.leaves.shape[0]
        L = lib()
        self._h = L.orc_tree_new(self.leaves.shape[0], self.leaves.ctypes.data_as(_I32), _dp(self.rho))
        err = L.orc_tree_error(self._h).decode()
        if err:
            L.orc_tree_free(self._h)
            self._h = None
            raise ValueError(err)
        self.n_cells = self.leaves.shape[0] * 512

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_tree_free(self._h)
            self._h = None

    @property
    def n_levels(self) -> int:
        return lib().orc_tree_nlev(self._h)

    CENTRES = {"mass": 0, "geometric": 1, "geometric-no-dipole": 2}

    def set_centres(self, mode: str) -> None:
        """Expansion centres of interior cells for later solves: "mass"
        (centre of mass, the default reading of Sec. 2.2), "geometric" (the
        geometric centre, dipole carried) or "geometric-no-dipole" (geometric
        centre, dipole dropped).  The last two serve the study of the
        static-sphere residuals (Sec. 3.4) only."""
        if lib().orc_tree_set_centres(self._h, self.CENTRES[mode]) != 0:
            raise ValueError(mode)

    def solve(self, theta=0.5, G=1.0, amc=True, kernel=None, sample=None, threads=0):
        """phi (n,) and g (3, n) at every leaf cell, or at the sampled leaf-cell
        ids (leaf index * 512 + local cell index)."""
        mode, coef = _kernel(kernel)
        if sample is None:
            n = self.n_cells
            sp, ns = ctypes.cast(None, _I64), 0
        else:
            sample = np.ascontiguousarray(sample, dtype=np.int64)
            n = sample.shape[0]
            sp, ns = sample.ctypes.data_as(_I64), n
        phi = np.empty(n)
        g = np.empty((3, n))
        rc = lib().orc_solve(self._h, float(theta), float(G), int(bool(amc)), mode, _dp(coef), sp, ns, int(threads),
                             _dp(phi), _dp(g))
        if rc != 0:
            raise RuntimeError(f"orc_solve failed ({rc})")
        return phi, g

    def solve_source(self, src, theta=0.5, G=1.0, kernel=None, sample=None, threads=0):
        """Potential of a second, signed source `src` (same layout as the
        density, e.g. a density rate) expanded about the density's centres of
        mass with the density's interaction lists; returns it at every leaf
        cell or at the sampled ids.  No correction (it acts on forces)."""
        mode, coef = _kernel(kernel)
        src = np.ascontiguousarray(np.asarray(src, dtype=np.float64).reshape(-1, 512))
        assert src.shape == self.rho.shape
        if sample is None:
            n = self.n_cells
            sp, ns = ctypes.cast(None, _I64), 0
        else:
            sample = np.ascontiguousarray(sample, dtype=np.int64)
            n = sample.shape[0]
            sp, ns = sample.ctypes.data_as(_I64), n
        phi = np.empty(n)
        rc = lib().orc_solve_source(self._h, float(theta), float(G), mode, _dp(coef), _dp(src), sp, ns, int(threads),
                                    _dp(phi))
        if rc != 0:
            raise RuntimeError(f"orc_solve_source failed ({rc})")
        return phi

    def last_counts(self, split=False):
        """(multipole pairs, direct pairs) of the last solve, ordered pairs;
        with split=True also the multipole pairs between two leaf cells."""
        out = np.zeros(3, dtype=np.int64)
        lib().orc_last_counts(self._h, out.ctypes.data_as(_I64))
        return (int(out[0]), int(out[1]), int(out[2])) if split else (int(out[0]), int(out[1]))

    def cell_moments(self, level, gx, gy, gz):
        out = np.empty(43)
        if lib().orc_cell_moments(self._h, level, gx, gy, gz, _dp(out)) != 0:
            raise KeyError((level, gx, gy, gz))
        return dict(m=out[0], z=out[1:4].copy(), M1=out[40:43].copy(), M2=out[4:13].reshape(3, 3).copy(),
                    M3=out[13:40].reshape(3, 3, 3).copy())

    def leaf_cells(self):
        """Centres x (3, n) and masses m (n) of the leaf cells in leaf order."""
        x = np.empty((3, self.n_cells))
        m = np.empty(self.n_cells)
        lib().orc_leaf_cells(self._h, _dp(x), _dp(m))
        return x, m


def dtensors(R, kernel=None):
    mode, coef = _kernel(kernel)
    R = np.ascontiguousarray(R, dtype=np.float64)
    out = np.empty(121)
    lib().orc_dtensors(_dp(R), mode, _dp(coef), _dp(out))
    return (out[0], out[1:4], out[4:13].reshape(3, 3), out[13:40].reshape(3, 3, 3), out[40:121].reshape(3, 3, 3, 3))


def m2l_pair(a, b, G=1.0, amc=True, kernel=None):
    """Locals (L0, L1, L2, L3) and correction C of cell a from cell b; a and b
    are dicts with m, z, M2 (3x3), M3 (3x3x3)."""
    mode, coef = _kernel(kernel)

    def pack(c):
        return np.ascontiguousarray(np.concatenate([[c["m"]], np.ravel(c["z"]), np.ravel(c["M2"]), np.ravel(c["M3"])]),
                                    dtype=np.float64)

    pa, pb = pack(a), pack(b)
    out = np.empty(43)
    lib().orc_m2l_pair(_dp(pa), _dp(pb), float(G), int(bool(amc)), mode, _dp(coef), _dp(out))
    return dict(L0=out[0], L1=out[1:4].copy(), L2=out[4:13].reshape(3, 3).copy(),
                L3=out[13:40].reshape(3, 3, 3).copy(), C=out[40:43].copy())


def direct(x, m, G=1.0, kernel=None, i0=0, i1=None, threads=0):
    """Compensated direct sum over all j != i for targets i in [i0, i1).
    x: (3, n), m: (n,).  Returns phi (k,), g (3, k)."""
    mode, coef = _kernel(kernel)
    x = np.ascontiguousarray(x, dtype=np.float64)
    m = np.ascontiguousarray(m, dtype=np.float64)
    n = m.shape[0]
    i1 = n if i1 is None else i1
    k = i1 - i0
    phi = np.empty(k)
    g = np.empty((3, k))
    lib().orc_direct(n, _dp(x), _dp(m), float(G), mode, _dp(coef), i0, i1, int(threads), _dp(phi), _dp(g))
    return phi, g


def direct_points(x, m, xt, G=1.0, kernel=None, threads=0):
    """Compensated direct sum at target points xt (3, k) from all sources;
    a source exactly at a target is skipped."""
    mode, coef = _kernel(kernel)
    x = np.ascontiguousarray(x, dtype=np.float64)
    m = np.ascontiguousarray(m, dtype=np.float64)
    xt = np.ascontiguousarray(xt, dtype=np.float64)
    k = xt.shape[1]
    phi = np.empty(k)
    g = np.empty((3, k))
    lib().orc_direct_points(m.shape[0], _dp(x), _dp(m), k, _dp(xt), float(G), mode, _dp(coef), int(threads),
                            _dp(phi), _dp(g))
    return phi, g


def stats(x, m, g):
    """Net force F = sum m g, net torque T = sum x cross m g (about the origin)
    and their scales sum m|g|, sum |x| m |g|."""
    f = m[None, :] * g
    F = f.sum(axis=1)
    T = np.cross(x.T, f.T).sum(axis=0)
    gn = np.sqrt((g * g).sum(axis=0))
    xn = np.sqrt((x * x).sum(axis=0))
    SF = (m * gn).sum()
    ST = (xn * m * gn).sum()
    return dict(F=F, T=T, SF=SF, ST=ST, force=np.linalg.norm(F) / SF, torque=np.linalg.norm(T) / ST)
