"""Python binding of liboctofmm: an MI355X (gfx950) HIP implementation of the
gravity solve of Octo-Tiger (Marcello et al., arXiv 2101.08226, Sec. 2.2).

The functions named `octo_*` mirror the C interface in include/octo.h one to
one (ctypes marshalling only).  The small classes below (`Context`, `Tree`)
route device memory through PyTorch's caching allocator, use a PyTorch stream
and return results as PyTorch tensors; every step of the solve runs in the HIP
library.  Importing works without a GPU; any call that needs the library
raises if it has not been built or no GPU is present.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboctofmm.so")

# status codes (include/octo.h)
OCTO_OK, OCTO_E_INVALID, OCTO_E_DEVICE, OCTO_E_BUDGET, OCTO_E_UNSUPPORTED, OCTO_E_STATE, OCTO_E_PENDING = range(7)
OCTO_FP64, OCTO_MIXED = 0, 1
STATUS_NAMES = {0: "OCTO_OK", 1: "OCTO_E_INVALID", 2: "OCTO_E_DEVICE", 3: "OCTO_E_BUDGET",
                4: "OCTO_E_UNSUPPORTED", 5: "OCTO_E_STATE", 6: "OCTO_E_PENDING"}

# every symbol include/octo.h declares
EXPORTS = [
    "octo_ctx_create", "octo_ctx_destroy", "octo_ctx_memory", "octo_ctx_set_profiling", "octo_ctx_set_batch_shapes", "octo_tree_build", "octo_tree_build_device", "octo_tree_build_uniform",
    "octo_tree_build_adaptive", "octo_tree_set_density", "octo_tree_get_density", "octo_tree_info", "octo_tree_leaves", "octo_tree_level_tables", "octo_tree_destroy",
    "octo_solve", "octo_solve_device_stats", "octo_tree_autotune", "octo_solve_batch", "octo_solve_dphidt", "octo_gravity_sources", "octo_energy_update", "octo_scf_step", "octo_scf_step_noalloc", "octo_scf_run", "octo_regrid", "octo_submit", "octo_poll", "octo_wait", "octo_last_error", "octo_build_id",
    "octo_host_stencil_sizes", "octo_host_near_lists", "octo_host_near_stage", "octo_host_layout", "octo_host_level_tables", "octo_host_adaptive_leaves",
]


class OctoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class octo_leaf(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("ix", ctypes.c_int32), ("iy", ctypes.c_int32), ("iz", ctypes.c_int32)]


class octo_level_tables(ctypes.Structure):
    _fields_ = [("nbr", ctypes.c_void_p), ("child", ctypes.c_void_p), ("parent", ctypes.c_void_p),
                ("coord", ctypes.c_void_p), ("out_base", ctypes.c_void_p), ("flags", ctypes.c_void_p),
                ("int_child", ctypes.c_void_p)]


class octo_opts(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("G", ctypes.c_double), ("precision", ctypes.c_int32),
                ("amc", ctypes.c_int32)]


class octo_scf_params(ctypes.Structure):
    _fields_ = [("M1", ctypes.c_double), ("M2", ctypes.c_double), ("n", ctypes.c_double), ("a0", ctypes.c_double),
                ("f", ctypes.c_double), ("K0", ctypes.c_double), ("rho_floor", ctypes.c_double),
                ("G", ctypes.c_double), ("x_L1", ctypes.c_double)]


class octo_scf_state(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("K", ctypes.c_double), ("C1", ctypes.c_double), ("C2", ctypes.c_double),
                ("x_L1", ctypes.c_double), ("a", ctypes.c_double), ("mass1", ctypes.c_double),
                ("mass2", ctypes.c_double), ("c1", ctypes.c_int64), ("c2", ctypes.c_int64), ("l1", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def make_scf_params(M1, M2, n=1.5, a0=0.35, f=0.9, K0=0.1, rho_floor=1e-10, G=1.0, x_L1=0.0) -> octo_scf_params:
    return octo_scf_params(float(M1), float(M2), float(n), float(a0), float(f), float(K0), float(rho_floor), float(G),
                           float(x_L1))


class octo_regrid_params(ctypes.Structure):
    _fields_ = [("l_max", ctypes.c_int32), ("rho_r", ctypes.c_double), ("n_target", ctypes.c_int64)]


class octo_regrid_stats(ctypes.Structure):
    _fields_ = [("refined", ctypes.c_int64), ("balance_refined", ctypes.c_int64), ("derefined", ctypes.c_int64),
                ("n_leaves", ctypes.c_int64), ("n_grids", ctypes.c_int64), ("rho_r_next", ctypes.c_double),
                ("flag_ms", ctypes.c_double), ("layout_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class octo_stats(ctypes.Structure):
    _fields_ = [("total_mass", ctypes.c_double), ("net_force", ctypes.c_double * 3),
                ("net_torque", ctypes.c_double * 3), ("force_scale", ctypes.c_double),
                ("torque_scale", ctypes.c_double), ("n_leaf_cells", ctypes.c_int64), ("m2l_pairs", ctypes.c_int64),
                ("direct_pairs", ctypes.c_int64), ("m2l_lds_pairs", ctypes.c_int64), ("device_ms", ctypes.c_double),
                ("phase_ms", ctypes.c_double * 8)]

    def as_dict(self):
        F = np.array(self.net_force[:])
        T = np.array(self.net_torque[:])
        return dict(total_mass=self.total_mass, net_force=F, net_torque=T, force_scale=self.force_scale,
                    torque_scale=self.torque_scale, n_leaf_cells=self.n_leaf_cells, m2l_pairs=self.m2l_pairs,
                    direct_pairs=self.direct_pairs, m2l_lds_pairs=self.m2l_lds_pairs, device_ms=self.device_ms,
                    phase_ms=list(self.phase_ms),
                    force=float(np.linalg.norm(F) / self.force_scale) if self.force_scale else 0.0,
                    torque=float(np.linalg.norm(T) / self.torque_scale) if self.torque_scale else 0.0)


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
DENSITY_FN = ctypes.CFUNCTYPE(None, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                              ctypes.c_void_p)
BOXMAX_FN = ctypes.CFUNCTYPE(None, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double), ctypes.c_void_p)


class octo_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


_lib = None
_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.c_int
_I64 = ctypes.c_int64


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load liboctofmm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2101_08226_amd.build` "
                           "or __graft_entry__.build()")
    # PyTorch first: its HIP runtime is then the one the library binds to.
    # Loaded the other way round, the process holds two HIP runtimes (the
    # system's, then PyTorch's bundled one) and the second to start finds no
    # device.
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    sig = {
        "octo_ctx_create": [_I, _P, ctypes.POINTER(octo_allocator), ctypes.c_size_t, _PP],
        "octo_ctx_destroy": [_P],
        "octo_ctx_memory": [_P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)],
        "octo_ctx_set_profiling": [_P, _I],
        "octo_ctx_set_batch_shapes": [_P, _I],
        "octo_tree_build": [_P, ctypes.POINTER(octo_leaf), _I64, _D, _I, _PP],
        "octo_tree_build_device": [_P, _P, _I64, _D, _PP],
        "octo_tree_build_uniform": [_P, _I, _D, _I, _PP],
        "octo_tree_build_adaptive": [_P, DENSITY_FN, BOXMAX_FN, _P, _I, ctypes.c_double, _PP],
        "octo_tree_set_density": [_P, _D, _I],
        "octo_tree_get_density": [_P, _D, _I],
        "octo_regrid": [_P, _P, ctypes.POINTER(octo_regrid_params), _PP, ctypes.POINTER(octo_regrid_stats)],
        "octo_tree_info": [_P, ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_size_t)],
        "octo_tree_leaves": [_P, ctypes.POINTER(octo_leaf)],
        "octo_tree_level_tables": [_P, ctypes.c_int32, ctypes.POINTER(_I64), ctypes.POINTER(octo_level_tables)],
        "octo_tree_destroy": [_P],
        "octo_solve": [_P, _P, ctypes.POINTER(octo_opts), _D, _D, _I, ctypes.POINTER(octo_stats)],
        "octo_solve_device_stats": [_P, _P, ctypes.POINTER(octo_opts), _D, _D, _D],
        "octo_tree_autotune": [_P, _P, ctypes.POINTER(octo_opts), ctypes.POINTER(ctypes.c_int32)],
        "octo_solve_batch": [_P, _PP, ctypes.c_int32, ctypes.POINTER(octo_opts), ctypes.POINTER(_D),
                             ctypes.POINTER(_D), _I, ctypes.POINTER(octo_stats), ctypes.POINTER(ctypes.c_int)],
        "octo_submit": [_P, _P, ctypes.POINTER(octo_opts), _D, _D, ctypes.POINTER(_I64)],
        "octo_solve_dphidt": [_P, _P, ctypes.POINTER(octo_opts), _D, _D],
        "octo_gravity_sources": [_P, _P, _D, _D, _D, _D, _D, _D, _D, _D, _D],
        "octo_energy_update": [_P, _P, _D, _D, _D, _D],
        "octo_scf_step": [_P, _I, ctypes.POINTER(octo_scf_params), ctypes.c_double, ctypes.c_double, _D, _D, _D,
                          ctypes.POINTER(octo_scf_state)],
        "octo_scf_step_noalloc": [_P, _I, ctypes.POINTER(octo_scf_params), ctypes.c_double, ctypes.c_double, _D, _D,
                                  _D, ctypes.POINTER(octo_scf_state)],
        "octo_scf_run": [_P, _P, ctypes.POINTER(octo_opts), ctypes.POINTER(octo_scf_params), ctypes.c_int32, _D, _D,
                         ctypes.POINTER(octo_scf_state)],
        "octo_poll": [_P, _I64, ctypes.POINTER(_I)],
        "octo_wait": [_P, _I64, ctypes.POINTER(octo_stats)],
        "octo_host_stencil_sizes": [ctypes.c_double, ctypes.POINTER(ctypes.c_int32)],
        "octo_host_near_stage": [ctypes.POINTER(ctypes.c_int32), _I64, ctypes.POINTER(_I64)],
        "octo_host_near_lists": [ctypes.c_double, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), _I64,
                                 ctypes.POINTER(_I64)],
        "octo_host_layout": [ctypes.POINTER(octo_leaf), _I64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_I64)],
        "octo_host_level_tables": [ctypes.POINTER(octo_leaf), _I64, ctypes.c_int32, ctypes.POINTER(_I64),
                                   ctypes.POINTER(octo_level_tables)],
        "octo_host_adaptive_leaves": [BOXMAX_FN, _P, _I, ctypes.c_double, ctypes.POINTER(octo_leaf), _I64,
                                      ctypes.POINTER(_I64)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.octo_last_error.argtypes = []
    L.octo_last_error.restype = ctypes.c_char_p
    L.octo_build_id.argtypes = []
    L.octo_build_id.restype = ctypes.c_char_p
    from .build import source_id

    built, want = L.octo_build_id().decode(), source_id()
    if built != want:
        raise RuntimeError(f"{path} was built from other sources (build id {built}, sources {want}): rebuild it "
                           "with `python -m paper_2101_08226_amd.build` or __graft_entry__.build()")
    _lib = L
    return L


def _check(status: int, allow=()):
    if status != OCTO_OK and status not in allow:
        raise OctoError(status, load_library().octo_last_error().decode())
    return status


# ---------------------------------------------------------------- C names

def octo_last_error() -> str:
    return load_library().octo_last_error().decode()


def octo_ctx_create(device: int = 0, hip_stream: int = 0, alloc: Optional[octo_allocator] = None,
                    hbm_budget: int = 0) -> int:
    out = ctypes.c_void_p()
    _check(load_library().octo_ctx_create(device, ctypes.c_void_p(hip_stream or None),
                                          ctypes.byref(alloc) if alloc is not None else None, hbm_budget,
                                          ctypes.byref(out)))
    return out.value


def octo_ctx_destroy(ctx: int) -> None:
    _check(load_library().octo_ctx_destroy(ctx))


def octo_ctx_set_profiling(ctx: int, on) -> None:
    _check(load_library().octo_ctx_set_profiling(ctx, int(on)))


def octo_ctx_set_batch_shapes(ctx: int, mode: int) -> None:
    _check(load_library().octo_ctx_set_batch_shapes(ctx, int(mode)))


def octo_ctx_memory(ctx: int):
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    _check(load_library().octo_ctx_memory(ctx, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def _dptr(p: int):
    return ctypes.cast(ctypes.c_void_p(p), _D)


def octo_tree_build(ctx: int, leaves: np.ndarray, rho_ptr: int, rho_on_device: bool) -> int:
    lv = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32).reshape(-1, 4))
    out = ctypes.c_void_p()
    _check(load_library().octo_tree_build(ctx, lv.ctypes.data_as(ctypes.POINTER(octo_leaf)), lv.shape[0],
                                          _dptr(rho_ptr), int(rho_on_device), ctypes.byref(out)))
    return out.value


def octo_tree_build_device(ctx: int, leaves_ptr: int, n_leaves: int, rho_ptr: int) -> int:
    """Tree from a leaf list (n_leaves x 4 int32) and densities in device memory."""
    out = ctypes.c_void_p()
    _check(load_library().octo_tree_build_device(ctx, leaves_ptr, int(n_leaves), _dptr(rho_ptr), ctypes.byref(out)))
    return out.value


def octo_tree_build_uniform(ctx: int, level: int, rho_ptr: int, rho_on_device: bool) -> int:
    out = ctypes.c_void_p()
    _check(load_library().octo_tree_build_uniform(ctx, level, _dptr(rho_ptr), int(rho_on_device), ctypes.byref(out)))
    return out.value


def octo_tree_build_adaptive(ctx: int, field, max_level: int, threshold: float) -> int:
    """`field` provides density(x, y, z) and boxmax(lo, hi) on numpy arrays."""
    def dens(n, xyz, out, user):
        a = np.ctypeslib.as_array(xyz, shape=(n, 3))
        np.ctypeslib.as_array(out, shape=(n,))[:] = field.density(a[:, 0], a[:, 1], a[:, 2])

    def bmax(n, lo, hi, out, user):
        lo_a = np.ctypeslib.as_array(lo, shape=(n, 3))
        hi_a = np.ctypeslib.as_array(hi, shape=(n, 3))
        np.ctypeslib.as_array(out, shape=(n,))[:] = field.boxmax(lo_a, hi_a)

    fd, fb = DENSITY_FN(dens), BOXMAX_FN(bmax)
    out = ctypes.c_void_p()
    _check(load_library().octo_tree_build_adaptive(ctx, fd, fb, None, max_level, float(threshold), ctypes.byref(out)))
    return out.value


def octo_tree_set_density(tree: int, rho_ptr: int, rho_on_device: bool) -> None:
    _check(load_library().octo_tree_set_density(tree, _dptr(rho_ptr), int(rho_on_device)))


def octo_tree_get_density(tree: int, rho_ptr: int, rho_on_device: bool) -> None:
    _check(load_library().octo_tree_get_density(tree, _dptr(rho_ptr), int(rho_on_device)))


def octo_regrid(ctx: int, tree: int, l_max: int, rho_r: float, n_target: int = 0):
    """One regrid (Sec. 2.7): (new tree handle, octo_regrid_stats)."""
    p = octo_regrid_params(int(l_max), float(rho_r), int(n_target))
    out = ctypes.c_void_p()
    st = octo_regrid_stats()
    _check(load_library().octo_regrid(ctx, tree, ctypes.byref(p), ctypes.byref(out), ctypes.byref(st)))
    return out.value, st


def octo_tree_info(tree: int):
    n, lv, b = _I64(), ctypes.c_int32(), ctypes.c_size_t()
    _check(load_library().octo_tree_info(tree, ctypes.byref(n), ctypes.byref(lv), ctypes.byref(b)))
    return n.value, lv.value, b.value


def octo_tree_leaves(tree: int) -> np.ndarray:
    n, _, _ = octo_tree_info(tree)
    out = np.empty((n // 512, 4), dtype=np.int32)
    _check(load_library().octo_tree_leaves(tree, out.ctypes.data_as(ctypes.POINTER(octo_leaf))))
    return out


def _level_tables(call) -> dict:
    """Sizes, then the tables of one level (the octo_level_tables format) as
    numpy arrays: nbr (n, 27), child (n_int, 8), parent (n,), coord (n, 3),
    out_base (n,), flags (n,), int_child (n_int,)."""
    sizes = np.zeros(3, dtype=np.int64)
    _check(call(sizes.ctypes.data_as(ctypes.POINTER(_I64)), None))
    n, n_int, n_rec = (int(v) for v in sizes)
    t = {"nbr": np.empty((n, 27), np.int32), "child": np.empty((n_int, 8), np.int32),
         "parent": np.empty(n, np.int32), "coord": np.empty((n, 3), np.int32), "out_base": np.empty(n, np.int64),
         "flags": np.empty(n, np.int32), "int_child": np.empty(n_int, np.int32)}
    out = octo_level_tables(*(t[k].ctypes.data for k in ("nbr", "child", "parent", "coord", "out_base", "flags",
                                                         "int_child")))
    _check(call(sizes.ctypes.data_as(ctypes.POINTER(_I64)), ctypes.byref(out)))
    t.update(n_nodes=n, n_int=n_int, n_rec=n_rec)
    return t


def octo_tree_level_tables(tree: int, level: int) -> dict:
    """The node tables of one level of a tree, copied from device memory."""
    return _level_tables(lambda sz, out: load_library().octo_tree_level_tables(tree, int(level), sz, out))


def octo_host_level_tables(leaves, level: int) -> dict:
    """The node tables the host builder gives one level of a leaf list."""
    lv = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32).reshape(-1, 4))
    ptr = lv.ctypes.data_as(ctypes.POINTER(octo_leaf))
    return _level_tables(lambda sz, out: load_library().octo_host_level_tables(ptr, lv.shape[0], int(level), sz,
                                                                               out))


def octo_tree_destroy(tree: int) -> None:
    _check(load_library().octo_tree_destroy(tree))


def make_opts(theta=0.5, G=1.0, precision=OCTO_FP64, amc=True) -> octo_opts:
    return octo_opts(float(theta), float(G), int(precision), int(bool(amc)))


def octo_solve(ctx: int, tree: int, opts: octo_opts, phi_ptr: int, g_ptr: int, out_on_device: bool,
               want_stats: bool = True):
    st = octo_stats()
    _check(load_library().octo_solve(ctx, tree, ctypes.byref(opts), _dptr(phi_ptr), _dptr(g_ptr),
                                     int(out_on_device), ctypes.byref(st) if want_stats else None))
    return st if want_stats else None


def octo_tree_autotune(ctx: int, tree: int, opts: octo_opts) -> list:
    _, nl, _ = octo_tree_info(tree)
    out = (ctypes.c_int32 * nl)()
    _check(load_library().octo_tree_autotune(ctx, tree, ctypes.byref(opts), out))
    return list(out)


def octo_solve_batch(ctx: int, trees: Sequence[int], opts: octo_opts, phi_ptrs: Sequence[int],
                     g_ptrs: Sequence[int], out_on_device: bool, want_stats: bool = True, status_out=None):
    """Solve the trees together; raises on any refused tree unless
    `status_out` (a list) is given, which then receives every tree's status."""
    n = len(trees)
    tr = (ctypes.c_void_p * n)(*[t or None for t in trees])
    ph = (_D * n)(*[_dptr(p) for p in phi_ptrs])
    gg = (_D * n)(*[_dptr(p) for p in g_ptrs])
    st = (octo_stats * n)()
    ss = (ctypes.c_int * n)()
    rc = load_library().octo_solve_batch(ctx, tr, n, ctypes.byref(opts), ph, gg, int(out_on_device),
                                         st if want_stats else None, ss)
    if status_out is not None:
        status_out[:] = list(ss)
    else:
        _check(rc)
    return list(st) if want_stats else None


def octo_solve_device_stats(ctx: int, tree: int, opts: octo_opts, phi_ptr: int, g_ptr: int, stats_ptr: int) -> None:
    _check(load_library().octo_solve_device_stats(ctx, tree, ctypes.byref(opts), _dptr(phi_ptr), _dptr(g_ptr),
                                                  _dptr(stats_ptr)))


def octo_solve_dphidt(ctx: int, tree: int, opts: octo_opts, drho_dt: int, dphi_dt: int) -> None:
    _check(load_library().octo_solve_dphidt(ctx, tree, ctypes.byref(opts), _dptr(drho_dt), _dptr(dphi_dt)))


def octo_gravity_sources(ctx: int, tree: int, omega, rho: int, s: int, phi: int, g: int, drho_dt: int,
                         dphi_dt: int, src_s: int, src_e: int) -> None:
    om = np.ascontiguousarray(omega, dtype=np.float64)
    _check(load_library().octo_gravity_sources(ctx, tree, om.ctypes.data_as(_D), _dptr(rho), _dptr(s), _dptr(phi),
                                               _dptr(g), _dptr(drho_dt), _dptr(dphi_dt), _dptr(src_s), _dptr(src_e)))


def octo_energy_update(ctx: int, tree: int, rho: int, phi_before: int, phi_after: int, E: int) -> None:
    _check(load_library().octo_energy_update(ctx, tree, _dptr(rho), _dptr(phi_before), _dptr(phi_after), _dptr(E)))


def octo_scf_step(ctx: int, level: int, params: octo_scf_params, K: float, x_L1: float, rho: int, phi: int,
                  rho_out: int) -> octo_scf_state:
    st = octo_scf_state()
    _check(load_library().octo_scf_step(ctx, int(level), ctypes.byref(params), float(K), float(x_L1), _dptr(rho),
                                        _dptr(phi), _dptr(rho_out), ctypes.byref(st)))
    return st


def octo_scf_step_noalloc(ctx: int, level: int, params: octo_scf_params, K: float, x_L1: float, rho: int, phi: int,
                          rho_out: int) -> octo_scf_state:
    st = octo_scf_state()
    _check(load_library().octo_scf_step_noalloc(ctx, int(level), ctypes.byref(params), float(K), float(x_L1),
                                                _dptr(rho), _dptr(phi), _dptr(rho_out), ctypes.byref(st)))
    return st


def octo_scf_run(ctx: int, tree: int, opts: octo_opts, params: octo_scf_params, iterations: int, rho_out: int,
                 phi_out: int) -> list:
    hist = (octo_scf_state * max(1, iterations))()
    _check(load_library().octo_scf_run(ctx, tree, ctypes.byref(opts), ctypes.byref(params), int(iterations),
                                       _dptr(rho_out), _dptr(phi_out), hist))
    return list(hist)[:iterations]


def octo_submit(ctx: int, tree: int, opts: octo_opts, phi_ptr: int, g_ptr: int) -> int:
    t = _I64()
    _check(load_library().octo_submit(ctx, tree, ctypes.byref(opts), _dptr(phi_ptr), _dptr(g_ptr), ctypes.byref(t)))
    return t.value


def octo_poll(ctx: int, ticket: int) -> bool:
    d = _I()
    s = _check(load_library().octo_poll(ctx, ticket, ctypes.byref(d)), allow=(OCTO_E_PENDING,))
    return s == OCTO_OK and d.value == 1


def octo_wait(ctx: int, ticket: int) -> octo_stats:
    st = octo_stats()
    _check(load_library().octo_wait(ctx, ticket, ctypes.byref(st)))
    return st


def octo_host_stencil_sizes(theta: float) -> np.ndarray:
    out = np.zeros(24, dtype=np.int32)
    _check(load_library().octo_host_stencil_sizes(float(theta), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return out


def octo_host_near_lists(theta: float) -> tuple:
    """(beg (73,), d (n, 3)) of the leaf kernel's near-field walk; padding rows are (0, 0, 0)."""
    beg = np.zeros(73, dtype=np.int32)
    n = _I64(0)
    P32 = ctypes.POINTER(ctypes.c_int32)
    _check(load_library().octo_host_near_lists(float(theta), beg.ctypes.data_as(P32), None, 0, ctypes.byref(n)))
    packed = np.zeros(n.value, dtype=np.int32)
    _check(load_library().octo_host_near_lists(float(theta), beg.ctypes.data_as(P32), packed.ctypes.data_as(P32),
                                               n.value, ctypes.byref(n)))
    d = np.stack([((packed >> (8 * a)) & 255).astype(np.int8).astype(np.int64) for a in range(3)], axis=1)
    return beg, d


def octo_host_near_stage() -> np.ndarray:
    """The near-field kernel's halo staging table (6144 packed entries, -1 past the 18^3 halo cells)."""
    n = _I64(0)
    _check(load_library().octo_host_near_stage(None, 0, ctypes.byref(n)))
    out = np.zeros(n.value, dtype=np.int32)
    _check(load_library().octo_host_near_stage(out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n.value,
                                               ctypes.byref(n)))
    return out


def octo_host_layout(leaves) -> tuple:
    lv = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32).reshape(-1, 4))
    n = ctypes.c_int32()
    out = np.zeros(30, dtype=np.int64)
    _check(load_library().octo_host_layout(lv.ctypes.data_as(ctypes.POINTER(octo_leaf)), lv.shape[0],
                                           ctypes.byref(n), out.ctypes.data_as(ctypes.POINTER(_I64))))
    return n.value, out.reshape(10, 3)[: n.value]


def octo_host_adaptive_leaves(field, max_level: int, threshold: float) -> np.ndarray:
    def bmax(n, lo, hi, out, user):
        lo_a = np.ctypeslib.as_array(lo, shape=(n, 3))
        hi_a = np.ctypeslib.as_array(hi, shape=(n, 3))
        np.ctypeslib.as_array(out, shape=(n,))[:] = field.boxmax(lo_a, hi_a)

    fb = BOXMAX_FN(bmax)
    n = _I64()
    _check(load_library().octo_host_adaptive_leaves(fb, None, max_level, float(threshold), None, 0, ctypes.byref(n)))
    out = np.empty((n.value, 4), dtype=np.int32)
    _check(load_library().octo_host_adaptive_leaves(fb, None, max_level, float(threshold),
                                                    out.ctypes.data_as(ctypes.POINTER(octo_leaf)), n.value,
                                                    ctypes.byref(n)))
    return out


# ---------------------------------------------------------------- torch glue

class Context:
    """A library context on one GPU whose device memory comes from PyTorch's
    caching allocator and whose launches go to a dedicated PyTorch stream."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the HIP library needs a ROCm device")
        load_library()
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.Stream(device=self.device)
        self._blocks = {}

        def _alloc(nbytes, user):
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            p = t.data_ptr()
            self._blocks[p] = t
            return p

        def _free(ptr, user):
            self._blocks.pop(ptr, None)

        self._cb = (ALLOC_FN(_alloc), FREE_FN(_free))
        self._alloc = octo_allocator(self._cb[0], self._cb[1], None)
        self.handle = octo_ctx_create(device, self.stream.cuda_stream, self._alloc, hbm_budget)

    def close(self):
        if getattr(self, "handle", None):
            octo_ctx_destroy(self.handle)
            self.handle = None

    def memory(self):
        return octo_ctx_memory(self.handle)

    def set_profiling(self, on) -> None:
        """0/False off; 1/True phase timings with statistics; 2 timings only."""
        octo_ctx_set_profiling(self.handle, int(on))

    def set_batch_shapes(self, mode: int) -> None:
        """Batches of several trees: 0 each tree's own plan (bitwise as
        alone), 1 work shapes fitted to the batch."""
        octo_ctx_set_batch_shapes(self.handle, int(mode))

    def uniform_tree(self, rho) -> "Tree":
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        n = rho.shape[0]
        level = int(np.log2(n // 8))
        assert rho.shape == (n, n, n) and (8 << level) == n
        return Tree(self, octo_tree_build_uniform(self.handle, level, rho.ctypes.data, False), grid=n)

    def tree(self, leaves, rho) -> "Tree":
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        return Tree(self, octo_tree_build(self.handle, leaves, rho.ctypes.data, False))

    def tree_from_device(self, leaves, rho) -> "Tree":
        """Tree laid out on the device from a leaf list and densities in
        device memory (int32 (n, 4) and float64 (n, 512) tensors)."""
        torch = self.torch
        leaves = leaves.to(device=self.device, dtype=torch.int32).contiguous()
        rho = rho.to(device=self.device, dtype=torch.float64).contiguous()
        if leaves.dim() != 2 or leaves.shape[1] != 4 or rho.numel() != leaves.shape[0] * 512:
            raise ValueError("leaves must be (n, 4) and rho n x 512 values")
        self.stream.wait_stream(torch.cuda.current_stream(self.device))  # the tensors are written first
        return Tree(self, octo_tree_build_device(self.handle, leaves.data_ptr(), leaves.shape[0], rho.data_ptr()))

    def adaptive_tree(self, field, max_level: int, threshold: float) -> "Tree":
        return Tree(self, octo_tree_build_adaptive(self.handle, field, max_level, threshold))

    def solve(self, tree: "Tree", theta=0.5, precision=OCTO_FP64, amc=True, G=1.0, out=None, stats=True):
        """phi (n,) and g (3, n) as float64 tensors on the device, in the tree's
        density layout, plus the solve statistics."""
        torch = self.torch
        n = tree.n_leaf_cells
        if out is None:
            phi = torch.empty(n, dtype=torch.float64, device=self.device)
            g = torch.empty((3, n), dtype=torch.float64, device=self.device)
        else:
            phi, g = out
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        st = octo_solve(self.handle, tree.handle, make_opts(theta, G, precision, amc), phi.data_ptr(), g.data_ptr(),
                        True, want_stats=stats)
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return phi, g, (st.as_dict() if st is not None else None)

    def solve_batch(self, trees, theta=0.5, precision=OCTO_FP64, amc=True, G=1.0, outs=None, stats=True):
        torch = self.torch
        if outs is None:
            outs = [(torch.empty(t.n_leaf_cells, dtype=torch.float64, device=self.device),
                     torch.empty((3, t.n_leaf_cells), dtype=torch.float64, device=self.device)) for t in trees]
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        st = octo_solve_batch(self.handle, [t.handle for t in trees], make_opts(theta, G, precision, amc),
                              [o[0].data_ptr() for o in outs], [o[1].data_ptr() for o in outs], True,
                              want_stats=stats)
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return outs, ([s.as_dict() for s in st] if st is not None else None)

    def solve_dphidt(self, tree: "Tree", drho_dt, theta=0.5, precision=OCTO_FP64, G=1.0, out=None):
        """dphi/dt (n,) on the device from the density rate drho_dt (a float64
        device tensor in the tree's density layout)."""
        torch = self.torch
        n = tree.n_leaf_cells
        assert drho_dt.dtype == torch.float64 and drho_dt.is_contiguous() and drho_dt.numel() == n
        dphi = torch.empty(n, dtype=torch.float64, device=self.device) if out is None else out
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        octo_solve_dphidt(self.handle, tree.handle, make_opts(theta, G, precision, False), drho_dt.data_ptr(),
                          dphi.data_ptr())
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return dphi

    def scf_step(self, level: int, rho, phi, K: float, x_L1: float, params: octo_scf_params, out=None):
        """Steps 2-6 of one SCF iteration (Sec. 4.1) from a normalised density
        and its potential (float64 device tensors, n^3 in grid order): the new
        density and the iteration's scalars."""
        torch = self.torch
        n3 = (8 << level) ** 3
        for t in (rho, phi):
            assert t.dtype == torch.float64 and t.is_contiguous() and t.numel() == n3 and t.device == self.device
        rho_out = torch.empty(n3, dtype=torch.float64, device=self.device) if out is None else out
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        st = octo_scf_step(self.handle, level, params, K, x_L1, rho.data_ptr(), phi.data_ptr(), rho_out.data_ptr())
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return rho_out, st.as_dict()

    def scf_run(self, tree: "Tree", params: octo_scf_params, iterations: int, theta=0.5, precision=OCTO_FP64,
                amc=True):
        """SCF iterations (Sec. 4.1) on a uniform tree from its density: the
        final normalised density, its potential (n^3 device tensors, grid
        order) and the scalars of every iteration."""
        torch = self.torch
        n = tree.n_leaf_cells
        rho = torch.empty(n, dtype=torch.float64, device=self.device)
        phi = torch.empty(n, dtype=torch.float64, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        hist = octo_scf_run(self.handle, tree.handle, make_opts(theta, params.G, precision, amc), params, iterations,
                            rho.data_ptr(), phi.data_ptr())
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return rho, phi, [h.as_dict() for h in hist]

    def gravity_sources(self, tree: "Tree", omega, rho, s, phi, g, drho_dt=None, dphi_dt=None):
        """Source terms (src_s (3, n), src_e (n)) from device tensors in the
        tree's layout."""
        torch = self.torch
        n = tree.n_leaf_cells
        src_s = torch.empty((3, n), dtype=torch.float64, device=self.device)
        src_e = torch.empty(n, dtype=torch.float64, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        octo_gravity_sources(self.handle, tree.handle, omega, rho.data_ptr(), s.data_ptr(), phi.data_ptr(),
                             g.data_ptr(), drho_dt.data_ptr() if drho_dt is not None else 0,
                             dphi_dt.data_ptr() if dphi_dt is not None else 0, src_s.data_ptr(), src_e.data_ptr())
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return src_s, src_e

    def energy_update(self, tree: "Tree", rho, phi_before, phi_after, E) -> None:
        torch = self.torch
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        octo_energy_update(self.handle, tree.handle, rho.data_ptr(), phi_before.data_ptr(), phi_after.data_ptr(),
                           E.data_ptr())
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tree:
    def __init__(self, ctx: Context, handle: int, grid: Optional[int] = None):
        self.ctx = ctx
        self.handle = handle
        self.grid = grid
        self.n_leaf_cells, self.n_levels, self.bytes = octo_tree_info(handle)

    def leaves(self) -> np.ndarray:
        return octo_tree_leaves(self.handle)

    def level_tables(self, level: int) -> dict:
        return octo_tree_level_tables(self.handle, level)

    def autotune(self, theta=0.5, precision=OCTO_FP64, amc=True, G=1.0) -> list:
        """Pick the multipole work shape per level by timing; returns the choice
        per level (-1 none, 0 LDS-staged, k chunks)."""
        return octo_tree_autotune(self.ctx.handle, self.handle, make_opts(theta, G, precision, amc))

    def set_density(self, rho) -> None:
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        octo_tree_set_density(self.handle, rho.ctypes.data, False)

    def density(self) -> np.ndarray:
        """The tree's density (its layout) copied to the host."""
        out = np.empty(self.n_leaf_cells, dtype=np.float64)
        octo_tree_get_density(self.handle, out.ctypes.data, False)
        return out

    def regrid(self, l_max: int, rho_r: float, n_target: int = 0):
        """One regrid by the density criterion (Sec. 2.7): the new Tree and the
        regrid statistics; this tree is unchanged."""
        h, st = octo_regrid(self.ctx.handle, self.handle, l_max, rho_r, n_target)
        return Tree(self.ctx, h), st.as_dict()

    def destroy(self):
        if self.handle:
            octo_tree_destroy(self.handle)
            self.handle = None
