"""The allocation-free SCF step (octo_scf_step_noalloc) against the allocating
one (octo_scf_step), both called through the C interface.

Both run the same kernels with the same launch shapes; only where the scratch
lives differs (a fixed per-device array instead of memory from the context's
allocator), so the new density and every scalar must agree bit for bit.  Two
calls in a row, the second on a smaller grid, check that what the first call
leaves in the shared array does not leak into the second.
"""
import sys

import numpy as np
import pytest

import paper_2101_08226_amd as lib
import workloads as w
from helpers import fft_poisson
from oracle import scf as S

pytestmark = pytest.mark.gpu

FIELDS = ("omega", "K", "C1", "C2", "x_L1", "a", "mass1", "mass2", "c1", "c2", "l1")


def say(*a):
    print("[no-alloc]", *a, flush=True)
    sys.stdout.flush()


def _inputs(level, x_L1):
    p = S.SCFParams(M1=1.0, M2=0.7, a0=0.4, f=0.9)
    rho0, p.K0 = w.scf_initial_binary(level, 1.0, 0.7, 0.4, 0.12, 0.10, yz=(0.0123, 0.0071))
    rho = S.normalise(rho0, level, p, x_L1)
    phi = fft_poisson(level)(rho)
    par = lib.make_scf_params(p.M1, p.M2, p.n, p.a0, p.f, p.K0, p.floor, p.G, 0.0)
    return rho, phi, par, p.K0


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).to("cuda:0")


def _run(fn, ctx, level, rho, phi, par, K, x_L1):
    import torch

    n3 = (8 << level) ** 3
    d_rho, d_phi = _dev(rho), _dev(phi)
    out = torch.full((n3,), float("nan"), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    st = fn(ctx.handle, level, par, K, x_L1, d_rho.data_ptr(), d_phi.data_ptr(), out.data_ptr())
    torch.cuda.synchronize()
    return out.cpu().numpy(), st.as_dict()


def test_noalloc_step_equals_allocating_step():
    ctx = lib.Context(0)
    try:
        # level 4 (128^3, 1024 partials) first, then level 2 (32^3, 16
        # partials): the second call's partials sit where the first call's
        # larger set was
        for level, x_L1 in ((4, 0.0), (2, -3.0 / 64)):
            rho, phi, par, K = _inputs(level, x_L1)
            say(f"level={level} x_L1={x_L1}: octo_scf_step_noalloc then octo_scf_step")
            out_n, st_n = _run(lib.octo_scf_step_noalloc, ctx, level, rho, phi, par, K, x_L1)
            out_a, st_a = _run(lib.octo_scf_step, ctx, level, rho, phi, par, K, x_L1)
            assert np.all(np.isfinite(out_n))
            assert np.array_equal(out_n.view(np.uint64), out_a.view(np.uint64)), level
            for k in FIELDS:
                assert st_n[k] == st_a[k], (level, k, st_n[k], st_a[k])
            say(f"level={level}: bitwise equal, c=({st_n['c1']},{st_n['c2']}) l1={st_n['l1']}")
        # outside the levels the fixed array covers: rejected, nothing launched
        rho, phi, par, K = _inputs(0, 0.0)
        with pytest.raises(lib.OctoError) as e:
            lib.octo_scf_step_noalloc(ctx.handle, 7, par, K, 0.0, 1, 1, 1)
        assert e.value.status == lib.OCTO_E_INVALID
    finally:
        ctx.close()
