"""Benchmark: FMM leaf cells solved per second on one MI355X.

Headline workload (the default, --config all): the adaptive tree of the
binary-polytrope field (two n = 3/2 polytropes, radii 0.12 and 0.10, centres
0.35 apart, mass ratio 0.7, maximum density 1, floor 1e-10) refined where the
box maximum of the density exceeds 1e-4, to level 6 with the root sub-grid at
level 0 (7,736 leaf sub-grids, 3.96M leaf cells), theta = 0.5, FP64 with the
angular-momentum correction.  One step = one full solve with the tree and
density resident in HBM: P2M, M2M, M2L with the correction, L2L, leaf near
field, L2P and the net force / torque reductions, whose results stay in
device memory (octo_solve_device_stats), steps queued back to back on the
library's stream.  Beside it: the same solve with the statistics copied to the
host (pairs counted, each step waiting for its solve), the solve without the
reductions, and mixed precision.

Further fields of the default line: the same field to level 7 (20.0M leaf
cells); the uniform 128^3 grid of that field (c2) with the roofline of its
multipole kernel and the self-consistent-field iteration; 256 independent
uniform trees solved together (c4: work shapes fitted to the batch, and each
tree's own plan beside it); a Poisson stream of 2,000 solve requests
served with continuous batching (c5: p50/p99 latency, throughput); the time
derivative of the potential and one regrid of the headline tree; and the CPU
oracle timed on this host.  --config c1..c5 runs one workload alone.

Prints one JSON line.  The roofline block is the dominant kernel of the
headline workload (the LDS-staged multipole-to-local kernel), its duration
measured with HIP events on the library's stream.
"""
import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FMM cells solved/s (FP64 vs mixed, 1 GPU); p50/p99 served solve latency"

# Algorithmic FP64 operations per ordered multipole-to-local pair with an
# interior target and the correction on, in the trace-free formulation the
# kernels use: adds, multiplies and rsqrt count as one, a fused multiply-add as
# two (150 for R and the L0..L3 terms, 64 for the correction and the mass
# ratio); the accounting is in the design notes.
M2L_FLOPS_PER_PAIR = 214
PEAK_FP64_TFLOPS = 78.6  # MI355X FP64 vector
PEAK_HBM_GBS = 8000.0    # MI355X HBM3E
PHASES = ["p2m", "near", "m2m", "m2l", "l2l", "l2p", "stats", "m2l_lds_kernel"]
KERNEL_SOURCE = os.path.join(ROOT, "paper_2101_08226_amd", "csrc", "kernels.hip")
LDS_KERNEL = "k_m2l_lds<double, false, true, false>"


def traffic_record(workload):
    """HBM traffic of the LDS-staged multipole kernel (rocprofv3 FETCH_SIZE and
    WRITE_SIZE passes scaled by a copy of known size) from its record under
    profiles/, or None when there is none or it was taken with another
    kernels.hip."""
    path = os.path.join(ROOT, "profiles", f"k_m2l_lds_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if rec.get("kernels_hip_sha256") != src or "traffic_bytes_per_launch" not in rec:
        return None
    return float(rec["traffic_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", choices=["all", "c1", "c2", "c3", "c3l7", "c4", "c5"], default="all")
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-threads", type=int, default=int(os.environ.get("OMP_NUM_THREADS", "16") or 16))
    ap.add_argument("--requests", type=int, default=2000, help="c5: number of requests")
    ap.add_argument("--rate", type=float, default=0.0, help="c5: arrivals per second (0: 0.8 x measured saturation)")
    ap.add_argument("--budget-gib", type=float, default=16.0, help="c5: HBM budget of the server context")
    ap.add_argument("--scf-level", type=int, default=4, help="c2: uniform level of the SCF grid (4: 128^3)")
    ap.add_argument("--scf-iters", type=int, default=20, help="c2: SCF iterations per timed run")
    ap.add_argument("--skip", default="", help="comma list of default-line blocks to leave out "
                                               "(c3l7,c2,c4,c5,dphidt,regrid,scf)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device-to-device copy of this many bytes (counter calibration) and exit")
    return ap.parse_args()


def say(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def timed(step, sync, steps, warmup):
    for _ in range(warmup):
        step()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    sync()
    return (time.perf_counter() - t0) / steps


def phase_times(ctx, solve_once, n=5):
    # timing-only profiling: the kernels one by one, as they run in solves
    # without statistics (no pair-counting pass)
    ctx.set_profiling(2)
    acc = np.zeros(8)
    for _ in range(n):
        acc += np.array(solve_once().phase_ms[:])
    ctx.set_profiling(False)
    return acc / n


def roofline_m2l(pairs, kernel_ms, traffic=None):
    """The LDS-staged multipole kernel alone: its pairs (counted in a solve
    with statistics) x the per-pair count over its own launch duration (HIP
    events around it, kernels one by one, timing-only profiling)."""
    achieved = pairs * M2L_FLOPS_PER_PAIR / (kernel_ms * 1e-3) / 1e12
    # the FP64 solve's kernel, against the FP64 peak (the mixed mode's FP32 variant is reported by its time only)
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": traffic,
            "kernel": LDS_KERNEL, "kernel_ms": round(kernel_ms, 4), "pairs_per_launch": int(pairs),
            "flops_per_pair": M2L_FLOPS_PER_PAIR}


def tree_counts(leaves):
    """Leaf cells and interior cells of a leaf list."""
    interior = set()
    for l, x, y, z in leaves:
        for k in range(1, int(l) + 1):
            interior.add((int(l) - k, int(x) >> k, int(y) >> k, int(z) >> k))
    n_leaf = 512 * len(leaves)
    n_int = 512 * len(interior)
    return n_leaf, n_int


def hbm_phases(phases, leaves):
    """Algorithmic bytes of the HBM-bound phases over their measured
    durations (timing-only profiling): P2M reads rho and writes m and the
    parent cell's child-mass entry (24 B per leaf cell); M2M writes a 160 B record (mass, centre, 6 + 10 moments) per
    interior cell and reads each child once (160 B per interior child cell,
    8 B per leaf child cell); L2L reads 184 B of partial sums and writes 184 B
    of locals per interior cell below the root, plus the parent's 184 B per
    8 children; L2P reads the 32 B near-field sums and writes phi and g (32
    B) per leaf cell, plus the parent's locals (184 B per 8 leaf cells)."""
    n_leaf, n_int = tree_counts(leaves)
    root_int = 512 if n_int else 0
    b = {"p2m": 24.0 * n_leaf,
         "m2m": 160.0 * n_int + 160.0 * (n_int - root_int) + 8.0 * n_leaf,
         "l2l": (184.0 * 2 + 23.0) * (n_int - root_int),
         "l2p": (32.0 + 32.0 + 23.0) * n_leaf}
    out = {}
    for k, idx in (("p2m", 0), ("m2m", 2), ("l2l", 4), ("l2p", 5)):
        ms = float(phases[idx])
        gbs = b[k] / (ms * 1e-3) / 1e9 if ms > 0 else None
        out[k] = {"ms": round(ms, 4), "bytes": int(b[k]), "GB/s": round(gbs, 1) if gbs else None,
                  "frac_of_8TB/s": round(gbs / PEAK_HBM_GBS, 4) if gbs else None}
    return out


def single_tree(a, lib, ctx, tree, rate=None, with_dphidt=True, stats_steps=None):
    """FP64 and mixed solves of one tree.  The step timed for the headline is
    the whole solve including the net force / torque reductions, left in
    device memory (octo_solve_device_stats), steps queued back to back on the
    stream; beside it the same solve with the statistics copied to the host
    (each step waits for its solve) and without reductions; phase times; and
    dphi/dt of a density rate."""
    import torch

    dev = ctx.device
    n = tree.n_leaf_cells
    phi = torch.empty(n, dtype=torch.float64, device=dev)
    g = torch.empty((3, n), dtype=torch.float64, device=dev)
    dst = torch.zeros(9, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def sync():
        ctx.stream.synchronize()
        torch.cuda.synchronize()

    res = {}
    for pn, prec in (("fp64", lib.OCTO_FP64), ("mixed", lib.OCTO_MIXED)):
        opts = lib.make_opts(a.theta, 1.0, prec, True)
        st = lib.octo_solve(ctx.handle, tree.handle, opts, phi.data_ptr(), g.data_ptr(), True).as_dict()
        say(f"{n} cells {pn}: with the reductions on the device")
        sec = timed(lambda: lib.octo_solve_device_stats(ctx.handle, tree.handle, opts, phi.data_ptr(), g.data_ptr(),
                                                        dst.data_ptr()), sync, a.steps, a.warmup)
        say(f"{n} cells {pn}: with host statistics")
        sec_host = timed(lambda: lib.octo_solve(ctx.handle, tree.handle, opts, phi.data_ptr(), g.data_ptr(), True),
                         sync, stats_steps or a.steps, a.warmup)
        say(f"{n} cells {pn}: no reductions")
        sec_ns = timed(lambda: lib.octo_solve(ctx.handle, tree.handle, opts, phi.data_ptr(), g.data_ptr(), True,
                                              want_stats=False), sync, a.steps, a.warmup)
        ph = phase_times(ctx, lambda: lib.octo_solve(ctx.handle, tree.handle, opts, phi.data_ptr(),
                                                     g.data_ptr(), True))
        res[pn] = dict(sec=sec, sec_host=sec_host, sec_ns=sec_ns, stats=st, phases=ph)
    if rate is not None and with_dphidt:
        drho = torch.tensor(np.ascontiguousarray(rate).ravel(), dtype=torch.float64, device=dev)
        dphi = torch.empty(n, dtype=torch.float64, device=dev)
        for pn, prec in (("fp64", lib.OCTO_FP64), ("mixed", lib.OCTO_MIXED)):
            opts = lib.make_opts(a.theta, 1.0, prec, False)
            say(f"{n} cells dphi/dt {pn}")
            sec = timed(lambda: lib.octo_solve_dphidt(ctx.handle, tree.handle, opts, drho.data_ptr(),
                                                      dphi.data_ptr()), sync, a.steps, a.warmup)
            res["dphidt_" + pn] = dict(sec=sec)
    return res


def block(res, n, desc, theta, traffic=None, leaves=None):
    """JSON fields of a single-tree workload."""
    r, m = res["fp64"], res["mixed"]
    out = {"workload": desc, "leaf_cells": int(n), "theta": theta,
           "value": round(n / r["sec"], 1), "ms_per_step": round(r["sec"] * 1e3, 4),
           "with_host_statistics": {"value": round(n / r["sec_host"], 1),
                                    "ms_per_step": round(r["sec_host"] * 1e3, 4),
                                    "note": "pairs counted, statistics copied to the host and awaited every step"},
           "no_reductions": {"value": round(n / r["sec_ns"], 1), "ms_per_step": round(r["sec_ns"] * 1e3, 4)},
           "m2l_pairs": int(r["stats"]["m2l_pairs"]), "direct_pairs": int(r["stats"]["direct_pairs"]),
           "torque": r["stats"]["torque"], "force": r["stats"]["force"],
           "roofline": roofline_m2l(r["stats"]["m2l_lds_pairs"], r["phases"][7], traffic),
           "phase_ms": {k: round(v, 4) for k, v in zip(PHASES, r["phases"])},
           "mixed": {"value": round(n / m["sec"], 1), "ms_per_step": round(m["sec"] * 1e3, 4),
                     "with_host_statistics_ms": round(m["sec_host"] * 1e3, 4),
                     "no_reductions_ms": round(m["sec_ns"] * 1e3, 4),
                     "torque": m["stats"]["torque"],
                     "phase_ms": {k: round(v, 4) for k, v in zip(PHASES, m["phases"])}}}
    if leaves is not None:
        out["hbm_phases"] = hbm_phases(r["phases"], leaves)
    for k in ("dphidt_fp64", "dphidt_mixed"):
        if k in res:
            out.setdefault("dphidt", {})[k.split("_")[1]] = {
                "value": round(n / res[k]["sec"], 1), "ms_per_step": round(res[k]["sec"] * 1e3, 4)}
    return out


def scf_bench(a, lib, w, ctx, level, iters):
    """Self-consistent-field iterations (initial binary model, Sec. 4.1) on
    the uniform grid of `level`: each timed run restores the starting
    density, then runs `iters` iterations (normalise, solve, steps 2-6) plus
    the closing normalise and solve; a run of 0 iterations times that
    frame, and the difference over `iters` is the time of one iteration."""
    import torch

    rho0, K0 = w.scf_initial_binary(level, 1.0, 0.7, 0.4, 0.12, 0.10, yz=(0.0123, 0.0071))
    n = rho0.shape[0]
    par = lib.make_scf_params(1.0, 0.7, 1.5, 0.4, 0.9, K0, 1e-10, 1.0, 0.0)
    tree = ctx.uniform_tree(rho0)
    start = torch.tensor(rho0.ravel(), dtype=torch.float64, device=ctx.device)
    rho = torch.empty(n ** 3, dtype=torch.float64, device=ctx.device)
    phi = torch.empty(n ** 3, dtype=torch.float64, device=ctx.device)
    opts = lib.make_opts(a.theta, 1.0, lib.OCTO_FP64, True)
    torch.cuda.synchronize()

    def run(k):
        lib.octo_tree_set_density(tree.handle, start.data_ptr(), True)
        return lib.octo_scf_run(ctx.handle, tree.handle, opts, par, k, rho.data_ptr(), phi.data_ptr())

    say(f"SCF {n}^3: {iters} iterations per run")
    for _ in range(2):
        run(iters)
        run(0)
    t_it, t_0 = [], []
    for _ in range(5):
        t0 = time.perf_counter()
        hist = run(iters)
        t_it.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        run(0)
        t_0.append(time.perf_counter() - t0)
    tree.destroy()
    per = (float(np.median(t_it)) - float(np.median(t_0))) / iters
    last = hist[-1]
    return {"grid": f"{n}^3", "cells": n ** 3, "iterations": iters, "ms_per_iteration": round(per * 1e3, 4),
            "iterations_per_s": round(1.0 / per, 1), "frame_ms": round(float(np.median(t_0)) * 1e3, 4),
            "model": "n=1.5 binary, M1=1, M2=0.7, a0=0.4, f=0.9, R=0.12/0.10 start, stars' axis at y,z=0.0123,0.0071",
            "last": {"omega": last.omega, "K": last.K, "C1": last.C1, "C2": last.C2, "x_L1": last.x_L1, "a": last.a}}


def regrid_bench(tree, host_build_ms, l_max=7, rho_r=0.1, n_target=4000, reps=5):
    """One regrid of the adaptive tree by the density criterion on the device
    (flags, balance, new leaves and densities) plus the new tree's layout
    (on the device) and work plan; the tree's own host build from the
    analytic field beside it."""
    say(f"regrid: {reps} runs")
    t2, st = tree.regrid(l_max, rho_r, n_target)  # warm-up
    t2.destroy()
    wall, flag, lay = [], [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        t2, st = tree.regrid(l_max, rho_r, n_target)
        wall.append((time.perf_counter() - t0) * 1e3)
        flag.append(st["flag_ms"])
        lay.append(st["layout_ms"])
        t2.destroy()
    return {"l_max": l_max, "rho_r": rho_r, "n_target": n_target, "ms": round(float(np.median(wall)), 3),
            "device_part_ms": round(float(np.median(flag)), 3), "layout_ms": round(float(np.median(lay)), 3),
            "refined": st["refined"], "balance_refined": st["balance_refined"], "derefined": st["derefined"],
            "n_leaves_out": st["n_leaves"], "n_grids_out": st["n_grids"], "rho_r_next": st["rho_r_next"],
            "host_build_from_field_ms": round(host_build_ms, 3)}


def c4_bench(a, lib, w, ctx):
    import torch

    mix = w.mixes.batched_mix(256)
    say("c4: building 256 uniform trees")
    trees = [ctx.uniform_tree(w.uniform_grid(b.field, b.level)) for b in mix]
    n_cells = sum(t.n_leaf_cells for t in trees)
    outs = [(torch.empty(t.n_leaf_cells, dtype=torch.float64, device=ctx.device),
             torch.empty((3, t.n_leaf_cells), dtype=torch.float64, device=ctx.device)) for t in trees]
    ptr_phi = [o[0].data_ptr() for o in outs]
    ptr_g = [o[1].data_ptr() for o in outs]
    handles = [t.handle for t in trees]

    def sync():
        ctx.stream.synchronize()
        torch.cuda.synchronize()

    res = {}
    # batch-fitted work shapes (every level below the root LDS-staged, one
    # class-group count for the batch) first, then each tree's own plan
    for mode in (1, 0):
        ctx.set_batch_shapes(mode)
        for pn, prec in (("fp64", lib.OCTO_FP64), ("mixed", lib.OCTO_MIXED)):
            opts = lib.make_opts(a.theta, 1.0, prec, True)
            sts = lib.octo_solve_batch(ctx.handle, handles, opts, ptr_phi, ptr_g, True)
            say(f"c4 shapes {mode} {pn}: batched")
            sec = timed(lambda: lib.octo_solve_batch(ctx.handle, handles, opts, ptr_phi, ptr_g, True),
                        sync, a.steps, a.warmup)
            sec_ns = timed(lambda: lib.octo_solve_batch(ctx.handle, handles, opts, ptr_phi, ptr_g, True,
                                                        want_stats=False), sync, a.steps, a.warmup)
            res[mode, pn] = dict(sec=sec, sec_ns=sec_ns, torque=max(s.as_dict()["torque"] for s in sts))
    ctx.set_batch_shapes(0)
    opts = lib.make_opts(a.theta, 1.0, lib.OCTO_FP64, True)
    say("c4 fp64: one by one")
    sec1 = timed(lambda: [lib.octo_solve(ctx.handle, h, opts, p, q, True, want_stats=False)
                          for h, p, q in zip(handles, ptr_phi, ptr_g)], sync, max(2, a.steps // 4), 1)
    for t in trees:
        t.destroy()

    def rec(sec):
        return {"value": round(n_cells / sec, 1), "ms_per_step": round(sec * 1e3, 4)}

    r = res[1, "fp64"]
    return {"workload": "256 independent uniform trees (16^3/32^3/64^3 from log-uniform [16,96]), seeded single/"
                        "binary n=1.5 polytropes R~U(0.05,0.2); one launch per phase over all trees, HIP-graph "
                        "replay, work shapes fitted to the batch", "leaf_cells": int(n_cells), "trees": 256,
            "theta": a.theta, "value": round(n_cells / r["sec"], 1), "ms_per_step": round(r["sec"] * 1e3, 4),
            "stream_ordered_no_statistics": rec(r["sec_ns"]),
            "mixed": rec(res[1, "mixed"]["sec"]),
            "own_shapes": {"note": "each tree's own single-tree plan (results bitwise as alone)",
                           **rec(res[0, "fp64"]["sec"]),
                           "stream_ordered_no_statistics": rec(res[0, "fp64"]["sec_ns"]),
                           "mixed": rec(res[0, "mixed"]["sec"])},
            "one_by_one": rec(sec1),
            "torque_max": max(r["torque"], res[0, "fp64"]["torque"])}


def c5_bench(a, lib, w):
    from paper_2101_08226_amd import serve

    ctx = lib.Context(0, hbm_budget=int(a.budget_gib * (1 << 30)))

    def count(field, lv):
        return 512 * len(lib.octo_host_adaptive_leaves(field, lv, 1e-4))

    say(f"c5: preparing {a.requests} request payloads")
    t_prep = time.perf_counter()
    stream = w.mixes.served_stream(a.requests, 1.0, count_leaves=count)
    payloads = []
    for r in stream:
        lv = lib.octo_host_adaptive_leaves(r.field, r.max_level, 1e-4)
        payloads.append(serve.Payload(r.index, r.arrival, lv, w.leaf_density(r.field, lv), r.precision, a.theta))
    t_prep = time.perf_counter() - t_prep
    # saturation: all requests present at t = 0
    sat_p = [serve.Payload(p.index, 0.0, p.leaves, p.rho, p.precision, p.theta) for p in payloads]
    say("c5: saturation run")
    rec, _, wall = serve.serve(ctx, sat_p)
    sat = serve.summary(rec, wall)
    rate = a.rate if a.rate > 0 else 0.8 * sat["throughput_req_s"]
    scale = 1.0 / rate  # the stream was drawn at rate 1: rescale arrival times
    run_p = [serve.Payload(p.index, p.arrival * scale, p.leaves, p.rho, p.precision, p.theta) for p in payloads]
    say(f"c5: served run at {rate:.1f} req/s")
    rec, _, wall = serve.serve(ctx, run_p)
    s = serve.summary(rec, wall)
    prof = dict(getattr(serve.serve, "last_profile", {}))
    # the same stream once more on the same server
    say(f"c5: repeated run at {rate:.1f} req/s")
    rec2, _, wall2 = serve.serve(ctx, run_p)
    s2 = serve.summary(rec2, wall2)
    ctx.close()
    return {"workload": f"{a.requests} Poisson requests at {rate:.1f}/s (0.8 x saturation), adaptive trees to "
                        "level 3-6 with 4k-2M leaf cells, 50/50 FP64 and mixed, HBM budget "
                        f"{a.budget_gib} GiB; the first served run after the saturation run", "requests": a.requests,
            "rate": round(rate, 2),
            "p50_ms": round(s["p50_ms"], 3), "p99_ms": round(s["p99_ms"], 3),
            "throughput_req_s": round(s["throughput_req_s"], 2), "cells_per_s": round(s["cells_per_s"], 1),
            "repeated_run": {"p50_ms": round(s2["p50_ms"], 3), "p99_ms": round(s2["p99_ms"], 3),
                             "throughput_req_s": round(s2["throughput_req_s"], 2)},
            "saturation_req_s": round(sat["throughput_req_s"], 2),
            "host": {k: round(v, 4) if isinstance(v, float) else v for k, v in prof.items()},
            "wall_s": round(wall, 3), "payload_preparation_s": round(t_prep, 2)}


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        info = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                info[k.strip()] = v.strip()
        return {"model": info.get("Model name", platform.processor()), "sockets": info.get("Socket(s)"),
                "cores_per_socket": info.get("Core(s) per socket"), "threads_per_core": info.get("Thread(s) per core"),
                "online_cpus": info.get("CPU(s)")}
    except (OSError, subprocess.SubprocessError):
        return {"model": platform.processor()}


def root_cell_sample(x, fraction, seed=210108226):
    """Leaf cells under a seeded random `fraction` of the 512 root cells
    (cells of width 1/8): the oracle's recursion runs per root cell, so such a
    sample costs about that fraction of a full solve."""
    r = np.clip(np.floor((x + 0.5) * 8.0).astype(np.int64), 0, 7)
    rid = (r[0] * 8 + r[1]) * 8 + r[2]
    chosen = np.random.default_rng(seed).permutation(512)[:max(1, int(round(512 * fraction)))]
    return np.nonzero(np.isin(rid, chosen))[0], len(chosen)


def cpu_baseline(a, otree, n_cells, desc):
    """The oracle timed on this host's cores on a bounded sample of the
    headline tree: all leaf cells under a seeded random eighth of the root
    cells with all threads (median of 5 after a warm-up), and under a
    thirty-second of them on one thread; the upward pass runs over the whole
    tree in each."""
    x, _ = otree.leaf_cells()
    res = {}
    for key, frac, threads, reps in (("all_threads", 1 / 8, a.cpu_threads, 5), ("one_thread", 1 / 32, 1, 1)):
        sel, n_roots = root_cell_sample(x, frac)
        say(f"CPU oracle: {len(sel)} cells under {n_roots} root cells, {threads} threads, {reps} runs")
        if reps > 1:
            otree.solve(theta=a.theta, sample=sel, threads=threads)
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            otree.solve(theta=a.theta, sample=sel, threads=threads)
            ts.append(time.perf_counter() - t0)
        t = float(np.median(ts))
        res[key] = {"value": round(len(sel) / t, 1), "cells": int(len(sel)), "root_cells": n_roots, "s": round(t, 3),
                    "threads": threads, "runs": reps}
    m = res["all_threads"]
    return {"value": m["value"], "unit": "cells/s", "cores": a.cpu_threads, "kind": "oracle",
            "sample": f"FP64 oracle solve of {desc} ({n_cells} cells) restricted to the {m['cells']} leaf cells "
                      f"under {m['root_cells']} of the 512 root cells (seeded random; the upward pass covers the "
                      f"whole tree), median of {m['runs']} runs after a warm-up, tree build excluded",
            "one_thread": res["one_thread"], "host": cpu_model()}


def headline(a, lib, w, ctx, out, skip):
    import oracle

    f = w.binary_polytrope_128()
    say("building the adaptive tree (level 6)")
    tb = time.perf_counter()
    tree = ctx.adaptive_tree(f, 6, 1e-4)
    host_build_ms = (time.perf_counter() - tb) * 1e3
    leaves = tree.leaves()
    rate = w.leaf_density(w.OrbitalRate(f, 1.0, 1e-3), leaves) if "dphidt" not in skip else None
    n = tree.n_leaf_cells
    desc = ("binary n=1.5 polytropes R=0.12/0.10, sep 0.35, q=0.7, max rho 1, floor 1e-10; adaptive to level 6 "
            "(root sub-grid = level 0; 7736 leaf sub-grids, 3.96M leaf cells), refined where box-max rho > 1e-4, "
            "26-neighbour 2:1 balance")
    res = single_tree(a, lib, ctx, tree, rate)
    b = block(res, n, desc, a.theta, traffic_record("c3"), leaves)
    out.update(value=b["value"], ms_per_step=b["ms_per_step"], dtype="f64")
    out["config"] = {"workload": f"{desc}; theta={a.theta}; fp64; angular-momentum correction on; one step = "
                                 "one full solve including the net force/torque reductions (left on the device)",
                     "leaf_cells": int(n), "theta": a.theta, "precision": "fp64",
                     "m2l_pairs": b["m2l_pairs"], "direct_pairs": b["direct_pairs"]}
    for k in ("with_host_statistics", "no_reductions", "torque", "force", "roofline", "mixed", "hbm_phases", "dphidt"):
        if k in b:
            out[k] = b[k]
    out["roofline"]["phase_ms"] = b["phase_ms"]
    if "regrid" not in skip:
        out["regrid"] = regrid_bench(tree, host_build_ms)
    cpu = None
    if not a.no_cpu:
        say("CPU oracle: building its tree")
        ot = oracle.Tree(leaves, w.leaf_density(f, leaves))
        cpu = cpu_baseline(a, ot, n, "the headline tree")
        del ot
    tree.destroy()
    return cpu


def level7(a, lib, w, ctx):
    f = w.binary_polytrope_128()
    say("building the adaptive tree (level 7)")
    tree = ctx.adaptive_tree(f, 7, 1e-4)
    res = single_tree(a, lib, ctx, tree, with_dphidt=False, stats_steps=max(3, a.steps // 2))
    n = tree.n_leaf_cells
    b = block(res, n, "the headline field adaptive to level 7 (paper numbering with the root at level 0; "
                      f"{len(tree.leaves())} leaf sub-grids)", a.theta)
    tree.destroy()
    return b


def c2(a, lib, w, ctx, skip):
    rho = w.uniform_grid(w.binary_polytrope_128(), 4)
    rate = w.uniform_grid(w.OrbitalRate(w.binary_polytrope_128(), 1.0, 1e-3), 4) if "dphidt" not in skip else None
    tree = ctx.uniform_tree(rho)
    res = single_tree(a, lib, ctx, tree, rate)
    b = block(res, tree.n_leaf_cells, "uniform 128^3 (16^3 sub-grids) of the headline field", a.theta,
              traffic_record("c2"), w.uniform_leaves(4))
    tree.destroy()
    if "scf" not in skip:
        b["scf"] = scf_bench(a, lib, w, ctx, a.scf_level, a.scf_iters)
    return b


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {a.gpus}); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch

    if a.copy_probe:
        n = a.copy_probe // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(max(1, a.steps)):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 8, "copies": max(1, a.steps)}))
        return

    import paper_2101_08226_amd as lib
    import workloads as w

    skip = set(s for s in a.skip.split(",") if s)
    out = {"metric": METRIC, "value": None, "unit": "cells/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic"}
    cpu = None
    t_start = time.perf_counter()
    if a.config in ("all", "c3"):
        ctx = lib.Context(0)
        cpu = headline(a, lib, w, ctx, out, skip)
        if a.config == "all":
            if "c3l7" not in skip:
                out["c3_level7"] = level7(a, lib, w, ctx)
            if "c2" not in skip:
                out["c2"] = c2(a, lib, w, ctx, skip)
            if "c4" not in skip:
                out["c4"] = c4_bench(a, lib, w, ctx)
        ctx.close()
        if a.config == "all" and "c5" not in skip:
            out["c5"] = c5_bench(a, lib, w)
    elif a.config == "c3l7":
        ctx = lib.Context(0)
        b = level7(a, lib, w, ctx)
        ctx.close()
        out.update(value=b["value"], ms_per_step=b["ms_per_step"], config={"workload": b["workload"]}, c3_level7=b)
    elif a.config in ("c1", "c2"):
        ctx = lib.Context(0)
        if a.config == "c1":
            rho = w.noisy_sphere_16()
            tree = ctx.uniform_tree(rho)
            res = single_tree(a, lib, ctx, tree, w.noisy_rate(rho, 1))
            b = block(res, tree.n_leaf_cells, "uniform 16^3 (2^3 sub-grids), noisy sphere rho=1(1+0.01N) "
                                              "inside r=0.4, floor 1e-10", a.theta)
            tree.destroy()
        else:
            b = c2(a, lib, w, ctx, skip | {"scf"})
        ctx.close()
        out.update(value=b["value"], ms_per_step=b["ms_per_step"], config={"workload": b["workload"]})
        out.update({k: b[k] for k in ("roofline", "mixed", "torque", "force") if k in b})
    elif a.config == "c4":
        ctx = lib.Context(0)
        b = c4_bench(a, lib, w, ctx)
        ctx.close()
        out.update(value=b["value"], ms_per_step=b["ms_per_step"], config={"workload": b["workload"]}, c4=b,
                   roofline=None)
    else:
        b = c5_bench(a, lib, w)
        out.update(value=b["cells_per_s"], ms_per_step=round(1e3 * b["wall_s"] / b["requests"], 4),
                   config={"workload": b["workload"]}, c5=b, roofline=None, dtype="f64/f32+f64")
    out["cpu_baseline"] = cpu
    out["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
