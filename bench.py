"""Benchmark: FMM leaf cells solved per second on one MI355X.

Workload (default): uniform 128^3 grid (16^3 sub-grids of 8^3 cells, levels
0-4) holding two n = 3/2 polytropes (radii 0.12 and 0.10, centres 0.35 apart,
mass ratio 0.7, maximum density 1, floor 1e-10), theta = 0.5, FP64 with the
angular-momentum correction.  One step = one full solve (P2M, M2M, M2L with
the correction, L2L, leaf near field and L2P, statistics) with the tree and
density already resident in HBM.

Prints one JSON line with the throughput, the roofline position of the
dominant kernel (the multipole-to-local interactions), and the CPU oracle timed
on this host.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FMM cells solved/s (FP64 vs mixed, 1 GPU); p50/p99 served solve latency"

# Algorithmic FP64 operations per ordered multipole-to-local pair with an
# interior target and the correction on (adds, multiplies and rsqrt counted
# as one each, a fused multiply-add as two), counted from the operator as
# implemented: see the kernel accounting in the design notes.
M2L_FLOPS_PER_PAIR = 298
# Near field: 4 fused multiply-adds per leaf pair with tabulated weights.
NEAR_FLOPS_PER_PAIR = 8
PEAK_FP64_TFLOPS = 78.6  # MI355X FP64 vector (= FP64 matrix)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-threads", type=int, default=int(os.environ.get("OMP_NUM_THREADS", "16") or 16))
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {a.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2101_08226_amd as lib
    import workloads as w

    prec = lib.OCTO_FP64 if a.precision == "fp64" else lib.OCTO_MIXED
    field = w.binary_polytrope_128()
    rho = w.uniform_grid(field, 4)
    n_cells = rho.size
    ctx = lib.Context(0)
    tree = ctx.uniform_tree(rho)
    dev = torch.device("cuda", 0)
    phi = torch.empty(n_cells, dtype=torch.float64, device=dev)
    g = torch.empty((3, n_cells), dtype=torch.float64, device=dev)
    opts = lib.make_opts(a.theta, 1.0, prec, True)

    def step():
        lib.octo_solve(ctx.handle, tree.handle, opts, phi.data_ptr(), g.data_ptr(), True, want_stats=False)

    # correctness stats of this exact configuration (one solve with statistics)
    st = lib.octo_solve(ctx.handle, tree.handle, opts, phi.data_ptr(), g.data_ptr(), True).as_dict()
    print(f"[bench] warmup {a.warmup}", file=sys.stderr, flush=True)
    for _ in range(a.warmup):
        step()
    ctx.stream.synchronize()
    torch.cuda.synchronize()
    print(f"[bench] timing {a.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
    ctx.stream.synchronize()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1e3 * dt / a.steps
    value = n_cells / (dt / a.steps)

    # per-phase device times with HIP events on the library's stream
    ctx.set_profiling(True)
    phases = np.zeros(6)
    n_prof = max(3, min(a.steps, 10))
    for _ in range(n_prof):
        s = lib.octo_solve(ctx.handle, tree.handle, opts, phi.data_ptr(), g.data_ptr(), True)
        phases += np.array(s.phase_ms[:])
    phases /= n_prof
    ctx.set_profiling(False)
    m2l_ms = phases[2]
    achieved = st["m2l_pairs"] * M2L_FLOPS_PER_PAIR / (m2l_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": None,
                "kernel": "k_m2l", "kernel_ms": round(m2l_ms, 4),
                "phase_ms": {k: round(v, 4) for k, v in zip(["p2m", "m2m", "m2l", "l2l", "leaf", "stats"], phases)}}

    cpu = None
    if not a.no_cpu:
        import oracle

        print(f"[bench] CPU oracle, {a.cpu_threads} threads", file=sys.stderr, flush=True)
        t = oracle.Tree(w.uniform_leaves(4), w.grid_to_leaves(rho))
        t0 = time.perf_counter()
        t.solve(theta=a.theta, threads=a.cpu_threads)
        ct = time.perf_counter() - t0
        cpu = {"value": round(n_cells / ct, 1), "unit": "cells/s", "cores": a.cpu_threads, "kind": "oracle",
               "sample": f"one full FP64 oracle solve of the same 128^3 tree ({ct:.1f} s, tree build excluded)"}

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "cells/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == lib.OCTO_FP64 else "f32+f64", "data": "synthetic",
        "config": {"workload": "uniform 128^3 (16^3 sub-grids), binary n=1.5 polytropes R=0.12/0.10, sep 0.35, "
                               f"q=0.7; theta={a.theta}; {a.precision}; angular-momentum correction on",
                   "leaf_cells": int(n_cells), "theta": a.theta, "precision": a.precision,
                   "m2l_pairs": int(st["m2l_pairs"]), "direct_pairs": int(st["direct_pairs"])},
        "torque": st["torque"], "force": st["force"],
        "roofline": roofline, "cpu_baseline": cpu,
    }
    tree.destroy()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
