"""Seeded workload mixes: many independent trees (batched) and a Poisson
stream of solve requests (served).  Input generation only."""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List

import numpy as np

from .fields import Polytropes, Star, binary_polytrope, single_polytrope

SEED = 210108226


def random_polytrope_field(rng: np.random.Generator) -> Polytropes:
    """A single (p = 0.5) or binary n = 3/2 polytrope with radii U(0.05, 0.2);
    binaries have mass ratio U(0.3, 1) and separation (R1 + R2) U(1.05, 1.5),
    centre of mass at the origin, both stars inside the box; max density 1."""
    while True:
        if rng.uniform() < 0.5:
            r = float(rng.uniform(0.05, 0.2))
            return single_polytrope(r)
        r1, r2 = (float(v) for v in rng.uniform(0.05, 0.2, 2))
        q = float(rng.uniform(0.3, 1.0))
        sep = (r1 + r2) * float(rng.uniform(1.05, 1.5))
        f = binary_polytrope(r1, r2, sep, q)
        s1, s2 = f.stars
        if s1.centre[0] - s1.radius > -0.5 and s2.centre[0] + s2.radius < 0.5:
            return f


@dataclass
class BatchTree:
    index: int
    level: int  # uniform tree level: n = 8 * 2^level cells per axis
    field: Polytropes


def batched_mix(count: int = 256, seed0: int = SEED) -> List[BatchTree]:
    """Uniform trees with n drawn log-uniform on [16, 96] and snapped to the
    nearest octree size 8 * 2^k in {16, 32, 64} (log2 distance)."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        n = math.exp(rng.uniform(math.log(16.0), math.log(96.0)))
        k = int(min(3, max(1, round(math.log2(n / 8.0)))))
        out.append(BatchTree(i, k, random_polytrope_field(rng)))
    return out


@dataclass
class ServedRequest:
    index: int
    arrival: float      # seconds after the start of the stream
    max_level: int      # adaptive tree depth (root sub-grid = level 0)
    field: Polytropes
    precision: int      # 0 = FP64, 1 = mixed


def served_stream(count: int, rate: float, seed: int = SEED, count_leaves=None,
                  min_cells: int = 4096, max_cells: int = 1 << 21) -> List[ServedRequest]:
    """Poisson arrivals at `rate` per second; depth drawn from {3, 4, 5, 6}
    (paper numbering 4-7 with the root at level 1), star parameters as in the
    batched mix, resampled until the leaf-cell count lies in [min_cells,
    max_cells] (count_leaves(field, max_level) -> cells); half the requests in
    mixed precision."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        while True:
            lv = int(rng.choice([3, 4, 5, 6]))
            f = random_polytrope_field(rng)
            if count_leaves is None:
                break
            c = count_leaves(f, lv)
            if min_cells <= c <= max_cells:
                break
        out.append(ServedRequest(i, t, lv, f, int(rng.uniform() < 0.5)))
    return out
