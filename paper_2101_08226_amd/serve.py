"""Request server: solves of differently sized octrees arriving over time.

Each request carries its tree (leaf list and leaf-cell densities, prepared by
the client).  The server admits requests in arrival order while the context's
HBM budget holds their trees (octo_tree_build fails with OCTO_E_BUDGET when it
does not), submits them with octo_submit -- the library merges requests that
are pending while earlier ones run into its next launch wave (continuous
batching) -- polls for completions, releases finished trees, and records the
latency from arrival to result.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import (OCTO_E_BUDGET, Context, OctoError, Tree, make_opts, octo_poll, octo_submit, octo_tree_build,
               octo_wait)


@dataclass
class Payload:
    index: int
    arrival: float       # seconds after stream start
    leaves: np.ndarray   # (n, 4) int32
    rho: np.ndarray      # (n, 512) float64
    precision: int = 0
    theta: float = 0.5


@dataclass
class Record:
    index: int
    arrival: float
    admitted: float
    done: float
    cells: int
    precision: int
    stats: dict = field(default_factory=dict)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def serve(ctx: Context, payloads: List[Payload], keep_outputs: bool = False, poll_sleep: float = 2e-4,
          time_limit: Optional[float] = None):
    """Run the stream in real time; returns (records, outputs by index if
    keep_outputs, wall seconds)."""
    import torch

    pending = sorted(payloads, key=lambda p: p.arrival)
    nxt = 0
    queue: List[Payload] = []
    inflight = {}  # ticket -> (payload, tree, phi, g, admitted)
    records: List[Record] = []
    outputs = {}
    t0 = time.perf_counter()
    while nxt < len(pending) or queue or inflight:
        now = time.perf_counter() - t0
        if time_limit is not None and now > time_limit:
            raise TimeoutError(f"serving exceeded {time_limit} s")
        while nxt < len(pending) and pending[nxt].arrival <= now:
            queue.append(pending[nxt])
            nxt += 1
        # admission in arrival order while the budget holds
        while queue:
            p = queue[0]
            try:
                h = octo_tree_build(ctx.handle, p.leaves, p.rho.ctypes.data, False)
            except OctoError as e:
                if e.status == OCTO_E_BUDGET and inflight:
                    break  # wait for completions to free memory
                raise
            tree = Tree(ctx, h)
            phi = torch.empty(tree.n_leaf_cells, dtype=torch.float64, device=ctx.device)
            g = torch.empty((3, tree.n_leaf_cells), dtype=torch.float64, device=ctx.device)
            tk = octo_submit(ctx.handle, h, make_opts(p.theta, 1.0, p.precision, True), phi.data_ptr(), g.data_ptr())
            inflight[tk] = (p, tree, phi, g, time.perf_counter() - t0)
            queue.pop(0)
        # completions
        progressed = False
        for tk in list(inflight):
            if octo_poll(ctx.handle, tk):
                st = octo_wait(ctx.handle, tk).as_dict()
                p, tree, phi, g, adm = inflight.pop(tk)
                done = time.perf_counter() - t0
                records.append(Record(p.index, p.arrival, adm, done, tree.n_leaf_cells, p.precision, st))
                if keep_outputs:
                    outputs[p.index] = (phi.cpu().numpy(), g.cpu().numpy())
                tree.destroy()
                progressed = True
        if not progressed and (not queue or inflight):
            wait = poll_sleep
            if not inflight and not queue and nxt < len(pending):
                wait = max(0.0, pending[nxt].arrival - (time.perf_counter() - t0))
            time.sleep(min(wait, 0.01))
    wall = time.perf_counter() - t0
    return records, outputs, wall


def summary(records: List[Record], wall: float) -> dict:
    lat = np.array([r.latency for r in records]) * 1e3
    cells = sum(r.cells for r in records)
    return dict(requests=len(records), p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                mean_ms=float(lat.mean()), throughput_req_s=len(records) / wall, cells_per_s=cells / wall,
                wall_s=wall)
