"""Request server: solves of differently sized octrees arriving over time.

Each request carries its tree (leaf list and leaf-cell densities, prepared by
the client).  The server builds the trees of arrived requests on a pool of
host threads (the library validates and lays out a tree before taking the
context's lock, so builds run in parallel), admits them in arrival order
while the context's HBM budget holds their trees (a build fails with
OCTO_E_BUDGET when it does not), submits them with octo_submit -- the library
merges requests that are pending while earlier ones run into its next launch
wave (continuous batching) -- polls for completions, releases finished trees,
and records the latency from arrival to result.
"""
from __future__ import annotations

import gc
import time
from collections import deque
from concurrent.futures import Future, ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import (OCTO_E_BUDGET, Context, OctoError, Tree, make_opts, octo_poll, octo_submit, octo_tree_build,
               octo_tree_destroy, octo_wait)


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


class _Slot:
    """A queued request and its tree build (a future of a tree handle);
    `frees` counts the trees the server had released when the build was
    started."""

    def __init__(self, p: Payload):
        self.p = p
        self.build = None
        self.frees = 0


def serve(ctx: Context, payloads: List[Payload], keep_outputs: bool = False, poll_sleep: float = 2e-4,
          time_limit: Optional[float] = None, builders: int = 12, lookahead: int = 24):
    """Run the stream in real time; returns (records, outputs by index if
    keep_outputs, wall seconds).  `builders` host threads build the trees of
    up to `lookahead` queued requests ahead of admission.  Host time spent in
    builds, admission, completions and idle waits is left in
    serve.last_profile."""
    import torch

    prof = dict(build_s=0.0, builds=0, admit_s=0.0, complete_s=0.0, idle_s=0.0, loops=0)
    frees = [0]  # trees released so far (completed requests and builds given up)

    def release_lookahead(queue) -> bool:
        """Destroy the trees built ahead for queued requests after the head
        of the queue (they are rebuilt later); True when any was freed."""
        freed = False
        for later in list(queue)[1:]:
            if later.build is not None:
                try:
                    octo_tree_destroy(later.build.result())
                    freed = True
                    frees[0] += 1
                except OctoError:
                    pass
                later.build = None
        return freed

    def build(p: Payload) -> int:
        b0 = time.perf_counter()
        try:
            return octo_tree_build(ctx.handle, p.leaves, p.rho.ctypes.data, False)
        finally:
            prof["build_s"] += time.perf_counter() - b0  # float += under the GIL
            prof["builds"] += 1

    pending = sorted(payloads, key=lambda p: p.arrival)
    nxt = 0
    queue: deque = deque()
    inflight = {}  # ticket -> (payload, tree, phi, g, admitted)
    records: List[Record] = []
    outputs = {}
    pool = ThreadPoolExecutor(max_workers=max(1, builders))
    # Objects alive before the run (the payloads, the caller's state) are
    # moved out of the collector's generations for its duration: a full
    # collection scanning them holds the interpreter lock for tens of
    # milliseconds, and every thread that calls into Python (the device
    # allocator's callbacks in the builders, the admission loop) waits for it.
    gc.collect()
    gc.freeze()
    t0 = time.perf_counter()
    try:
        while nxt < len(pending) or queue or inflight:
            now = time.perf_counter() - t0
            if time_limit is not None and now > time_limit:
                raise TimeoutError(f"serving exceeded {time_limit} s")
            while nxt < len(pending) and pending[nxt].arrival <= now:
                queue.append(_Slot(pending[nxt]))
                nxt += 1
            for k, slot in enumerate(queue):
                if k >= lookahead:
                    break
                if slot.build is None:
                    slot.frees = frees[0]
                    slot.build = pool.submit(build, slot.p)
            progressed = False
            prof["loops"] += 1
            a0 = time.perf_counter()
            # admission in arrival order
            while queue and queue[0].build is not None and queue[0].build.done():
                slot = queue[0]
                try:
                    h = slot.build.result()
                except OctoError as e:
                    if e.status != OCTO_E_BUDGET:
                        raise
                    if inflight:
                        slot.build = None  # retry once completions free memory
                        break
                    # nothing on the device: release trees built ahead so the
                    # head of the queue fits, then retry it; also retry when
                    # trees were released while the build ran (it may have
                    # failed against memory that is free now)
                    if not release_lookahead(queue) and frees[0] == slot.frees:
                        raise
                    slot.build = None
                    break
                p = slot.p
                tree = Tree(ctx, h)
                phi = torch.empty(tree.n_leaf_cells, dtype=torch.float64, device=ctx.device)
                g = torch.empty((3, tree.n_leaf_cells), dtype=torch.float64, device=ctx.device)
                try:
                    tk = octo_submit(ctx.handle, h, make_opts(p.theta, 1.0, p.precision, True), phi.data_ptr(),
                                     g.data_ptr())
                except OctoError as e:
                    if e.status != OCTO_E_BUDGET:
                        raise
                    break  # not admitted yet: the head stays queued with its tree
                inflight[tk] = (p, tree, phi, g, time.perf_counter() - t0)
                queue.popleft()
                progressed = True
            a1 = time.perf_counter()
            prof["admit_s"] += a1 - a0
            # completions: requests finish with their launch wave and waves
            # retire in submission order, so stop at the first unfinished one
            for tk in list(inflight):
                try:
                    if not octo_poll(ctx.handle, tk):
                        break
                    st = octo_wait(ctx.handle, tk).as_dict()
                except OctoError as e:
                    if e.status != OCTO_E_BUDGET:
                        raise
                    # its work plan did not fit with nothing else in flight:
                    # free the trees built ahead and queue it again first
                    try:
                        octo_wait(ctx.handle, tk)
                    except OctoError:
                        pass  # the failed ticket is gone now
                    p, tree, phi, g, adm = inflight.pop(tk)
                    if not release_lookahead(queue) and not inflight:
                        tree.destroy()
                        raise  # nothing else holds memory that could be freed
                    again = _Slot(p)
                    again.build = Future()
                    again.build.set_result(tree.handle)
                    queue.appendleft(again)
                    progressed = True
                    continue
                p, tree, phi, g, adm = inflight.pop(tk)
                done = time.perf_counter() - t0
                records.append(Record(p.index, p.arrival, adm, done, tree.n_leaf_cells, p.precision, st))
                if keep_outputs:
                    outputs[p.index] = (phi.cpu().numpy(), g.cpu().numpy())
                tree.destroy()
                frees[0] += 1
                progressed = True
            prof["complete_s"] += time.perf_counter() - a1
            if not progressed:
                wait = poll_sleep
                if not inflight and not queue and nxt < len(pending):
                    wait = max(0.0, pending[nxt].arrival - (time.perf_counter() - t0))
                i0 = time.perf_counter()
                time.sleep(min(wait, 0.01))
                prof["idle_s"] += time.perf_counter() - i0
    finally:
        # trees built for requests that were never admitted
        for slot in queue:
            if slot.build is not None:
                try:
                    octo_tree_destroy(slot.build.result())
                except OctoError:
                    pass
        pool.shutdown(wait=True)
        gc.unfreeze()
    wall = time.perf_counter() - t0
    serve.last_profile = prof
    return records, outputs, wall


def summary(records: List[Record], wall: float) -> dict:
    lat = np.array([r.latency for r in records]) * 1e3
    cells = sum(r.cells for r in records)
    return dict(requests=len(records), p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                mean_ms=float(lat.mean()), throughput_req_s=len(records) / wall, cells_per_s=cells / wall,
                wall_s=wall)
