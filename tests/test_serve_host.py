"""Request-server admission logic on the host, against a stand-in library
with an HBM budget (no device): tree builds that fail against memory held by
a request that has since completed are retried, trees built ahead are
released when the head of the queue cannot fit, and every request completes
in arrival order of admission."""
import threading
import time

import numpy as np
import pytest

import paper_2101_08226_amd as lib
from paper_2101_08226_amd import serve


class FakeLib:
    """Budgeted trees and tickets: a build takes `tree_bytes` at once (or
    fails with OCTO_E_BUDGET) and then spends `build_s` of host work; a
    ticket completes `solve_s` after submission."""

    def __init__(self, budget, tree_bytes, build_s, solve_s):
        self.budget, self.tree_bytes, self.build_s, self.solve_s = budget, tree_bytes, build_s, solve_s
        self.mu = threading.Lock()
        self.in_use = 0
        self.next = 1
        self.alive = set()
        self.tickets = {}
        self.failed_builds = 0
        self.peak = 0

    def build(self, ctx, leaves, rho_ptr, on_device):
        with self.mu:
            ok = self.in_use + self.tree_bytes <= self.budget
            if ok:
                h = self.next
                self.next += 1
                self.alive.add(h)
                self.in_use += self.tree_bytes
                self.peak = max(self.peak, self.in_use)
            else:
                self.failed_builds += 1
        time.sleep(self.build_s)
        if not ok:
            raise lib.OctoError(lib.OCTO_E_BUDGET, "HBM budget exceeded")
        return h

    def destroy(self, h):
        with self.mu:
            self.alive.remove(h)
            self.in_use -= self.tree_bytes

    def submit(self, ctx, h, opts, phi, g):
        with self.mu:
            tk = self.next
            self.next += 1
            self.tickets[tk] = time.perf_counter() + self.solve_s
        return tk

    def poll(self, ctx, tk):
        return time.perf_counter() >= self.tickets[tk]

    def wait(self, ctx, tk):
        while time.perf_counter() < self.tickets[tk]:
            time.sleep(1e-4)
        del self.tickets[tk]

        class St:
            def as_dict(self):
                return {}

        return St()


class FakeCtx:
    handle = 0
    device = "cpu"


def _install(monkeypatch, fake):
    class FakeTree:
        def __init__(self, ctx, h):
            self.handle = h
            self.n_leaf_cells = 512

        def destroy(self):
            fake.destroy(self.handle)

    monkeypatch.setattr(serve, "octo_tree_build", fake.build)
    monkeypatch.setattr(serve, "octo_tree_destroy", fake.destroy)
    monkeypatch.setattr(serve, "octo_submit", fake.submit)
    monkeypatch.setattr(serve, "octo_poll", fake.poll)
    monkeypatch.setattr(serve, "octo_wait", fake.wait)
    monkeypatch.setattr(serve, "Tree", FakeTree)


def _payloads(n, gap):
    lv = np.zeros((1, 4), dtype=np.int32)
    rho = np.zeros((1, 512))
    return [serve.Payload(i, i * gap, lv, rho) for i in range(n)]


@pytest.mark.parametrize("builders,lookahead", [(1, 1), (2, 4), (4, 6)])
def test_build_failing_against_completed_request_is_retried(monkeypatch, builders, lookahead):
    """One tree fits at a time; builds are slow next to the solves, so a
    build started while a request was in flight fails against its tree and
    is only seen after that request completed: the server retries it
    instead of giving up."""
    fake = FakeLib(budget=150, tree_bytes=100, build_s=0.02, solve_s=0.005)
    _install(monkeypatch, fake)
    recs, _, _ = serve.serve(FakeCtx(), _payloads(6, 0.0), builders=builders, lookahead=lookahead,
                             time_limit=20.0)
    assert sorted(r.index for r in recs) == list(range(6))
    assert fake.peak <= fake.budget
    assert not fake.alive and not fake.tickets


def test_lookahead_released_for_the_head(monkeypatch):
    """Two trees fit; trees built ahead for later requests give way when the
    head of the queue cannot be built with nothing in flight."""
    fake = FakeLib(budget=250, tree_bytes=100, build_s=0.002, solve_s=0.01)
    _install(monkeypatch, fake)
    recs, _, _ = serve.serve(FakeCtx(), _payloads(12, 0.001), builders=4, lookahead=8, time_limit=20.0)
    assert sorted(r.index for r in recs) == list(range(12))
    assert fake.peak <= fake.budget
    assert not fake.alive


def test_tree_larger_than_budget_raises(monkeypatch):
    """A tree that cannot fit even alone ends the run with OCTO_E_BUDGET."""
    fake = FakeLib(budget=50, tree_bytes=100, build_s=0.001, solve_s=0.001)
    _install(monkeypatch, fake)
    with pytest.raises(lib.OctoError) as e:
        serve.serve(FakeCtx(), _payloads(2, 0.0), builders=2, lookahead=2, time_limit=20.0)
    assert e.value.status == lib.OCTO_E_BUDGET
