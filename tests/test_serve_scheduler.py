"""Scheduler of the continuous-batching server against a fake backend (CPU only):
admission by memory footprint, FIFO order, concurrency limits, rejection and failure."""

import threading
import time

import pytest

from paper_1904_00182_amd.serve import Request, Scheduler, summarize


class FakeBackend:
    def __init__(self, cost, footprint, fail_ids=(), unconverged_ids=()):
        self.cost = cost
        self.fp = footprint
        self.fail = set(fail_ids)
        self.unconverged = set(unconverged_ids)
        self.lock = threading.Lock()
        self.running = 0
        self.max_running = 0
        self.mem = 0
        self.max_mem = 0
        self.order = []

    def footprint(self, r):
        return self.fp(r)

    def run(self, r, slot):
        with self.lock:
            self.running += 1
            self.mem += self.fp(r)
            self.max_running = max(self.max_running, self.running)
            self.max_mem = max(self.max_mem, self.mem)
            self.order.append(r.id)
        time.sleep(self.cost(r))
        with self.lock:
            self.running -= 1
            self.mem -= self.fp(r)
        if r.id in self.fail:
            raise RuntimeError("forced failure")
        if r.id in self.unconverged:
            return {"slot": slot, "status": "not converged"}
        return {"slot": slot}


def reqs(n, gap, grids=((16, 8, 16),)):
    return [Request(i, i * gap, grids[i % len(grids)], 1e3, 1.0, 1000 + i) for i in range(n)]


def test_concurrency_and_memory_cap_respected():
    be = FakeBackend(cost=lambda r: 0.02, footprint=lambda r: 3)
    sch = Scheduler(be, slots=4, mem_cap=10)
    out = sch.serve(reqs(20, 0.0))
    assert all(r.status == "done" for r in out)
    assert be.max_running <= 3          # 3 x 3 <= 10 < 4 x 3
    assert be.max_mem <= 10
    assert be.max_running >= 2          # work overlapped


def test_arrivals_are_admitted_while_others_run():
    be = FakeBackend(cost=lambda r: 0.05, footprint=lambda r: 1)
    sch = Scheduler(be, slots=4, mem_cap=100)
    out = sch.serve(reqs(8, 0.01))
    # request 1 arrives while request 0 is still running and is admitted at once
    assert out[1].admit < out[0].finish
    assert max(r.admit - r.arrival for r in out) < 0.03
    s = summarize(out, max(r.finish for r in out))
    assert s["completed"] == 8 and s["p99_s"] >= s["p50_s"] > 0


def test_fifo_order_and_rejection_and_failure():
    fp = {0: 6, 1: 6, 2: 2, 3: 50, 4: 1}
    be = FakeBackend(cost=lambda r: 0.02, footprint=lambda r: fp[r.id], fail_ids={4})
    sch = Scheduler(be, slots=4, mem_cap=10)
    out = sch.serve(reqs(5, 0.0))
    assert out[3].status.startswith("rejected")
    assert out[4].status.startswith("failed")
    assert [r.status for r in out[:3]] == ["done"] * 3
    # FIFO: request 2 (small) does not overtake request 1 (waiting for memory)
    assert out[2].admit >= out[1].admit
    assert be.order[:3] == [0, 1, 2]


def test_single_slot_is_serial():
    be = FakeBackend(cost=lambda r: 0.01, footprint=lambda r: 1)
    out = Scheduler(be, slots=1, mem_cap=100).serve(reqs(6, 0.0))
    assert be.max_running == 1
    fin = sorted(r.finish for r in out)
    assert fin == [r.finish for r in out]


def test_unconverged_requests_are_not_counted_as_completed():
    """A request whose solve did not converge finishes (its slot and memory are released)
    but counts neither as a completed solve nor in the latency percentiles."""
    be = FakeBackend(cost=lambda r: 0.01 if r.id != 2 else 0.2, footprint=lambda r: 1, unconverged_ids={2})
    out = Scheduler(be, slots=2, mem_cap=100).serve(reqs(6, 0.0))
    assert out[2].status == "not converged" and out[2].finish is not None
    s = summarize(out, max(r.finish for r in out))
    assert s["completed"] == 5 and s["not_converged"] == 1
    assert s["p99_s"] < 0.2          # the slow unconverged request is not in the percentiles
