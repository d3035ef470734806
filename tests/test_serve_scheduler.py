"""CPU tests of the serving scheduler with a fake executor (admission by slots and
HBM budget, FIFO order without starvation, error isolation, overlap)."""
import dataclasses

import pytest

from paper_2601_08374_amd.serve import Scheduler, summarize


@dataclasses.dataclass
class Req:
    rid: int
    arrival: float
    size: int          # bytes
    work: int          # steps to finish
    bad: bool = False


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 0.001
        return self.t


class FakeExec:
    def __init__(self, budget):
        self.budget = budget
        self.used = 0
        self.max_used = 0
        self.started = []
        self.live = {}
        self.concurrent = 0

    def bytes_required(self, r):
        if r.bad:
            raise ValueError("invalid request")
        return r.size

    def start(self, r, slot):
        self.used += r.size
        assert self.used <= self.budget
        self.max_used = max(self.max_used, self.used)
        self.started.append(r.rid)
        h = {"r": r, "left": r.work}
        self.live[r.rid] = h
        self.concurrent = max(self.concurrent, len(self.live))
        return h

    def step(self, h, n):
        h["left"] -= n

    def poll(self, h):
        return h["left"] <= 0, 0

    def finish(self, h):
        return {"iters": h["r"].work}

    def release(self, h):
        self.used -= h["r"].size
        del self.live[h["r"].rid]


def test_fifo_budget_and_slots():
    reqs = [Req(i, 0.0005 * i, size=(i % 5 + 1) * 10, work=(i % 7) + 1) for i in range(60)]
    ex = FakeExec(budget=100)
    s = Scheduler(ex, slots=4, budget_bytes=100, iters_per_step=1, clock=FakeClock())
    recs = s.run(reqs)
    assert all(r.status == 0 for r in recs)
    assert ex.started == sorted(ex.started)              # admitted in arrival order
    assert ex.max_used <= 100 and ex.concurrent <= 4
    assert ex.concurrent > 1                              # solves overlap
    adm = [r.admitted for r in recs]
    assert adm == sorted(adm)
    for r in recs:
        assert r.arrival <= r.admitted <= r.finished


def test_large_request_blocks_later_ones_but_is_served():
    # request 1 needs the whole budget: later small requests must wait (no overtaking),
    # and request 1 is served once the earlier one completes (no starvation)
    reqs = [Req(0, 0.0, 60, 20), Req(1, 0.0001, 100, 3)] + [Req(i, 0.0002, 10, 1) for i in range(2, 8)]
    ex = FakeExec(budget=100)
    s = Scheduler(ex, slots=8, budget_bytes=100, iters_per_step=1, clock=FakeClock())
    recs = s.run(reqs)
    assert ex.started == list(range(8))
    assert recs[1].admitted >= recs[0].finished
    assert min(r.admitted for r in recs[2:]) >= recs[1].admitted


def test_invalid_and_oversized_requests_do_not_poison_neighbours():
    reqs = [Req(0, 0.0, 10, 2), Req(1, 0.0, 10, 2, bad=True), Req(2, 0.0, 1000, 2), Req(3, 0.0, 10, 2)]
    ex = FakeExec(budget=100)
    s = Scheduler(ex, slots=2, budget_bytes=100, iters_per_step=1, clock=FakeClock())
    recs = s.run(reqs)
    assert recs[0].status == 0 and recs[3].status == 0
    assert recs[1].status == -1 and "invalid" in recs[1].error
    assert recs[2].status == -2
    summ = summarize(recs)
    assert summ["solves"] == 2 and summ["failed"] == 2
