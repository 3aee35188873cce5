"""The serving scheduler's policy on the CPU: a fake clock and a fake executor
(durations and footprints chosen by the test) stand in for the GPU."""
import numpy as np
import pytest

from paper_2504_14497_amd.serving import (CANCELLED, DONE, QUEUED, REFUSED, RUNNING, Arena, Request, Server,
                                          latency_summary, poisson_arrivals, run_arrivals)


class FakeClock:
    def __init__(self, step=0.0):
        self.t = 0.0
        self.step = step  # advance on every read (drives busy loops)

    def __call__(self):
        self.t += self.step
        return self.t


class FakeExecutor:
    """footprint = sum of per-layer bytes + 1 KiB; a batch takes
    `per_request` seconds per request; launches are recorded."""

    def __init__(self, clock, layer_bytes, per_request=1.0):
        self.clock = clock
        self.layer_bytes = layer_bytes
        self.per_request = per_request
        self.launches = []

    def footprint(self, layers):
        return sum(self.layer_bytes[x] for x in layers) + 1024

    def launch(self, slot, reqs, offset, nbytes):
        self.launches.append((slot, [r.rid for r in reqs], offset, nbytes))
        return self.clock.t + self.per_request * len(reqs)

    def done(self, handle):
        return self.clock.t >= handle


def _reqs(n, layer=0, t=0.0):
    return [Request(rid=k, layer=layer, arrival=t) for k in range(n)]


def test_arena_first_fit():
    a = Arena(4096)
    assert [a.alloc(1000), a.alloc(1000), a.alloc(1000)] == [0, 1024, 2048]
    assert a.find(1100) is None and a.find(1024) == 3072
    a.free(1024)
    assert a.find(1024) == 1024 and a.find(1025) is None
    assert a.in_use == 2048
    with pytest.raises(KeyError):
        a.free(512)


def test_fifo_batches_and_completion():
    clk = FakeClock()
    ex = FakeExecutor(clk, {0: 1 << 20})
    srv = Server(ex, budget=1 << 30, slots=2, max_batch=4, clock=clk)
    rs = _reqs(10)
    for r in rs:
        assert srv.submit(r)
    srv.poll()
    assert [l[1] for l in ex.launches] == [[0, 1, 2, 3], [4, 5, 6, 7]]
    assert [r.state for r in rs[:8]] == [RUNNING] * 8 and rs[8].state == QUEUED
    clk.t = 4.0
    done = srv.poll()
    assert sorted(r.rid for r in done) == list(range(8))
    assert ex.launches[-1][1] == [8, 9]
    clk.t = 10.0
    srv.poll()
    assert srv.idle and all(r.state == DONE for r in rs)
    assert all(r.t_done >= r.t_admit >= r.arrival for r in rs)


def test_admission_by_table_footprint_without_overtaking():
    clk = FakeClock()
    # layer 0 needs 300 KiB, layer 1 needs 3 MiB; the budget holds ~3.2 MiB
    ex = FakeExecutor(clk, {0: 300 << 10, 1: 3 << 20})
    srv = Server(ex, budget=(3 << 20) + (300 << 10), slots=2, max_batch=64, clock=clk)
    order = [0, 0, 1, 0]
    rs = [Request(rid=k, layer=x) for k, x in enumerate(order)]
    for r in rs:
        srv.submit(r)
    srv.poll()
    # the first batch takes the two small requests (the big one does not fit
    # beside them); the big one waits at the head and the last small request
    # may not overtake it
    assert ex.launches == [(0, [0, 1], 0, ex.footprint([0, 0]))]
    assert rs[2].state == QUEUED and rs[3].state == QUEUED
    clk.t = 2.0
    srv.poll()
    assert ex.launches[1][1] == [2]
    assert rs[3].state == QUEUED          # does not fit beside the big one
    clk.t = 3.0
    srv.poll()
    assert ex.launches[2][1] == [3]
    clk.t = 10.0
    srv.poll()
    assert all(r.state == DONE for r in rs)
    assert srv.arena.in_use == 0


def test_refusals():
    clk = FakeClock()
    ex = FakeExecutor(clk, {0: 1 << 20, 1: 64 << 20})
    srv = Server(ex, budget=8 << 20, slots=1, max_batch=2, max_queue=3, clock=clk)
    big = Request(rid=0, layer=1)
    assert not srv.submit(big) and big.state == REFUSED  # never fits the budget
    rs = _reqs(4)
    assert [srv.submit(r) for r in rs] == [True, True, True, False]
    assert rs[3].state == REFUSED
    assert big in srv.finished and rs[3] in srv.finished


def test_timeout_cancels_queued_requests():
    clk = FakeClock()
    ex = FakeExecutor(clk, {0: 1 << 20}, per_request=5.0)
    srv = Server(ex, budget=1 << 30, slots=1, max_batch=1, timeout=2.0, clock=clk)
    rs = _reqs(3)
    for r in rs:
        srv.submit(r)
    srv.poll()                     # r0 runs for 5 s
    clk.t = 2.5
    out = srv.poll()
    assert {r.rid for r in out} == {1, 2} and all(r.state == CANCELLED for r in out)
    clk.t = 5.0
    srv.poll()
    assert rs[0].state == DONE and srv.idle
    assert len(ex.launches) == 1


def test_arrivals_join_while_other_batches_run():
    """Continuous batching: a request arriving while a batch runs starts on
    the free slot at once, overlapping the running batch."""
    clk = FakeClock()
    ex = FakeExecutor(clk, {0: 1 << 20}, per_request=1.0)
    srv = Server(ex, budget=1 << 30, slots=2, max_batch=8, clock=clk)
    first = _reqs(4)
    for r in first:
        srv.submit(r)
    srv.poll()                     # batch on slot 0 until t = 4
    clk.t = 1.0
    late = Request(rid=10, layer=0, arrival=1.0)
    srv.submit(late)
    srv.poll()
    assert late.state == RUNNING and late.t_admit == 1.0
    assert ex.launches[-1][0] == 1
    clk.t = 2.0
    srv.poll()
    assert late.state == DONE and all(r.state == RUNNING for r in first)
    assert late.latency == pytest.approx(1.0)


def test_overlap_only_with_a_backlog():
    """With overlap_min = 3 a lone request arriving during a batch waits for
    it and then runs alone; three or more waiting requests fill the free slot
    at once."""
    clk = FakeClock()
    ex = FakeExecutor(clk, {0: 1 << 20}, per_request=1.0)
    srv = Server(ex, budget=1 << 30, slots=2, max_batch=8, clock=clk, overlap_min=3)
    first = _reqs(2)
    for r in first:
        srv.submit(r)
    srv.poll()                     # batch on slot 0 until t = 2 (the only batch: no wait)
    assert all(r.state == RUNNING for r in first)
    clk.t = 0.5
    late = Request(rid=10, layer=0, arrival=0.5)
    srv.submit(late)
    srv.poll()
    assert late.state == QUEUED and len(ex.launches) == 1
    clk.t = 2.0
    srv.poll()                     # the first batch retires, the lone request starts
    assert all(r.state == DONE for r in first) and late.state == RUNNING and late.t_admit == 2.0
    backlog = [Request(rid=20 + k, layer=0, arrival=2.0) for k in range(3)]
    for r in backlog:
        srv.submit(r)
    srv.poll()                     # three waiting: the free slot takes them now
    assert all(r.state == RUNNING for r in backlog) and len(ex.launches) == 3
    assert ex.launches[-1][0] != ex.launches[-2][0]


def test_poisson_driver_with_fake_clock():
    arr = poisson_arrivals(200, rate=50.0, seed=3)
    assert np.all(np.diff(arr) > 0)
    assert abs(200 / arr[-1] - 50.0) < 15.0
    clk = FakeClock(step=1e-4)
    ex = FakeExecutor(clk, {0: 1 << 20, 1: 2 << 20}, per_request=4e-3)
    srv = Server(ex, budget=64 << 20, slots=2, max_batch=16, clock=clk)
    rs = [Request(rid=k, layer=k % 2) for k in range(200)]
    wall = run_arrivals(srv, rs, arr, clock=clk)
    assert all(r.state == DONE for r in rs) and wall > 0
    s = latency_summary(rs)
    assert s["done"] == 200 and 0 < s["p50_ms"] <= s["p99_ms"] <= s["max_ms"]
    sizes = [n for _, n, _ in srv.batches]
    assert sum(sizes) == 200 and max(sizes) > 1
