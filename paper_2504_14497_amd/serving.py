"""Continuous-batching server for encrypted linear layers.

A request asks for C = W x X: W is one of the server's static plaintext layers
(compiled once into a plan whose arrays stay resident in HBM) and X a matrix of
EC-ElGamal ciphertexts already in HBM; C is written to the request's own
device buffer.  Every request is one Cussen PC-MM (Alg. 3 with Alg. 2).

Scheduling (host side; the GPU work of a batch is one pcmm_plan_run_selected):
  * arrivals queue in FIFO order; a full queue refuses new requests;
  * whenever one of `slots` in-flight batches is free, the head of the queue
    is admitted into a new batch while the batch's workspace (the tables,
    chain scratch and partial sums of its requests) fits a free range of the
    workspace budget and the batch has fewer than `max_batch` requests.  A
    request that arrives while other batches run on the GPU therefore starts
    as soon as a slot and memory free up, and its batch overlaps on the device
    with the batches still running (each slot has its own stream).  With
    `overlap_min` > 1 a batch is admitted while another is in flight only
    when at least that many requests wait: a lone request then waits for the
    running batch and runs alone (overlapping batches share the GPU and both
    take longer), while a backlog still fills every slot;
  * a request whose footprint alone exceeds the whole budget is refused;
  * a request still queued after `timeout` seconds is cancelled;
  * a batch retires when its completion event has fired: its workspace range
    and slot are freed and its requests are stamped done.
The clock and the executor are injectable, so the policy runs on the CPU with
a fake clock and a fake executor; GpuExecutor drives the MI355X.
"""
import bisect
import time
from dataclasses import dataclass

import numpy as np

QUEUED, RUNNING, DONE, CANCELLED, REFUSED = "queued", "running", "done", "cancelled", "refused"


@dataclass
class Request:
    rid: int
    layer: int
    X: object = None          # device ciphertexts (n x l), for the GPU executor
    C: object = None          # device output (m x l)
    arrival: float = 0.0
    state: str = QUEUED
    t_admit: float = None
    t_done: float = None
    batch: int = None

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.arrival


class Arena:
    """First-fit allocator of byte ranges in [0, size), 256-byte aligned."""

    def __init__(self, size: int):
        self.size = int(size)
        self.used = []  # sorted (offset, length)

    @staticmethod
    def _align(x):
        return (int(x) + 255) // 256 * 256

    def find(self, nbytes: int):
        """Offset of the first free range of nbytes, or None (no allocation)."""
        n = self._align(nbytes)
        prev_end = 0
        for off, ln in self.used:
            if off - prev_end >= n:
                return prev_end
            prev_end = off + ln
        return prev_end if self.size - prev_end >= n else None

    def alloc(self, nbytes: int):
        off = self.find(nbytes)
        if off is not None:
            bisect.insort(self.used, (off, self._align(nbytes)))
        return off

    def free(self, off: int):
        for k, (o, _) in enumerate(self.used):
            if o == off:
                del self.used[k]
                return
        raise KeyError(off)

    @property
    def in_use(self):
        return sum(n for _, n in self.used)


@dataclass
class _Batch:
    bid: int
    slot: int
    reqs: list
    offset: int
    handle: object = None


class Server:
    def __init__(self, executor, budget: int, slots: int = 2, max_batch: int = 64, max_queue: int = 100000,
                 timeout: float = None, clock=time.perf_counter, overlap_min: int = 1):
        self.ex = executor
        self.arena = Arena(budget)
        self.slots = slots
        self.max_batch = max_batch
        self.overlap_min = max(1, overlap_min)
        self.max_queue = max_queue
        self.timeout = timeout
        self.clock = clock
        self.queue = []
        self.inflight = {}        # slot -> _Batch
        self.finished = []
        self._next_bid = 0
        self.batches = []         # (bid, size, t_launch) for statistics

    # -- requests -----------------------------------------------------------
    def submit(self, req: Request) -> bool:
        if len(self.queue) >= self.max_queue:
            req.state = REFUSED
            self.finished.append(req)
            return False
        if self.ex.footprint([req.layer]) > self.arena.size:
            req.state = REFUSED      # can never be admitted
            self.finished.append(req)
            return False
        req.state = QUEUED
        self.queue.append(req)
        return True

    @property
    def idle(self):
        return not self.queue and not self.inflight

    # -- one scheduling pass -------------------------------------------------
    def poll(self):
        """Retire finished batches, cancel timed-out requests, admit new
        batches.  Returns the requests that finished in this pass."""
        now = self.clock()
        out = []
        for slot, b in list(self.inflight.items()):
            if self.ex.done(b.handle):
                t = self.clock()
                for r in b.reqs:
                    r.state, r.t_done = DONE, t
                out.extend(b.reqs)
                self.arena.free(b.offset)
                del self.inflight[slot]
        if self.timeout is not None:
            keep = []
            for r in self.queue:
                if now - r.arrival > self.timeout:
                    r.state, r.t_done = CANCELLED, now
                    out.append(r)
                else:
                    keep.append(r)
            self.queue = keep
        for slot in range(self.slots):
            if slot in self.inflight or not self.queue:
                continue
            if self.inflight and len(self.queue) < self.overlap_min:
                break  # a short queue waits for the running batch instead of sharing the GPU
            take, offset = self._take()
            if not take:
                break  # the head does not fit yet: wait for memory (FIFO, no overtaking)
            t = self.clock()
            b = _Batch(self._next_bid, slot, take, offset)
            self._next_bid += 1
            for r in take:
                r.state, r.t_admit, r.batch = RUNNING, t, b.bid
            b.handle = self.ex.launch(slot, take, offset, self.ex.footprint([r.layer for r in take]))
            self.inflight[slot] = b
            self.batches.append((b.bid, len(take), t))
        self.finished.extend(out)
        return out

    def _take(self):
        """The longest queue head (<= max_batch) whose workspace fits a free
        range; allocates that range."""
        k = 0
        while k < min(self.max_batch, len(self.queue)):
            need = self.ex.footprint([r.layer for r in self.queue[:k + 1]])
            if self.arena.find(need) is None:
                break
            k += 1
        if k == 0:
            return [], None
        take = self.queue[:k]
        off = self.arena.alloc(self.ex.footprint([r.layer for r in take]))
        self.queue = self.queue[k:]
        return take, off

    def drain(self, spin=None):
        while not self.idle:
            self.poll()
            if spin:
                spin()


class GpuExecutor:
    """Runs a batch as one pcmm_plan_run_selected on its slot's stream, in a
    range of one workspace tensor; completion is a HIP event.  The plan must
    be resident (Plan.make_resident) before the first launch.

    Ordering contract: a request's X (ciphertexts) and C (output buffer) may
    have been written by work queued on the stream that is current when the
    batch is launched (uploads, encryption, zero fills); the slot stream
    waits for everything queued there before its run starts, and X and C are
    marked as used on the slot stream so that the allocator does not hand
    their memory out again before the run has finished.  A client that
    produces X on yet another stream makes the current stream wait for it
    before submitting."""

    # bound on a selected run's bytes beyond its problems' own regions
    # (descriptor block of up to 64 problems and the queue counter)
    SELECT_OVERHEAD = 64 << 10

    def __init__(self, plan, workspace, slots: int, count: int):
        import torch
        self.plan = plan
        self.ws = workspace
        self.base = workspace.data_ptr()
        self.streams = [torch.cuda.Stream() for _ in range(slots)]  # default priority
        self.layer_ws = [plan.stats(i)["workspace_bytes"] for i in range(count)]
        exact = plan.selected_workspace_bytes([0] * 64)
        assert exact <= 64 * self.layer_ws[0] + self.SELECT_OVERHEAD

    def footprint(self, layers):
        return sum(self.layer_ws[x] for x in layers) + self.SELECT_OVERHEAD

    def launch(self, slot, reqs, offset, nbytes):
        import ctypes
        import torch
        s = self.streams[slot]
        s.wait_stream(torch.cuda.current_stream())
        for r in reqs:
            r.X.t.record_stream(s)
            r.C.t.record_stream(s)
        self.plan.run_selected([r.layer for r in reqs], [r.X for r in reqs], [r.C for r in reqs],
                               (ctypes.c_void_p(self.base + offset), int(nbytes)), stream=s)
        ev = torch.cuda.Event()
        ev.record(s)
        return ev

    def done(self, handle):
        return handle.query()


def poisson_arrivals(count: int, rate: float, seed: int):
    """Arrival times (s) of a Poisson process of `rate` requests/s."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def run_arrivals(server: Server, reqs, arrivals, clock=time.perf_counter):
    """Submits reqs[k] at arrivals[k] seconds after the start (busy loop),
    drives the server until every request has finished; returns the wall
    time from the first arrival to the last completion."""
    t0 = clock()
    k = 0
    n = len(reqs)
    while k < n or not server.idle:
        now = clock() - t0
        while k < n and arrivals[k] <= now:
            reqs[k].arrival = t0 + arrivals[k]
            server.submit(reqs[k])
            k += 1
        server.poll()
    last = max(r.t_done for r in reqs if r.t_done is not None)
    return last - (t0 + arrivals[0])


def latency_summary(reqs):
    lat = np.array([r.latency for r in reqs if r.state == DONE])
    if lat.size == 0:
        return {"done": 0}
    return {"done": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "max_ms": float(lat.max() * 1e3)}
