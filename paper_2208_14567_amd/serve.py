"""Continuous-batching serving loop over the simulation library.

Requests (batches of candidates of any size) are admitted into a device-resident
ring of candidate slots as soon as the ring has room for them (admission by
memory).  Admitted candidates form ticks: each tick is one links_simulate call over
a contiguous run of ring slots, which may hold the tail of one request, several
whole requests and the head of another.  Two library contexts on two streams keep
up to two ticks on the device at once, so a request that arrives while a tick runs
starts in the next tick on the other stream without waiting for the first one.
When a tick finishes, each request's share of the results (status, fail_step,
esc_step and the coupler paths of its valid candidates) is copied into the
request's own device tensors on the tick's stream, and the request's slots are
returned to the ring once all of its candidates are done.

The decisions and paths of a candidate do not depend on which tick, ring slot or
neighbours it is simulated with (every kernel works per candidate), so a request
gives the same results alone and in the mix.

This module is the host scheduler only: ring bookkeeping, stream and event
handling.  All simulation work runs in the HIP library.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Deque, Dict, List, Optional, Tuple

import numpy as np


class RingAlloc:
    """FIFO allocator of `capacity` slots addressed by monotonically increasing
    coordinates (slot address = coordinate mod capacity).  Allocations are made in
    order; a freed allocation is returned once every earlier one is also freed."""

    def __init__(self, capacity: int):
        if capacity <= 0:
            raise ValueError("capacity must be positive")
        self.capacity = capacity
        self.head = 0          # next coordinate to hand out
        self.tail = 0          # first coordinate still in use
        self._live: Deque[List] = collections.deque()  # [start, size, freed]

    @property
    def used(self) -> int:
        return self.head - self.tail

    def alloc(self, size: int) -> Optional[int]:
        if size < 0 or size > self.capacity:
            raise ValueError(f"allocation of {size} slots in a ring of {self.capacity}")
        if self.used + size > self.capacity:
            return None
        start = self.head
        self.head += size
        self._live.append([start, size, False])
        return start

    def free(self, start: int):
        for e in self._live:
            if e[0] == start and not e[2]:
                e[2] = True
                break
        else:
            raise KeyError(start)
        while self._live and self._live[0][2]:
            s, n, _ = self._live.popleft()
            self.tail = s + n


def tick_range(lo: int, hi: int, capacity: int, tick_max: int) -> Tuple[int, int]:
    """The next tick over pending coordinates [lo, hi): at most tick_max slots and
    never across the end of the ring (a tick is one contiguous slot range)."""
    if hi <= lo:
        return lo, lo
    end_of_ring = (lo // capacity + 1) * capacity
    return lo, min(hi, lo + tick_max, end_of_ring)


def overlaps(lo: int, hi: int, reqs: List[Tuple[int, int, int]]) -> List[Tuple[int, int, int]]:
    """(request id, first, last) ranges of the requests [(id, start, size)] that
    fall inside coordinates [lo, hi), as offsets within each request."""
    out = []
    for rid, start, size in reqs:
        a, b = max(lo, start), min(hi, start + size)
        if a < b:
            out.append((rid, a - start, b - start))
    return out


@dataclass
class Request:
    rid: int
    size: int
    arrival: float
    start: int = -1                   # ring coordinate once admitted
    done: int = 0                     # candidates finished
    admitted_at: float = -1.0
    finished_at: float = -1.0
    status: object = None             # device tensors [size]
    fail_step: object = None
    esc_step: object = None
    # per tick share: (first request-local index of the share, valid indices, device paths [k, T, 2]);
    # ticks on different streams can finish out of order
    pieces: List[Tuple[int, np.ndarray, object]] = field(default_factory=list)
    # events after the copies of each of its shares (a request can span ticks on
    # both lanes); it is retired only once every one of them has completed
    copy_events: List[object] = field(default_factory=list)
    source: object = None             # DeviceBatch until admitted

    @property
    def latency(self) -> float:
        return self.finished_at - self.arrival

    def valid(self) -> Tuple[np.ndarray, object]:
        """Request-local indices of the valid candidates and their coupler paths."""
        import torch
        if not self.pieces:
            return np.zeros(0, np.int64), None
        pieces = sorted(self.pieces, key=lambda q: q[0])
        return np.concatenate([q[1] for q in pieces]), torch.cat([q[2] for q in pieces])


class _Lane:
    """One library context with its stream, path pool and the tick in flight."""

    def __init__(self, links, device, tick_max, J, T):
        import torch
        self.ctx = links.Context(device)
        self.stream = torch.cuda.Stream(device=device)   # default priority
        self.path = torch.empty((tick_max, T, 2), dtype=torch.float32, device=device)
        self.path_index = torch.empty(tick_max, dtype=torch.int32, device=device)
        self.n_written = torch.empty(1, dtype=torch.int32, device=device)
        self.tick = None          # (lo, hi, event) of the tick in flight
        self.copies = None        # (event, finished requests) of result copies in flight


class Server:
    """Continuous-batching server (see the module docstring).

    capacity   candidate slots in the device ring (inputs plus per-slot results)
    tick_max   most candidates one tick simulates
    """

    def __init__(self, capacity: int = 1 << 21, tick_max: int = 1 << 19, J: int = 20, T: int = 200,
                 precision: int = 0, device: int = 0, lanes: int = 2):
        import torch
        from . import links
        self.L = links
        self.T, self.J, self.precision = T, J, precision
        self.capacity, self.tick_max = capacity, min(tick_max, capacity)
        dev = torch.device("cuda", device)
        self.dev = dev
        self.ring = RingAlloc(capacity)
        C = capacity
        self.n = torch.zeros(C, dtype=torch.uint8, device=dev)
        self.adj = torch.zeros((C, J), dtype=torch.int32, device=dev)
        self.fixed = torch.zeros(C, dtype=torch.int32, device=dev)
        self.motor = torch.zeros((C, 2), dtype=torch.uint8, device=dev)
        self.x0 = torch.zeros((C, J, 2), dtype=torch.float64, device=dev)
        self.status = torch.zeros(C, dtype=torch.uint8, device=dev)
        self.fail_step = torch.zeros(C, dtype=torch.int16, device=dev)
        self.esc_step = torch.zeros(C, dtype=torch.int16, device=dev)
        self.lanes = [_Lane(links, device, self.tick_max, J, T) for _ in range(lanes)]
        self.admit_stream = torch.cuda.Stream(device=dev)
        self.admit_event = None
        self.waiting: Deque[Request] = collections.deque()   # not yet admitted
        self.active: Deque[Request] = collections.deque()    # admitted, not finished (ring order)
        self.finished: List[Request] = []
        self.launched = 0        # ring coordinate up to which ticks have been launched
        self.admitted = 0        # ring coordinate up to which inputs are in the ring
        self.ticks = 0
        self.next_id = 0

    def warm(self, batch):
        """Sizes every lane's library workspace for a full tick (one simulation of
        `batch`, which should hold tick_max candidates) so that no allocation
        happens while serving."""
        import torch
        L = self.L
        for lane in self.lanes:
            out = {"path": lane.path, "path_index": lane.path_index, "n_written": lane.n_written}
            lane.ctx.simulate(batch, T=self.T, precision=self.precision, write=L.WRITE_VALID,
                              cap=self.tick_max, out=out, stream=lane.stream)
        torch.cuda.synchronize()

    # -------------------------------------------------------------- submission
    def submit(self, batch, arrival: Optional[float] = None) -> Request:
        """Queues a request (a DeviceBatch with the server's J); it is admitted as
        soon as the ring has room."""
        if batch.J != self.J:
            raise ValueError(f"request has J={batch.J}, server ring has J={self.J}")
        if batch.B > self.capacity:
            raise ValueError(f"request of {batch.B} candidates exceeds the ring ({self.capacity})")
        r = Request(self.next_id, batch.B, time.perf_counter() if arrival is None else arrival, source=batch)
        self.next_id += 1
        self.waiting.append(r)
        return r

    def _admit(self):
        import torch
        while self.waiting:
            r = self.waiting[0]
            start = self.ring.alloc(r.size)
            if start is None:
                return
            self.waiting.popleft()
            r.start = start
            r.admitted_at = time.perf_counter()
            dev = self.dev
            r.status = torch.empty(r.size, dtype=torch.uint8, device=dev)
            r.fail_step = torch.empty(r.size, dtype=torch.int16, device=dev)
            r.esc_step = torch.empty(r.size, dtype=torch.int16, device=dev)
            if r.size == 0:
                r.finished_at = r.admitted_at
                r.source = None
                self.ring.free(start)
                self.finished.append(r)
                continue
            # inputs written on the caller's stream are complete before they are read
            self.admit_stream.wait_stream(torch.cuda.current_stream(self.dev))
            with torch.cuda.stream(self.admit_stream):
                done = 0
                while done < r.size:           # a request may wrap around the ring end
                    a = (start + done) % self.capacity
                    k = min(r.size - done, self.capacity - a)
                    s = r.source
                    self.n[a:a + k].copy_(s.n[done:done + k], non_blocking=True)
                    self.adj[a:a + k].copy_(s.adj[done:done + k], non_blocking=True)
                    self.fixed[a:a + k].copy_(s.fixed[done:done + k], non_blocking=True)
                    self.motor[a:a + k].copy_(s.motor[done:done + k], non_blocking=True)
                    self.x0[a:a + k].copy_(s.x0[done:done + k], non_blocking=True)
                    done += k
                ev = torch.cuda.Event()
                ev.record(self.admit_stream)
            self.admit_event = ev
            r.source = None
            self.active.append(r)
            self.admitted = start + r.size

    # -------------------------------------------------------------- ticks
    def _launch(self, lane: _Lane) -> bool:
        import torch
        lo, hi = tick_range(self.launched, self.admitted, self.capacity, self.tick_max)
        if hi <= lo:
            return False
        a, b = lo % self.capacity, lo % self.capacity + (hi - lo)
        L = self.L
        batch = L.DeviceBatch(self.n[a:b], self.adj[a:b], self.fixed[a:b], self.motor[a:b], self.x0[a:b])
        out = {"status": self.status[a:b], "fail_step": self.fail_step[a:b], "esc_step": self.esc_step[a:b],
               "path": lane.path, "path_index": lane.path_index, "n_written": lane.n_written}
        if self.admit_event is not None:
            lane.stream.wait_event(self.admit_event)
        lane.ctx.simulate(batch, T=self.T, precision=self.precision, write=L.WRITE_VALID, cap=self.tick_max,
                          out=out, stream=lane.stream)
        ev = torch.cuda.Event()
        ev.record(lane.stream)
        lane.tick = (lo, hi, ev)
        self.launched = hi
        self.ticks += 1
        return True

    def _collect(self, lane: _Lane):
        """Results of a finished tick: copy each request's share on the lane's stream."""
        import torch
        if lane.copies is not None:      # enqueued before this tick on the same stream: done
            lane.copies[0].synchronize()
            self._retire(lane)
        lo, hi, _ = lane.tick
        lane.tick = None
        k = int(lane.n_written.cpu()[0])
        idx = lane.path_index[:k].cpu().numpy().astype(np.int64) + lo   # ring coordinates, ascending
        reqs = [(r.rid, r.start, r.size) for r in self.active]
        by_id = {r.rid: r for r in self.active}
        finished = []
        touched = []
        a0 = lo % self.capacity
        with torch.cuda.stream(lane.stream):
            for rid, first, last in overlaps(lo, hi, reqs):
                r = by_id[rid]
                ra = (r.start + first) - lo + a0           # slot address of the request's first candidate here
                rb = ra + (last - first)
                r.status[first:last].copy_(self.status[ra:rb], non_blocking=True)
                r.fail_step[first:last].copy_(self.fail_step[ra:rb], non_blocking=True)
                r.esc_step[first:last].copy_(self.esc_step[ra:rb], non_blocking=True)
                p0 = np.searchsorted(idx, r.start + first)
                p1 = np.searchsorted(idx, r.start + last)
                if p1 > p0:
                    r.pieces.append((first, idx[p0:p1] - r.start, lane.path[p0:p1].clone()))
                r.done += last - first
                touched.append(r)
                if r.done == r.size:
                    finished.append(r)
            ev = torch.cuda.Event()
            ev.record(lane.stream)
        for r in touched:
            r.copy_events.append(ev)
        lane.copies = (ev, finished)

    def _retire(self, lane: _Lane):
        ev, finished = lane.copies
        lane.copies = None
        for r in finished:
            # its shares copied on the other lane may still be in flight: its ring
            # slots are freed, and its latency stamped, once all of them are done
            for e in r.copy_events:
                e.synchronize()
            r.copy_events.clear()
        now = time.perf_counter()
        for r in finished:
            r.finished_at = now
            self.ring.free(r.start)
            self.active.remove(r)
            self.finished.append(r)

    def poll(self) -> bool:
        """One scheduling round: retire finished copies, collect finished ticks,
        admit waiting requests and launch ticks on idle lanes.  Returns True while
        work remains."""
        for lane in self.lanes:
            if lane.copies is not None and lane.copies[0].query():
                self._retire(lane)
            if lane.tick is not None and lane.tick[2].query():
                self._collect(lane)
        self._admit()
        for lane in self.lanes:
            if lane.tick is None:        # result copies of its last tick run first on its stream
                self._launch(lane)
        return bool(self.waiting or self.active)

    def drain(self):
        while self.poll():
            pass


def run_stream(server: Server, pool, sizes: np.ndarray, offsets: np.ndarray, arrivals: np.ndarray) -> List[Request]:
    """Submits request i (candidates pool[offsets[i] : offsets[i] + sizes[i]]) at
    arrivals[i] seconds after the start, polling the server in between; returns the
    finished requests in submission order."""
    t0 = time.perf_counter()
    order = np.argsort(arrivals, kind="stable")
    reqs: Dict[int, Request] = {}
    i = 0
    while i < len(order) or server.poll():
        now = time.perf_counter() - t0
        while i < len(order) and arrivals[order[i]] <= now:
            j = order[i]
            reqs[j] = server.submit(pool.slice(int(offsets[j]), int(offsets[j] + sizes[j])),
                                    arrival=t0 + float(arrivals[j]))
            i += 1
        server.poll()
    return [reqs[j] for j in range(len(sizes))]


def request_sizes(count: int, seed: int, lo: int = 1, hi: int = 200_000) -> np.ndarray:
    """Request sizes, log-uniform integers in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return np.minimum(hi, np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi + 1), count)))).astype(np.int64)


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed + 1)
    return np.cumsum(rng.exponential(1.0 / rate, count))


def latency_stats(reqs: List[Request]) -> dict:
    lat = np.array([r.latency for r in reqs]) * 1e3
    return {"requests": len(reqs), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max())}
