"""Continuous-batching serving loop over the simulation library.

Requests (batches of candidates of any size and any joint stride J up to the
server's) are admitted into a device-resident byte ring as soon as the ring has
room for their block (admission by the bytes a request really takes: a request
stored at stride J takes 20 J + 7 bytes per candidate, whatever the server's
widest stride).  A request block holds, each part
16-byte aligned: x0 [size][J][2] f64, adj [size][J] u32, fixed [size] u32,
n [size] u8, motor [size][2] u8 (block_layout; the layout links_gather reads).

Admitted candidates form ticks in admission order.  A tick takes up to tick_max
candidates, which may be the tail of one request, several whole requests and the
head of another; it is one links_gather (the candidates into the lane's staging
batch at the server's stride, one kernel) and one replay of a HIP graph of the
whole simulation, captured once per tick size class (powers of two from
min_class to tick_max; rows past the tick's candidates have no joints and are
never simulated).  Two lanes (library context, stream, staging, graphs) keep up
to two ticks on the device at once, so a request that arrives while a tick runs
starts in the next tick on the other lane.

A tick runs its candidates to their end (failure or all T steps), so a request
no larger than a tick is answered after about one tick; the persistent kernels
inside the graph refill a lane as soon as its candidate fails.

When a tick finishes, its outputs (status, fail_step, esc_step and the coupler
paths of its valid candidates) are copied out of the staging buffers once, on
the lane's stream, and each request keeps views of its share; the request's ring
block is freed once every tick holding its candidates has finished.

The decisions and paths of a candidate do not depend on which tick, staging row,
stride or neighbours it is simulated with (every kernel works per candidate), so
a request gives the same results alone and in the mix.

This module is the host scheduler only: ring bookkeeping, stream, event and
graph handling.  All simulation work runs in the HIP library.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Deque, Dict, List, Optional, Tuple

import numpy as np

ALIGN = 16


def _align(b: int) -> int:
    return (b + ALIGN - 1) // ALIGN * ALIGN


def block_layout(size: int, J: int) -> Tuple[Dict[str, int], int]:
    """Byte offsets of the parts of a request block of `size` candidates at stride
    J, and its total bytes (a multiple of 16)."""
    off = {"x0": 0}
    off["adj"] = _align(size * J * 16)
    off["fixed"] = off["adj"] + _align(size * J * 4)
    off["n"] = off["fixed"] + _align(size * 4)
    off["motor"] = off["n"] + _align(size)
    return off, off["motor"] + _align(size * 2)


class RingAlloc:
    """FIFO allocator of `capacity` units addressed by monotonically increasing
    coordinates (address = coordinate mod capacity).  Allocations are made in
    order; a freed allocation is returned once every earlier one is also freed.
    `alloc_contiguous` never lets an allocation cross the end of the ring: the
    units up to the end are skipped (held like an allocation freed at once)."""

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
            raise ValueError(f"allocation of {size} units in a ring of {self.capacity}")
        if self.used + size > self.capacity:
            return None
        start = self.head
        self.head += size
        self._live.append([start, size, False])
        return start

    def alloc_contiguous(self, size: int) -> Optional[int]:
        if size < 0 or size > self.capacity:
            raise ValueError(f"allocation of {size} units in a ring of {self.capacity}")
        a = self.head % self.capacity
        if self.used == 0 and a:   # empty: start at the next lap, so any size up to capacity fits
            self.head = self.tail = self.head - a + self.capacity
            a = 0
        skip = self.capacity - a if a + size > self.capacity else 0
        if self.used + skip + size > self.capacity:
            return None
        if skip:
            self._live.append([self.head, skip, True])
            self.head += skip
            self._pop()
        return self.alloc(size)

    def free(self, start: int):
        for e in self._live:
            if e[0] == start and not e[2]:
                e[2] = True
                break
        else:
            raise KeyError(start)
        self._pop()

    def _pop(self):
        while self._live and self._live[0][2]:
            s, n, _ = self._live.popleft()
            self.tail = s + n


def size_classes(tick_max: int, min_class: int) -> List[int]:
    """Tick size classes: tick_max, tick_max / 2, ... down to the first one at or
    below min_class (at least 1)."""
    out = [tick_max]
    while out[-1] > max(min_class, 1):
        out.append((out[-1] + 1) // 2)
    return out


def class_of(count: int, classes: List[int]) -> int:
    """The smallest class (classes in decreasing order) holding `count` rows."""
    best = classes[0]
    for c in classes:
        if c >= count:
            best = c
    return best


def plan_tick(queue: List[Tuple[int, int, int]], tick_max: int, max_pieces: int) -> Tuple[List[Tuple[int, int, int, int]], int]:
    """The next tick over queued requests [(id, next candidate, size)] in order:
    shares [(id, first, count, first output row)] of at most tick_max candidates
    and max_pieces requests, and the number of requests it finishes dispatching."""
    shares, rows, whole = [], 0, 0
    for rid, first, size in queue:
        if rows >= tick_max or len(shares) >= max_pieces:
            break
        take = min(size - first, tick_max - rows)
        if take <= 0:
            whole += 1
            continue
        shares.append((rid, first, take, rows))
        rows += take
        if first + take == size:
            whole += 1
        else:
            break
    return shares, whole


@dataclass
class Part:
    """A request's share of one tick: candidates first .. first+len-1."""
    first: int
    status: object
    fail_step: object
    esc_step: object
    valid: np.ndarray      # request-local indices of its valid candidates
    path: object           # [len(valid), T, 2]


@dataclass
class Request:
    rid: int
    size: int
    J: int
    arrival: float
    start: int = -1                   # ring coordinate of its block once admitted
    nbytes: int = 0
    dispatched: int = 0               # candidates handed to ticks
    collected: int = 0                # candidates whose tick has finished
    admitted_at: float = -1.0
    finished_at: float = -1.0
    parts: List[Part] = field(default_factory=list)
    # events after the output copies of each tick holding its candidates (a request
    # can span ticks on both lanes); it is retired once every one has completed
    copy_events: List[object] = field(default_factory=list)
    source: object = None             # DeviceBatch or packed block until admitted

    @property
    def done(self) -> int:
        return self.collected

    @property
    def latency(self) -> float:
        return self.finished_at - self.arrival

    def _cat(self, name: str, dtype):
        import torch
        parts = sorted(self.parts, key=lambda q: q.first)
        if not parts:
            return torch.empty(0, dtype=dtype)
        if len(parts) == 1:
            return getattr(parts[0], name)
        return torch.cat([getattr(q, name) for q in parts])

    @property
    def status(self):
        import torch
        return self._cat("status", torch.uint8)

    @property
    def fail_step(self):
        import torch
        return self._cat("fail_step", torch.int16)

    @property
    def esc_step(self):
        import torch
        return self._cat("esc_step", torch.int16)

    def valid(self) -> Tuple[np.ndarray, object]:
        """Request-local indices of the valid candidates and their coupler paths."""
        import torch
        parts = sorted(self.parts, key=lambda q: q.first)
        if not parts:
            return np.zeros(0, np.int64), None
        return np.concatenate([q.valid for q in parts]), torch.cat([q.path for q in parts])


def pack(batch, device=None) -> "Packed":
    """A request's candidates (DeviceBatch, x0 in f64) as one packed block (a uint8
    device tensor in block_layout), the form in which a client hands a request over
    with a single copy."""
    import torch
    off, nbytes = block_layout(batch.B, batch.J)
    dev = batch.n.device if device is None else device
    blk = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
    _write_block(blk, 0, batch, off)
    return Packed(blk, batch.B, batch.J)


def _write_block(buf, base: int, b, off: Dict[str, int]):
    import torch
    if b.x0.dtype != torch.float64:
        raise ValueError("serving requests carry x0 in float64")
    size, J = b.B, b.J
    if size == 0:
        return

    def part(name, nb, dtype, shape):
        a = base + off[name]
        return buf[a:a + nb].view(dtype).view(shape)

    part("x0", size * J * 16, torch.float64, (size, J, 2)).copy_(b.x0, non_blocking=True)
    part("adj", size * J * 4, torch.int32, (size, J)).copy_(b.adj, non_blocking=True)
    part("fixed", size * 4, torch.int32, (size,)).copy_(b.fixed, non_blocking=True)
    part("n", size, torch.uint8, (size,)).copy_(b.n, non_blocking=True)
    part("motor", size * 2, torch.uint8, (size, 2)).copy_(b.motor, non_blocking=True)


class Packed:
    """A request already in block form (see pack)."""

    def __init__(self, block, size: int, J: int):
        self.block, self.B, self.J = block, size, J


class _Lane:
    """One library context with its stream, staging batch and outputs, the graphs
    of every tick size class and the tick in flight."""

    def __init__(self, links, device, tick_max, J, T, max_pieces):
        import torch
        dev = torch.device("cuda", device)
        self.ctx = links.Context(device)
        self.stream = torch.cuda.Stream(device=device)   # default priority
        self.batch = links.DeviceBatch(torch.zeros(tick_max, dtype=torch.uint8, device=dev),
                                       torch.zeros((tick_max, J), dtype=torch.int32, device=dev),
                                       torch.zeros(tick_max, dtype=torch.int32, device=dev),
                                       torch.zeros((tick_max, 2), dtype=torch.uint8, device=dev),
                                       torch.zeros((tick_max, J, 2), dtype=torch.float64, device=dev))
        self.status = torch.empty(tick_max, dtype=torch.uint8, device=dev)
        self.fail_step = torch.empty(tick_max, dtype=torch.int16, device=dev)
        self.esc_step = torch.empty(tick_max, dtype=torch.int16, device=dev)
        self.path = torch.empty((tick_max, T, 2), dtype=torch.float32, device=dev)
        self.path_index = torch.empty(tick_max, dtype=torch.int32, device=dev)
        self.n_written = torch.zeros(1, dtype=torch.int32, device=dev)
        self.nw_host = torch.zeros(1, dtype=torch.int32).pin_memory()
        self.pieces_host = torch.zeros(max_pieces * links.PIECE_DTYPE.itemsize, dtype=torch.uint8).pin_memory()
        self.pieces_np = self.pieces_host.numpy().view(links.PIECE_DTYPE)
        self.pieces_dev = torch.empty_like(self.pieces_host, device=dev)
        self.graphs: Dict[int, object] = {}
        self.tick = None          # (shares, count, event) of the tick in flight
        self.copies = None        # (event, finished requests) of output copies in flight

    def prefix(self, links, rows: int):
        b = self.batch
        return links.DeviceBatch(b.n[:rows], b.adj[:rows], b.fixed[:rows], b.motor[:rows], b.x0[:rows])


class Server:
    """Continuous-batching server (see the module docstring).

    capacity    bytes of the device ring that holds admitted requests
    tick_max    most candidates one tick simulates
    J           the widest joint stride a request may have
    precision   links.FP32_RECHECK, FP64 or FP32_ONLY for every tick
    branch      links.BRANCH_CONTINUITY or BRANCH_ORIENTATION for every tick
    min_class   smallest tick size class (a graph per class and lane)
    max_pieces  most requests one tick takes candidates from
    """

    def __init__(self, capacity: int = 1 << 30, tick_max: int = 1 << 19, J: int = 20, T: int = 200,
                 precision: int = 0, device: int = 0, lanes: int = 2, min_class: int = 4096,
                 max_pieces: int = 8192, branch: int = 0):
        import torch
        from . import links
        if not 1 <= J <= 32:
            raise ValueError("J must be in 1..32")
        self.L = links
        self.T, self.J, self.precision, self.branch = T, J, precision, branch
        self.tick_max = tick_max
        self.capacity = _align(capacity)
        self.classes = size_classes(tick_max, min_class)
        self.max_pieces = max_pieces
        dev = torch.device("cuda", device)
        self.dev = dev
        self.ring = RingAlloc(self.capacity)
        self.buf = torch.zeros(self.capacity, dtype=torch.uint8, device=dev)
        self.lanes = [_Lane(links, device, tick_max, J, T, max_pieces) for _ in range(lanes)]
        self.admit_stream = torch.cuda.Stream(device=dev)
        self.admit_event = None
        self.waiting: Deque[Request] = collections.deque()   # not yet admitted
        self.queue: Deque[Request] = collections.deque()     # admitted, not all dispatched (admission order)
        self.active: Dict[int, Request] = {}                  # admitted, not retired
        self.finished: List[Request] = []
        self.ticks = 0
        self.next_id = 0
        self.warmed = False

    def warm(self, cfg: Optional[dict] = None):
        """Captures the graph of every tick size class on every lane, the largest
        first so that the context's workspace is sized once (after applying the
        tuning `cfg` if given), then replays each once on an empty batch, so that
        nothing is allocated or captured while serving."""
        import torch
        L = self.L
        for lane in self.lanes:
            if cfg:
                from . import tune
                tune.apply(lane.ctx, cfg)
            for c in self.classes:
                out = {"status": lane.status[:c], "fail_step": lane.fail_step[:c], "esc_step": lane.esc_step[:c],
                       "path": lane.path[:c], "path_index": lane.path_index[:c], "n_written": lane.n_written}
                lane.graphs[c] = lane.ctx.graph(lane.prefix(L, c), T=self.T, precision=self.precision,
                                                write=L.WRITE_VALID, cap=c, out=out, branch=self.branch)
            lane.batch.n.zero_()
            torch.cuda.synchronize()
            for c in self.classes:
                lane.graphs[c].launch(lane.stream)
        torch.cuda.synchronize()
        self.warmed = True

    def close(self):
        for lane in self.lanes:
            for g in lane.graphs.values():
                g.close()
            lane.graphs.clear()

    # -------------------------------------------------------------- submission
    def submit(self, batch, arrival: Optional[float] = None) -> Request:
        """Queues a request (a DeviceBatch with x0 in f64, or a Packed block) of
        stride J up to the server's; it is admitted as soon as the ring has room
        for its block."""
        if batch.J > self.J or batch.J < 1:
            raise ValueError(f"request has J={batch.J}, the server takes J in 1..{self.J}")
        nbytes = block_layout(batch.B, batch.J)[1]
        if nbytes > self.capacity:
            raise ValueError(f"request of {nbytes} bytes exceeds the ring ({self.capacity})")
        r = Request(self.next_id, batch.B, batch.J, time.perf_counter() if arrival is None else arrival,
                    nbytes=nbytes, source=batch)
        self.next_id += 1
        self.waiting.append(r)
        return r

    def _admit(self):
        import torch
        synced = False
        while self.waiting:
            r = self.waiting[0]
            if r.size == 0:
                self.waiting.popleft()
                r.admitted_at = r.finished_at = time.perf_counter()
                r.source = None
                self.finished.append(r)
                continue
            start = self.ring.alloc_contiguous(r.nbytes)
            if start is None:
                break
            self.waiting.popleft()
            r.start = start
            r.admitted_at = time.perf_counter()
            if not synced:   # inputs written on the caller's stream are complete before they are read
                self.admit_stream.wait_stream(torch.cuda.current_stream(self.dev))
                synced = True
            a = start % self.capacity
            with torch.cuda.stream(self.admit_stream):
                if isinstance(r.source, Packed):
                    srcs = [r.source.block]
                    self.buf[a:a + r.nbytes].copy_(r.source.block[:r.nbytes], non_blocking=True)
                else:
                    s = r.source
                    srcs = [s.n, s.adj, s.fixed, s.motor, s.x0]
                    _write_block(self.buf, a, s, block_layout(r.size, r.J)[0])
            for t in srcs:   # the caller's memory is not reused before the copy has read it
                t.record_stream(self.admit_stream)
            r.source = None
            self.queue.append(r)
            self.active[r.rid] = r
        if synced:
            ev = torch.cuda.Event()
            ev.record(self.admit_stream)
            self.admit_event = ev

    # -------------------------------------------------------------- ticks
    def _launch(self, lane: _Lane) -> bool:
        import torch
        if not self.queue:
            return False
        if not self.warmed:
            raise RuntimeError("Server.warm() captures the tick graphs before serving")
        q = [(r.rid, r.dispatched, r.size) for r in self.queue]
        shares, whole = plan_tick(q, self.tick_max, self.max_pieces)
        count = sum(s[2] for s in shares)
        cls = class_of(count, self.classes)
        pn = lane.pieces_np
        tick = []
        for p, (rid, first, take, dst) in enumerate(shares):
            r = self.active[rid]
            pn[p] = (r.start % self.capacity, dst, first, r.size, r.J)
            r.dispatched = first + take
            tick.append((r, first, take, dst))
        for _ in range(whole):
            self.queue.popleft()
        L = self.L
        nb = len(shares) * L.PIECE_DTYPE.itemsize
        with torch.cuda.stream(lane.stream):
            lane.pieces_dev[:nb].copy_(lane.pieces_host[:nb], non_blocking=True)
        if self.admit_event is not None:
            lane.stream.wait_event(self.admit_event)
        lane.ctx.gather(self.buf, lane.pieces_dev, len(shares), count, lane.prefix(L, cls), stream=lane.stream)
        lane.graphs[cls].launch(lane.stream)
        with torch.cuda.stream(lane.stream):
            lane.nw_host.copy_(lane.n_written, non_blocking=True)
        ev = torch.cuda.Event()
        ev.record(lane.stream)
        lane.tick = (tick, count, ev)
        self.ticks += 1
        return True

    def _collect(self, lane: _Lane):
        """Outputs of a finished tick: one copy of each on the lane's stream, and
        each request's share as views of them."""
        import torch
        if lane.copies is not None:      # enqueued before this tick on the same stream: done
            lane.copies[0].synchronize()
            self._retire(lane)
        tick, count, _ = lane.tick
        lane.tick = None
        k = int(lane.nw_host[0])
        idx = lane.path_index[:k].cpu().numpy().astype(np.int64) if k else np.zeros(0, np.int64)
        with torch.cuda.stream(lane.stream):
            st = lane.status[:count].clone()
            fs = lane.fail_step[:count].clone()
            es = lane.esc_step[:count].clone()
            pth = lane.path[:k].clone()
            ev = torch.cuda.Event()
            ev.record(lane.stream)
        finished = []
        for r, first, take, dst in tick:
            p0, p1 = np.searchsorted(idx, [dst, dst + take])
            r.parts.append(Part(first, st[dst:dst + take], fs[dst:dst + take], es[dst:dst + take],
                                idx[p0:p1] - dst + first, pth[p0:p1]))
            r.collected += take
            r.copy_events.append(ev)
            if r.collected == r.size:
                self.ring.free(r.start)   # every gather from its block has run
                finished.append(r)
        lane.copies = (ev, finished)

    def _retire(self, lane: _Lane):
        ev, finished = lane.copies
        lane.copies = None
        for r in finished:
            # its shares copied on the other lane may still be in flight: its latency
            # is stamped once all of them are done
            for e in r.copy_events:
                e.synchronize()
            r.copy_events.clear()
        now = time.perf_counter()
        for r in finished:
            r.finished_at = now
            del self.active[r.rid]
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
            if lane.tick is None:        # output copies of its last tick run first on its stream
                self._launch(lane)
        return bool(self.waiting or self.active)

    def drain(self):
        while self.poll():
            pass


def run_stream(server: Server, requests: List, arrivals: np.ndarray, pause_gc: bool = True) -> List[Request]:
    """Submits requests[i] (a DeviceBatch or Packed) at arrivals[i] seconds after the
    start, polling the server in between; returns the finished requests in
    submission order.  With pause_gc, Python's cyclic garbage collector is paused
    while the loop runs (a collection pass over the loop's objects stalls the
    scheduler for tens of milliseconds; reference counting still frees memory)."""
    import gc
    was = gc.isenabled()
    if pause_gc:
        gc.disable()
    try:
        t0 = time.perf_counter()
        order = np.argsort(arrivals, kind="stable")
        reqs: Dict[int, Request] = {}
        i = 0
        while i < len(order) or server.poll():
            now = time.perf_counter() - t0
            while i < len(order) and arrivals[order[i]] <= now:
                j = order[i]
                reqs[j] = server.submit(requests[j], arrival=t0 + float(arrivals[j]))
                i += 1
            server.poll()
    finally:
        if was:
            gc.enable()
    return [reqs[j] for j in range(len(requests))]


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
