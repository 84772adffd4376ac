"""Streamed generation and simulation of candidates in chunks, with a resume point.

The dataset pipeline's outer loop ("Scale of Infeasibilities": billions of
random candidates, of which the valid ones are kept): chunk c holds candidates
c * chunk .. (c + 1) * chunk - 1 of the seed's sequence, generated on the device
(links_generate_dyads), simulated (FP32 with FP64 escalation by default, valid
coupler paths compacted), and the valid paths normalised on the device; only
the valid paths, their candidate indices and transforms cross PCIe.

Two lanes (a library context and a stream each) alternate chunks, so one chunk's
copies to pinned host memory overlap the next chunk's simulation.  Chunks reach
the sink in order.

Resume point: with a progress file, the stream records after each chunk's
delivery the next chunk to run and the running totals, in a small JSON file
replaced atomically.  The generator is counter-based (a candidate's draws depend
only on the seed and its index), so a stream restarted from the file continues
with exactly the candidates it would have run, and a chunk delivered again after
a crash (between its sink call and the file update) is delivered with the same
contents.

Host source: given a batch in host memory (candidates generated elsewhere),
the stream copies chunk c's rows from pinned memory on the lane's stream instead
of generating them, so a chunk's inputs cross PCIe while the other lane
simulates.  Positions can cross in single precision when that is exact (the
library widens them on the device).

This module is host scheduling only; all generation, simulation and
normalisation run in the HIP library.
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import asdict, dataclass
from typing import Callable, Dict, Optional

import numpy as np


@dataclass
class StreamConfig:
    seed: int
    chunks: int
    chunk: int = 4_000_000
    J: int = 20
    n_lo: int = 6
    n_hi: int = 20
    T: int = 200
    paper_mode: bool = False
    rules: bool = False
    precision: int = 0          # links.FP32_RECHECK
    cap: int = 1_000_000        # most valid paths kept per chunk
    norm: int = 0               # links.NORM_PCA


class Progress:
    """The resume point of a stream: its configuration, the next chunk to run and
    the running totals."""

    VERSION = 1

    def __init__(self, path: str):
        self.path = path

    def load(self, cfg: StreamConfig) -> Optional[dict]:
        """The recorded state, or None when there is no file; raises ValueError when
        the file belongs to another stream configuration."""
        if not os.path.exists(self.path):
            return None
        with open(self.path) as f:
            st = json.load(f)
        if st.get("version") != self.VERSION or st.get("config") != asdict(cfg):
            raise ValueError(f"{self.path} records another stream: {st.get('config')}")
        return st

    def save(self, cfg: StreamConfig, next_chunk: int, totals: Dict[str, int]):
        st = {"version": self.VERSION, "config": asdict(cfg), "next_chunk": int(next_chunk),
              "totals": {k: int(v) for k, v in totals.items()}, "updated": time.time()}
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(st, f)
            f.flush()
            os.fsync(f.fileno())
        os.replace(tmp, self.path)


class NpzSink:
    """Writes each chunk's valid paths to out_dir/chunk_NNNNNN.npz (candidate index
    int64, normalised path f32 [k, T, 2], transform f32 [k, 5]), atomically."""

    def __init__(self, out_dir: str):
        self.out_dir = out_dir
        os.makedirs(out_dir, exist_ok=True)

    def path_of(self, c: int) -> str:
        return os.path.join(self.out_dir, f"chunk_{c:06d}.npz")

    def __call__(self, c: int, index: np.ndarray, paths: np.ndarray, xform: np.ndarray):
        final = self.path_of(c)
        tmp = final + ".tmp.npz"
        np.savez(tmp, index=index, paths=paths, xform=xform)
        os.replace(tmp, final)


class _Lane:
    def __init__(self, links, device, cfg: StreamConfig, keep_status: int, x0_dtype=None):
        import torch
        dev = torch.device("cuda", device)
        CH, J, T, cap = cfg.chunk, cfg.J, cfg.T, cfg.cap
        self.ctx = links.Context(device)
        self.stream = torch.cuda.Stream(device=dev)   # default priority
        self.batch = links.DeviceBatch(torch.empty(CH, dtype=torch.uint8, device=dev),
                                       torch.empty((CH, J), dtype=torch.int32, device=dev),
                                       torch.empty(CH, dtype=torch.int32, device=dev),
                                       torch.empty((CH, 2), dtype=torch.uint8, device=dev),
                                       torch.empty((CH, J, 2), dtype=x0_dtype or torch.float64, device=dev))
        self.out = {"status": torch.empty(CH, dtype=torch.uint8, device=dev),
                    "fail_step": torch.empty(CH, dtype=torch.int16, device=dev),
                    "esc_step": torch.empty(CH, dtype=torch.int16, device=dev),
                    "path": torch.empty((cap, T, 2), dtype=torch.float32, device=dev),
                    "path_index": torch.empty(cap, dtype=torch.int32, device=dev),
                    "n_written": torch.empty(1, dtype=torch.int32, device=dev)}
        self.norm = torch.empty((cap, T, 2), dtype=torch.float32, device=dev)
        self.xform = torch.empty((cap, 5), dtype=torch.float32, device=dev)
        self.h_path = torch.empty((cap, T, 2), dtype=torch.float32).pin_memory()
        self.h_index = torch.empty(cap, dtype=torch.int32).pin_memory()
        self.h_xform = torch.empty((cap, 5), dtype=torch.float32).pin_memory()
        self.h_count = torch.empty(1, dtype=torch.int32).pin_memory()
        m = min(keep_status, CH)
        self.h_status = torch.empty(m, dtype=torch.uint8).pin_memory()
        self.h_fail = torch.empty(m, dtype=torch.int16).pin_memory()
        self.chunk = -1           # the chunk being simulated
        self.computed = None      # event after its simulation (count copied)


@dataclass
class _Copied:
    """A chunk whose outputs are on their way to the lane's pinned buffers."""
    c: int
    k: int
    event: object
    lane: _Lane


class Streamer:
    """Runs a stream of chunks (see the module docstring).

    sink(c, index, paths, xform) receives chunk c's valid candidates in ascending
    order: index int64 [k] (candidate index in the seed's sequence), paths f32
    [k, T, 2] and xform f32 [k, 5], views of pinned host buffers valid during the
    call only.  A chunk with more valid candidates than cfg.cap delivers the first
    cap of them and counts the rest as dropped.  With keep_status = m > 0,
    inspect(c, status, fail_step) also receives the statuses and failure steps of
    the chunk's candidates 0, s, 2s, ... (s = status_stride), the first m of them
    (views, valid during the call).
    """

    def __init__(self, cfg: StreamConfig, device: int = 0, tuning: Optional[dict] = None, keep_status: int = 0,
                 status_stride: int = 1, host=None, x0_f32: bool = False):
        """host: a batch in host memory (numpy fields n, adj, fixed, motor, x0 as
        gen.Batch) whose row i is the stream's candidate i, at least chunks x chunk
        rows; None: candidates generated on the device.  x0_f32: host positions
        cross PCIe in single precision (they must be exact in it)."""
        import torch
        from . import links
        if cfg.chunk <= 0 or cfg.chunks < 0 or cfg.cap <= 0:
            raise ValueError("chunk and cap must be positive, chunks non-negative")
        self.L = links
        self.cfg = cfg
        if status_stride < 1:
            raise ValueError("status_stride must be positive")
        self.stride = status_stride
        self.keep = max(0, min(keep_status, -(-cfg.chunk // status_stride)))
        self.h_in = None
        x0_dtype = None
        if host is not None:
            rows = cfg.chunks * cfg.chunk
            if host.B < rows or host.J != cfg.J:
                raise ValueError(f"the host batch needs {rows} rows of stride {cfg.J}")
            x0 = host.x0[:rows]
            if x0_f32:
                x0 = x0.astype(np.float32)
                if not np.array_equal(x0.astype(np.float64), host.x0[:rows]):
                    raise ValueError("host positions are not exact in single precision")
                x0_dtype = torch.float32
            pin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
            self.h_in = {"n": pin(host.n[:rows].astype(np.uint8)), "adj": pin(host.adj[:rows].view(np.int32)),
                         "fixed": pin(host.fixed[:rows].view(np.int32)), "motor": pin(host.motor[:rows].astype(np.uint8)),
                         "x0": pin(x0)}
        self.lanes = [_Lane(links, device, cfg, self.keep, x0_dtype) for _ in range(2)]
        if tuning:
            from . import tune
            for lane in self.lanes:
                tune.apply(lane.ctx, tuning)
        self.totals = {"candidates": 0, "valid": 0, "dropped": 0, "d2h_bytes": 0, "h2d_bytes": 0}

    def _compute(self, lane: _Lane, c: int):
        """Chunk c on the lane's stream, behind the copies of its previous chunk."""
        import torch
        cfg, L = self.cfg, self.L
        s = lane.stream
        with torch.cuda.stream(s):
            if self.h_in is not None:
                lo, hi = c * cfg.chunk, (c + 1) * cfg.chunk
                b = lane.batch
                for name, dst in (("n", b.n), ("adj", b.adj), ("fixed", b.fixed), ("motor", b.motor), ("x0", b.x0)):
                    dst.copy_(self.h_in[name][lo:hi], non_blocking=True)
            else:
                lane.ctx.generate_dyads(cfg.chunk, cfg.seed, first=c * cfg.chunk, J=cfg.J, n_lo=cfg.n_lo,
                                        n_hi=cfg.n_hi, paper_mode=cfg.paper_mode, rules=cfg.rules, out=lane.batch,
                                        stream=s)
            lane.ctx.simulate(lane.batch, T=cfg.T, precision=cfg.precision, write=L.WRITE_VALID, cap=cfg.cap,
                              out=lane.out, stream=s)
            lane.ctx.normalize_paths_n(lane.out["path"], lane.out["n_written"], cfg.norm, out=lane.norm,
                                       xform=lane.xform, stream=s)
            lane.h_count.copy_(lane.out["n_written"], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        lane.chunk, lane.computed = c, ev

    def _copy(self, lane: _Lane) -> _Copied:
        """Once the lane's chunk is simulated: its valid paths to pinned memory."""
        import torch
        lane.computed.synchronize()
        k = int(lane.h_count[0])
        kk = min(k, self.cfg.cap)
        with torch.cuda.stream(lane.stream):
            lane.h_path[:kk].copy_(lane.norm[:kk], non_blocking=True)
            lane.h_index[:kk].copy_(lane.out["path_index"][:kk], non_blocking=True)
            lane.h_xform[:kk].copy_(lane.xform[:kk], non_blocking=True)
            if self.keep:
                sel = slice(0, self.keep * self.stride, self.stride)
                lane.h_status.copy_(lane.out["status"][sel], non_blocking=True)
                lane.h_fail.copy_(lane.out["fail_step"][sel], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(lane.stream)
        rec = _Copied(lane.chunk, k, ev, lane)
        lane.chunk, lane.computed = -1, None
        return rec

    def _deliver(self, rec: _Copied, sink, progress: Optional[Progress], inspect):
        rec.event.synchronize()
        cfg, c, lane = self.cfg, rec.c, rec.lane
        kk = min(rec.k, cfg.cap)
        index = lane.h_index[:kk].numpy().astype(np.int64) + np.int64(c) * cfg.chunk
        if inspect is not None and self.keep:
            inspect(c, lane.h_status.numpy(), lane.h_fail.numpy())
        if sink is not None:
            sink(c, index, lane.h_path[:kk].numpy(), lane.h_xform[:kk].numpy())
        t = self.totals
        t["candidates"] += cfg.chunk
        t["valid"] += rec.k
        t["dropped"] += rec.k - kk
        t["d2h_bytes"] += kk * (cfg.T * 8 + 4 + 20)
        if self.h_in is not None:
            t["h2d_bytes"] += sum(v[:cfg.chunk].numel() * v.element_size() for v in self.h_in.values())
        if progress is not None:
            progress.save(cfg, c + 1, t)

    def run(self, sink: Optional[Callable] = None, progress_path: Optional[str] = None,
            max_chunks: Optional[int] = None, inspect: Optional[Callable] = None) -> dict:
        """Runs the stream from its resume point (chunk 0 without a progress file)
        to the end, or for at most max_chunks chunks; returns the totals of the
        chunks delivered so far (those the progress file records included), the
        next chunk and the wall time of this run."""
        import torch
        cfg = self.cfg
        progress = Progress(progress_path) if progress_path else None
        start = 0
        self.totals = {"candidates": 0, "valid": 0, "dropped": 0, "d2h_bytes": 0, "h2d_bytes": 0}
        if progress is not None:
            st = progress.load(cfg)
            if st is not None:
                start = st["next_chunk"]
                self.totals.update(st["totals"])
        end = cfg.chunks if max_chunks is None else min(cfg.chunks, start + max_chunks)
        pending = []   # chunks with copies queued, in chunk order
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c in range(start, end):
            lane = self.lanes[c % 2]
            self._compute(lane, c)
            # chunk c - 2 goes out before the lane's copies of chunk c (queued at the
            # next iteration) rewrite its pinned buffers; its own copies ran before
            # chunk c on the lane's stream
            while pending and pending[0].c <= c - 2:
                self._deliver(pending.pop(0), sink, progress, inspect)
            prev = self.lanes[(c + 1) % 2]
            if prev.computed is not None:   # chunk c - 1: copies overlap chunk c's simulation
                pending.append(self._copy(prev))
        for lane in sorted((l for l in self.lanes if l.computed is not None), key=lambda l: l.chunk):
            pending.append(self._copy(lane))
        while pending:
            self._deliver(pending.pop(0), sink, progress, inspect)
        torch.cuda.synchronize()
        return dict(self.totals, next_chunk=end, wall_s=time.perf_counter() - t0)
