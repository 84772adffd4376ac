"""Autotuner of the simulation launch parameters.

The persistent passes have a handful of knobs whose best values depend on the
workload (batch size, joint-count mix, step count) and the device:

  waves32     wavefronts per workgroup of the FP32 pass (LDS sharing, occupancy)
  refill_min  idle lanes a wave of the FP32 pass waits for before refilling
  chunk       list items a wave claims with one atomic (guided down near the end)
  spread      FP32 waves start spread over the solve-order buckets or all at the top
  refill64    refill threshold of the FP64 passes
  deesc       FP64 steps after a hand-over before a candidate returns to FP32
  drain32     once the work list is exhausted, FP32 waves with fewer active lanes
              than this hand their candidates to the parallel-in-time pass (0: never)
  sort_esc    the FP64 hand-over pass takes its queue ordered by hand-over step
  wave64      FP64 passes with one candidate per wave and its positions in
              registers: 2 the path pass (whole rows, 63 steps per round), 6 also
              the FP64 decision pass of FP64 precision (0: none)

`autotune` runs the real pass sequence on the caller's batch, timing each
candidate setting with the library's own HIP events, and searches coordinate by
coordinate (each knob over its values with the others fixed, repeated until no
knob improves).  Results are cached in a JSON file keyed by device, joint stride,
batch-size class, step count and precision, so a later call with a similar
workload reuses them without measuring.
"""
from __future__ import annotations

import json
import math
import os
import tempfile
from typing import Callable, Dict, List, Optional

SPACE: Dict[str, List[int]] = {
    "waves32": [1, 2, 4],
    "refill_min": [8, 16, 32, 48],
    "chunk": [32, 64, 128, 256],
    "spread": [1, 0],
    "refill64": [8, 32],
    "deesc": [0, 8],
    "drain32": [0, 4, 12, 32],
    "sort_esc": [0, 1],
    "wave64": [0, 2],
}

DEFAULTS: Dict[str, int] = {"waves32": 4, "refill_min": 32, "chunk": 128, "spread": 1, "refill64": 32, "deesc": 0,
                            "drain32": 0, "sort_esc": 0, "wave64": 0}


def cache_path() -> str:
    p = os.environ.get("LINKS_TUNE_CACHE")
    if p:
        return p
    home = os.path.expanduser("~")
    base = os.path.join(home, ".cache") if os.access(home, os.W_OK) else tempfile.gettempdir()
    return os.path.join(base, "links_tune.json")


def cache_key(device_name: str, J: int, B: int, T: int, precision: int) -> str:
    bclass = 0 if B <= 0 else int(round(math.log2(B)))
    return f"{device_name}|J={J}|B=2^{bclass}|T={T}|p={precision}"


def coordinate_search(measure: Callable[[Dict[str, int]], float], space: Dict[str, List[int]],
                      start: Dict[str, int], rounds: int = 2) -> (Dict[str, int], float, int):
    """Minimises measure(config) one knob at a time.  Returns (best config, its
    time, number of measurements)."""
    best = dict(start)
    best_t = measure(best)
    n = 1
    for _ in range(rounds):
        improved = False
        for k, values in space.items():
            for v in values:
                if v == best[k]:
                    continue
                cfg = dict(best)
                cfg[k] = v
                t = measure(cfg)
                n += 1
                if t < best_t:
                    best, best_t, improved = cfg, t, True
        if not improved:
            break
    return best, best_t, n


def apply(ctx, cfg: Dict[str, int]):
    cur = ctx.get_tuning()
    ctx.set_tuning(cfg.get("waves32", cur["waves32"]), cfg.get("refill_min", cur["refill_min"]), cur["waves64"])
    for k in ("chunk", "spread", "refill64", "deesc", "drain32", "sort_esc", "wave64"):
        if k in cfg:
            ctx.set_option(k, cfg[k])


def current(ctx) -> Dict[str, int]:
    return {k: ctx.get_option(k) for k in SPACE}


def autotune(ctx, batch, T: int = 200, precision: int = 0, space: Optional[Dict[str, List[int]]] = None,
             reps: int = 2, use_cache: bool = True, path: Optional[str] = None, write: int = 0,
             cap: Optional[int] = None) -> dict:
    """Tunes `ctx` for `batch` (a DeviceBatch) and leaves the best setting applied.
    Each setting is timed on the call the caller will make: the same precision,
    write mode and row capacity.  Returns {"config", "ms", "measurements", "cached"}."""
    import torch
    space = space or SPACE
    dev = batch.n.device
    name = torch.cuda.get_device_name(dev)
    key = cache_key(name, batch.J, batch.B, T, precision) + f"|w={write}"
    path = path or cache_path()
    table = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
    if use_cache and key in table:
        cfg = {k: int(v) for k, v in table[key]["config"].items()}
        apply(ctx, cfg)
        return {"config": cfg, "ms": table[key]["ms"], "measurements": 0, "cached": True, "key": key}

    kw = dict(T=T, precision=precision, write=write, cap=cap)
    out = ctx.simulate(batch, **kw)     # workspace and tables outside the timing

    def measure(cfg):
        apply(ctx, cfg)
        ctx.simulate(batch, out=out, **kw)
        ctx.profile(True)
        tot = []
        for _ in range(reps):
            ctx.simulate(batch, out=out, **kw)
            tot.append(sum(ctx.last_timings().values()))
        ctx.profile(False)
        return min(tot)

    start = current(ctx)
    best, best_ms, n = coordinate_search(measure, space, start)
    apply(ctx, best)
    if use_cache:
        table[key] = {"config": best, "ms": best_ms}
        try:
            os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
            tmp = path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, path)
        except OSError:
            pass
    return {"config": best, "ms": best_ms, "measurements": n, "cached": False, "key": key}
