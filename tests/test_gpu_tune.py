"""Autotuner on the GPU: it applies a setting from its search space, caches it,
and the tuned launch gives the same results as the default one."""
import os
import sys

import numpy as np
import pytest

from paper_2208_14567_amd import gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_autotune_applies_and_caches(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_14567_amd import links as L, tune
    print("[tune] dyad_6_20 40000", flush=True)
    sys.stdout.flush()
    ctx = L.Context(0)
    db = L.to_device(gen.workload("dyad_6_20", 40000, seed=8))
    ref = {k: v.cpu().numpy() for k, v in ctx.simulate(db, write=L.WRITE_VALID, cap=40000).items()}
    space = {"waves32": [1, 4], "refill_min": [16, 48], "chunk": [64, 128]}
    start = tune.current(ctx)
    path = str(tmp_path / "tune.json")
    r = tune.autotune(ctx, db, space=space, path=path)
    assert not r["cached"] and r["measurements"] >= 1 and os.path.exists(path)
    for k, v in r["config"].items():
        assert v in space.get(k, []) + [start[k]]     # a searched value, or the start it kept
        assert ctx.get_option(k) == v
    got = {k: v.cpu().numpy() for k, v in ctx.simulate(db, write=L.WRITE_VALID, cap=40000).items()}
    for k in ("status", "fail_step", "esc_step", "n_written", "path_index"):
        assert np.array_equal(got[k], ref[k]), k
    n = int(ref["n_written"][0])
    assert np.array_equal(got["path"][:n], ref["path"][:n])
    ctx2 = L.Context(0)
    r2 = tune.autotune(ctx2, db, space=space, path=path)
    assert r2["cached"] and r2["config"] == r["config"]
    assert all(ctx2.get_option(k) == v for k, v in r["config"].items())


def test_pass_timings_ring():
    """Profiled calls record their pass timings without a host synchronisation;
    the ring returns the last call's timings and means over up to 64 calls."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_14567_amd import links as L
    print("[timings] dyad_6_20 20000", flush=True)
    ctx = L.Context(0)
    db = L.to_device(gen.workload("dyad_6_20", 20000, seed=9))
    ctx.simulate(db)
    ctx.profile(True)
    with pytest.raises(L.LinksError):
        ctx.mean_timings(1)                     # nothing recorded since profiling was enabled
    for _ in range(70):                         # wraps the 64-set ring
        ctx.simulate(db)
    torch.cuda.synchronize()
    last = ctx.last_timings()
    assert ctx.mean_timings(1) == last
    mean = ctx.mean_timings(64)
    assert set(mean) == set(L.TIMING_PASSES)
    assert mean["fp32_pass"] > 0 and mean["path_pass"] == 0 and mean["prep_fill"] > 0
    with pytest.raises(L.LinksError):
        ctx.mean_timings(65)
    ctx.profile(False)
