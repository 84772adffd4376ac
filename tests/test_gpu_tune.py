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
