"""Replays of a recorded launch sequence (links_graph_*) against eager calls.

Every replay must reproduce the eager links_simulate outputs bit for bit: the
graph runs the same kernels with the same arguments.  Replays are interleaved
with eager work and host synchronisations, and the inputs are refilled in place
between replays.
"""
import sys

import numpy as np
import pytest

from paper_2208_14567_amd import gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_14567_amd import links
    return links


def _np(r):
    return {k: v.cpu().numpy().copy() for k, v in r.items()}


def _same(a, b, keys):
    for k in keys:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replays_match_eager(L, precision):
    _say(f"[graph] precision={precision}")
    ctx = L.Context(0)
    B, T = 6000, 200
    h1 = gen.workload("dyad_6_20", B, seed=21)
    h2 = gen.workload("dyad_6_20", B, seed=22)
    db = L.to_device(h1)
    g = ctx.graph(db, T=T, precision=precision, write=L.WRITE_VALID, cap=B)
    keys = ["status", "fail_step", "esc_step", "n_written"]

    eager_ctx = L.Context(0)
    ref1 = _np(eager_ctx.simulate(L.to_device(h1), T=T, precision=precision, write=L.WRITE_VALID, cap=B))
    ref2 = _np(eager_ctx.simulate(L.to_device(h2), T=T, precision=precision, write=L.WRITE_VALID, cap=B))

    for rep, (host, ref) in enumerate([(h1, ref1), (h1, ref1), (h2, ref2), (h1, ref1)]):
        src = L.to_device(host)
        for name in ("n", "adj", "fixed", "motor", "x0"):
            getattr(db, name).copy_(getattr(src, name))
        torch.cuda.synchronize()
        out = _np(g.launch())
        torch.cuda.synchronize()
        _same(out, ref, keys)
        k = int(ref["n_written"][0])
        assert np.array_equal(out["path_index"][:k], ref["path_index"][:k])
        assert np.array_equal(out["path"][:k], ref["path"][:k], equal_nan=True)
        # unrelated eager work on the same context between replays
        eager = _np(ctx.simulate(L.to_device(gen.workload("fourbar", 500, seed=rep)), T=T, precision=precision))
        assert eager["status"].shape == (500,)
        _say(f"  replay {rep}: {k} paths, ok")
    g.close()
    ctx.close()
    eager_ctx.close()


def test_graph_holds_workspace(L):
    ctx = L.Context(0)
    small = L.to_device(gen.workload("dyad_6_20", 1000, seed=23))
    g = ctx.graph(small, T=50)
    g.launch()
    torch.cuda.synchronize()
    big = L.to_device(gen.workload("dyad_6_20", 50000, seed=24))
    with pytest.raises(L.LinksError):
        ctx.simulate(big, T=50)       # would reallocate workspace the graph uses
    g.close()
    r = ctx.simulate(big, T=50)       # fine once the graph is gone
    torch.cuda.synchronize()
    assert r["status"].shape == (50000,)
    ctx.close()
