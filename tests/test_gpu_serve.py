"""The serving loop on the GPU: every request's results are the same whether it is
simulated alone (one links_simulate call over just its candidates) or in the mix
(sharing ticks with other requests, split across ticks and across the ring end,
admitted while other ticks run).  The bar is bit-exact equality: each kernel
computes per candidate, independently of its neighbours and slot."""
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


def _alone(L, ctx, pool, lo, hi, T):
    r = ctx.simulate(pool.slice(lo, hi), T=T, write=L.WRITE_VALID, cap=hi - lo)
    k = int(r["n_written"].cpu()[0])
    return {"status": r["status"].cpu().numpy(), "fail_step": r["fail_step"].cpu().numpy(),
            "esc_step": r["esc_step"].cpu().numpy(), "idx": r["path_index"][:k].cpu().numpy().astype(np.int64),
            "path": r["path"][:k].cpu().numpy()}


def _check(req, ref):
    assert np.array_equal(req.status.cpu().numpy(), ref["status"])
    assert np.array_equal(req.fail_step.cpu().numpy(), ref["fail_step"])
    assert np.array_equal(req.esc_step.cpu().numpy(), ref["esc_step"])
    idx, paths = req.valid()
    assert np.array_equal(idx, ref["idx"])
    if len(idx):
        assert np.array_equal(paths.cpu().numpy(), ref["path"])


def test_same_alone_and_in_the_mix(L):
    from paper_2208_14567_amd import serve
    T = 200
    pool = L.to_device(gen.workload("dyad_4_20", 60000, seed=4))
    ctx = L.Context(0)
    rng = np.random.default_rng(7)
    sizes = [int(s) for s in rng.integers(1, 9000, 14)] + [0, 1, 12000]
    offs = [int(rng.integers(0, 60000 - s)) if s < 60000 else 0 for s in sizes]
    refs = [_alone(L, ctx, pool, o, o + s, T) for o, s in zip(offs, sizes)]
    _say(f"[serve] {len(sizes)} requests, {sum(sizes)} candidates")

    # small ring and ticks: requests share ticks, split across ticks and wrap the ring
    srv = serve.Server(capacity=20000, tick_max=5000, J=20, T=T)
    reqs = []
    for i, (o, s) in enumerate(zip(offs, sizes)):
        reqs.append(srv.submit(pool.slice(o, o + s)))
        if i % 3 == 0:
            srv.poll()          # later requests arrive while ticks are on the device
    srv.drain()
    torch.cuda.synchronize()
    assert srv.ticks >= 10
    for r, ref in zip(reqs, refs):
        assert r.finished_at >= r.arrival
        _check(r, ref)
    _say(f"  mixed: {srv.ticks} ticks, all {len(reqs)} requests equal to their solo runs")

    # the same request alone in a fresh server
    big = len(sizes) - 1
    solo = serve.Server(capacity=20000, tick_max=5000, J=20, T=T)
    r = solo.submit(pool.slice(offs[big], offs[big] + sizes[big]))
    solo.drain()
    torch.cuda.synchronize()
    _check(r, refs[big])


def test_poisson_stream_small(L):
    from paper_2208_14567_amd import serve
    pool = L.to_device(gen.workload("dyad_4_20", 50000, seed=4))
    sizes = serve.request_sizes(60, seed=5, hi=20000)
    offs = np.random.default_rng(5).integers(0, 50000 - sizes)
    arr = serve.poisson_arrivals(60, rate=400.0, seed=5)
    srv = serve.Server(capacity=1 << 16, tick_max=1 << 14, J=20, T=200)
    reqs = serve.run_stream(srv, pool, sizes, offs, arr)
    torch.cuda.synchronize()
    st = serve.latency_stats(reqs)
    _say(f"[serve] poisson: {st}")
    assert st["requests"] == 60 and st["p99_ms"] >= st["p50_ms"] > 0
    assert all(r.done == r.size for r in reqs)
    ctx = L.Context(0)
    for j in (0, 17, 59):
        _check(reqs[j], _alone(L, ctx, pool, int(offs[j]), int(offs[j] + sizes[j]), 200))
