"""The serving loop on the GPU.  links_gather moves bytes only, so it is checked
bit for bit against a plain PyTorch reference of the block layout.  Every
request's results are the same whether it is simulated alone (one links_simulate
call over just its candidates, at its own stride) or in the mix (gathered with
other requests of other strides into ticks replayed from graphs, split across
ticks and lanes, its block placed around the ring end, admitted while other ticks
run).  The bar is bit-exact equality: each kernel computes per candidate,
independently of its neighbours, row and stride."""
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


def _narrow(host, Jr):
    """The candidates of a host batch with at most Jr joints, stored at stride Jr."""
    idx = np.nonzero(host.n <= Jr)[0]
    b = host.take(idx)
    return gen.Batch(b.n, np.ascontiguousarray(b.adj[:, :Jr]), b.fixed, b.motor, np.ascontiguousarray(b.x0[:, :Jr]))


def _alone(L, ctx, b, T, **kw):
    r = ctx.simulate(b, T=T, write=L.WRITE_VALID, cap=b.B, **kw)
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


def test_gather_bytes(L):
    from paper_2208_14567_amd import serve
    _say("[serve] gather against the block layout")
    ctx = L.Context(0)
    wide = gen.workload("dyad_4_20", 3000, seed=11)
    reqs = [L.to_device(wide.take(np.arange(0, 700))), L.to_device(_narrow(wide, 8).take(np.arange(0, 333))),
            L.to_device(wide.take(np.arange(700, 701))), L.to_device(_narrow(wide, 5).take(np.arange(0, 90)))]
    # blocks one after another in a byte buffer, each at a 16-byte multiple
    starts, total = [], 48
    for b in reqs:
        starts.append(total)
        total += serve.block_layout(b.B, b.J)[1]
    buf = torch.full((total,), 0xAB, dtype=torch.uint8, device="cuda")
    for b, s in zip(reqs, starts):
        serve._write_block(buf, s, b, serve.block_layout(b.B, b.J)[0])
    # candidate 5 of the stride-8 request claims 11 joints: malformed at its stride
    off1 = serve.block_layout(reqs[1].B, reqs[1].J)[0]
    buf[starts[1] + off1["n"] + 5] = 11
    # pieces: a tail, a whole request, a one-candidate request, a head, and one bad piece (J > out J)
    J, rows = 20, 1400
    plan = [(0, 650, 50), (1, 0, 333), (2, 0, 1), (3, 0, 60), (0, 0, 10)]
    pieces = np.zeros(len(plan), L.PIECE_DTYPE)
    dst = 0
    for p, (ri, first, take) in enumerate(plan):
        pieces[p] = (starts[ri], dst, first, reqs[ri].B, reqs[ri].J if p < len(plan) - 1 else 21)
        dst += take
    count = dst
    pd = torch.from_numpy(pieces.view(np.uint8)).cuda()
    out = L.DeviceBatch(torch.full((rows,), 77, dtype=torch.uint8, device="cuda"),
                        torch.full((rows, J), -1, dtype=torch.int32, device="cuda"),
                        torch.full((rows,), -1, dtype=torch.int32, device="cuda"),
                        torch.full((rows, 2), 9, dtype=torch.uint8, device="cuda"),
                        torch.full((rows, J, 2), 3.5, dtype=torch.float64, device="cuda"))
    ctx.gather(buf, pd, len(plan), count, out)
    torch.cuda.synchronize()
    dst = 0
    for p, (ri, first, take) in enumerate(plan):
        b = reqs[ri]
        sl = slice(dst, dst + take)
        if p == len(plan) - 1:
            assert out.n[sl].eq(0).all()          # the malformed piece's rows are left empty
        else:
            Jr = b.J
            want = b.n[first:first + take].clone()
            if ri == 1:
                want[5 - first] = 0                # more joints than its stride: no joints
            assert torch.equal(out.n[sl], want)
            assert torch.equal(out.fixed[sl], b.fixed[first:first + take])
            assert torch.equal(out.motor[sl], b.motor[first:first + take])
            assert torch.equal(out.adj[sl, :Jr], b.adj[first:first + take])
            assert out.adj[sl, Jr:].eq(0).all()
            assert torch.equal(out.x0[sl, :Jr], b.x0[first:first + take])
            assert out.x0[sl, Jr:].eq(0).all()
        dst += take
    assert out.n[count:].eq(0).all()                # rows past the tick: no joints
    assert out.fixed[count:].eq(-1).all()           # and nothing else written there
    with pytest.raises(L.LinksError):
        ctx.gather(buf, pd, len(plan), rows + 1, out)


def test_same_alone_and_in_the_mix(L):
    from paper_2208_14567_amd import serve
    T = 200
    host = gen.workload("dyad_4_20", 60000, seed=4)
    pool = L.to_device(host)
    narrow = L.to_device(_narrow(host, 9))
    ctx = L.Context(0)
    rng = np.random.default_rng(7)
    sizes = [int(s) for s in rng.integers(1, 9000, 14)] + [0, 1, 12000]
    batches = []
    for i, s in enumerate(sizes):
        src = narrow if i % 4 == 1 else pool       # every fourth request at stride 9
        o = int(rng.integers(0, src.B - s)) if s < src.B else 0
        batches.append(src.slice(o, o + s))
    refs = [_alone(L, ctx, b, T) for b in batches]
    _say(f"[serve] {len(sizes)} requests, {sum(sizes)} candidates")

    # small ring and ticks: requests share ticks, split across ticks, wait for ring
    # room and are placed around the ring end; some arrive packed
    srv = serve.Server(capacity=6 << 20, tick_max=5000, J=20, T=T, min_class=512)
    srv.warm()
    assert srv.classes == [5000, 2500, 1250, 625, 313]
    reqs = []
    for i, b in enumerate(batches):
        reqs.append(srv.submit(serve.pack(b) if i % 3 == 2 else b))
        if i % 3 == 0:
            srv.poll()          # later requests arrive while ticks are on the device
    srv.drain()
    torch.cuda.synchronize()
    assert srv.ticks >= 10 and srv.ring.head > srv.capacity
    for r, ref in zip(reqs, refs):
        assert r.finished_at >= r.arrival
        _check(r, ref)
    _say(f"  mixed: {srv.ticks} ticks, all {len(reqs)} requests equal to their solo runs")

    # the largest request alone in a fresh server
    solo = serve.Server(capacity=8 << 20, tick_max=5000, J=20, T=T, min_class=512)
    solo.warm()
    r = solo.submit(batches[-1])
    solo.drain()
    torch.cuda.synchronize()
    _check(r, refs[-1])
    srv.close()
    solo.close()


def test_poisson_stream_small(L):
    from paper_2208_14567_amd import serve
    pool = L.to_device(gen.workload("dyad_4_20", 50000, seed=4))
    sizes = serve.request_sizes(60, seed=5, hi=20000)
    offs = np.random.default_rng(5).integers(0, 50000 - sizes)
    arr = serve.poisson_arrivals(60, rate=400.0, seed=5)
    srv = serve.Server(capacity=32 << 20, tick_max=1 << 14, J=20, T=200)
    srv.warm()
    reqs = serve.run_stream(srv, [pool.slice(int(o), int(o + s)) for o, s in zip(offs, sizes)], arr)
    torch.cuda.synchronize()
    st = serve.latency_stats(reqs)
    _say(f"[serve] poisson: {st}")
    assert st["requests"] == 60 and st["p99_ms"] >= st["p50_ms"] > 0
    assert all(r.done == r.size for r in reqs)
    ctx = L.Context(0)
    for j in (0, 17, 59):
        _check(reqs[j], _alone(L, ctx, pool.slice(int(offs[j]), int(offs[j] + sizes[j])), 200))
    srv.close()


def test_fp64_and_orientation_ticks(L):
    """Ticks replayed in plain FP64 with the starting-orientation rule equal solo
    calls with the same options."""
    from paper_2208_14567_amd import serve
    T = 120
    host = gen.workload("dyad_4_20", 30000, seed=9)
    pool = L.to_device(host)
    narrow = L.to_device(_narrow(host, 7))
    ctx = L.Context(0)
    kw = dict(precision=L.FP64, branch=L.BRANCH_ORIENTATION)
    batches = [pool.slice(0, 4000), narrow.slice(0, 1500), pool.slice(4000, 4001), pool.slice(5000, 11000),
               narrow.slice(1500, 1600)]
    refs = [_alone(L, ctx, b, T, **kw) for b in batches]
    srv = serve.Server(capacity=4 << 20, tick_max=3000, J=20, T=T, min_class=256, **kw)
    srv.warm()
    reqs = [srv.submit(b) for b in batches]
    srv.drain()
    torch.cuda.synchronize()
    assert srv.ticks >= 4
    for r, ref in zip(reqs, refs):
        _check(r, ref)
    srv.close()
    _say(f"[serve] FP64, orientation rule: {srv.ticks} ticks equal to the solo calls")
