"""Host-side bookkeeping of the serving loop (no GPU): the FIFO slot ring, tick
ranges and the split of a tick among requests, against brute force."""
import numpy as np
import pytest

from paper_2208_14567_amd.serve import RingAlloc, overlaps, poisson_arrivals, request_sizes, tick_range


def test_ring_fifo_and_deferred_free():
    r = RingAlloc(10)
    a = r.alloc(4)
    b = r.alloc(5)
    assert (a, b) == (0, 4) and r.used == 9
    assert r.alloc(2) is None            # only one slot left
    r.free(b)                            # freed out of order: held until a is freed
    assert r.used == 9
    r.free(a)
    assert r.used == 0 and r.tail == 9
    c = r.alloc(10)                      # wraps: coordinates 9..18 -> slots 9, 0..8
    assert c == 9 and r.used == 10
    with pytest.raises(KeyError):
        r.free(123)
    with pytest.raises(ValueError):
        r.alloc(11)


def test_ring_random_against_occupancy_model():
    rng = np.random.default_rng(0)
    C = 97
    r = RingAlloc(C)
    live = []
    for _ in range(3000):
        if live and rng.random() < 0.45:
            s = live.pop(int(rng.integers(len(live))))
            r.free(s[0])
        else:
            n = int(rng.integers(0, 30))
            st = r.alloc(n)
            if st is None:
                assert r.used + n > C
            else:
                live.append((st, n))
        # slots of live allocations never collide
        occ = np.zeros(C, int)
        for s, n in live:
            for k in range(s, s + n):
                occ[k % C] += 1
        assert occ.max(initial=0) <= 1
        assert r.used >= sum(n for _, n in live)


def test_tick_range():
    assert tick_range(5, 5, 10, 4) == (5, 5)
    assert tick_range(5, 30, 10, 100) == (5, 10)     # stops at the ring end
    assert tick_range(10, 30, 10, 4) == (10, 14)     # tick_max
    assert tick_range(12, 13, 10, 4) == (12, 13)


def test_overlaps_brute_force():
    rng = np.random.default_rng(1)
    starts = np.cumsum(rng.integers(0, 9, 40))
    reqs = [(i, int(starts[i]), int(rng.integers(0, 9))) for i in range(40)]
    for _ in range(200):
        lo = int(rng.integers(0, starts[-1] + 10))
        hi = lo + int(rng.integers(0, 30))
        got = overlaps(lo, hi, reqs)
        want = []
        for rid, s, n in reqs:
            ks = [k for k in range(s, s + n) if lo <= k < hi]
            if ks:
                want.append((rid, ks[0] - s, ks[-1] - s + 1))
        assert got == want


def test_request_mix_shapes():
    s = request_sizes(20000, seed=4)
    assert s.min() >= 1 and s.max() <= 200_000
    # log-uniform: about as many requests in [1, 447) as in [447, 200k]
    assert 0.4 < (s < 447).mean() < 0.6
    a = poisson_arrivals(20000, rate=1000.0, seed=4)
    assert np.all(np.diff(a) > 0)
    assert abs(np.diff(a).mean() - 1e-3) < 5e-5


def test_request_pieces_in_request_order():
    torch = pytest.importorskip("torch")
    from paper_2208_14567_amd.serve import Request
    r = Request(0, 100, 0.0)
    # shares of two ticks, the later share finished first
    r.pieces.append((60, np.array([61, 70]), torch.full((2, 3, 2), 2.0)))
    r.pieces.append((0, np.array([5, 9, 30]), torch.full((3, 3, 2), 1.0)))
    idx, paths = r.valid()
    assert idx.tolist() == [5, 9, 30, 61, 70]
    assert paths[:3].eq(1.0).all() and paths[3:].eq(2.0).all()
