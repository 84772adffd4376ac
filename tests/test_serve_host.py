"""Host-side bookkeeping of the serving loop (no GPU): the FIFO byte ring, the
request block layout, tick size classes and the split of the queue into ticks,
against brute force."""
import numpy as np
import pytest

from paper_2208_14567_amd.serve import (RingAlloc, block_layout, class_of, plan_tick, poisson_arrivals,
                                        request_sizes, size_classes)


def test_ring_fifo_and_deferred_free():
    r = RingAlloc(10)
    a = r.alloc(4)
    b = r.alloc(5)
    assert (a, b) == (0, 4) and r.used == 9
    assert r.alloc(2) is None            # only one unit left
    r.free(b)                            # freed out of order: held until a is freed
    assert r.used == 9
    r.free(a)
    assert r.used == 0 and r.tail == 9
    c = r.alloc(10)                      # wraps: coordinates 9..18 -> units 9, 0..8
    assert c == 9 and r.used == 10
    with pytest.raises(KeyError):
        r.free(123)
    with pytest.raises(ValueError):
        r.alloc(11)


def test_ring_contiguous_skips_the_end():
    r = RingAlloc(10)
    a = r.alloc_contiguous(6)
    assert a == 0
    assert r.alloc_contiguous(5) is None   # 4 units left at the end, none at the start yet
    b = r.alloc_contiguous(4)
    assert b == 6
    r.free(a)
    c = r.alloc_contiguous(5)              # nothing left at the end: starts the next lap
    assert c == 10 and c % 10 == 0
    r.free(b)
    r.free(c)
    assert r.used == 0
    d = r.alloc_contiguous(10)             # empty ring: any size up to capacity fits
    assert d % 10 == 0


def test_ring_random_against_occupancy_model():
    rng = np.random.default_rng(0)
    C = 97
    for contiguous in (False, True):
        r = RingAlloc(C)
        live = []
        for _ in range(3000):
            if live and rng.random() < 0.45:
                s = live.pop(int(rng.integers(len(live))))
                r.free(s[0])
            else:
                n = int(rng.integers(0, 30))
                st = r.alloc_contiguous(n) if contiguous else r.alloc(n)
                if st is None:
                    if contiguous:
                        assert live   # an empty ring always takes a block that fits
                    else:
                        assert r.used + n > C
                else:
                    live.append((st, n))
                    if contiguous:
                        assert st % C + n <= C   # never across the ring end
            # units of live allocations never collide
            occ = np.zeros(C, int)
            for s, n in live:
                for k in range(s, s + n):
                    occ[k % C] += 1
            assert occ.max(initial=0) <= 1
            assert r.used >= sum(n for _, n in live)


def test_block_layout():
    for size in (0, 1, 3, 17, 1000):
        for J in (1, 5, 20, 32):
            off, nb = block_layout(size, J)
            ends = {"x0": size * J * 16, "adj": size * J * 4, "fixed": size * 4, "n": size, "motor": size * 2}
            order = ["x0", "adj", "fixed", "n", "motor"]
            for k in order:
                assert off[k] % 16 == 0
            for k0, k1 in zip(order, order[1:]):
                assert off[k0] + ends[k0] <= off[k1] < off[k0] + ends[k0] + 16
            assert off["motor"] + ends["motor"] <= nb < off["motor"] + ends["motor"] + 16 and nb % 16 == 0
            assert nb <= size * (20 * J + 7) + 5 * 15 + 15


def test_size_classes_and_class_of():
    cl = size_classes(1 << 19, 4096)
    assert cl[0] == 1 << 19 and cl[-1] == 4096 and len(cl) == 8
    assert all(a == 2 * b for a, b in zip(cl, cl[1:]))
    assert size_classes(5000, 4096) == [5000, 2500]
    for count in (1, 4095, 4096, 4097, 70000, 1 << 19):
        c = class_of(count, cl)
        assert c >= count and (c == cl[-1] or c // 2 < count)


def test_plan_tick_brute_force():
    rng = np.random.default_rng(3)
    for _ in range(300):
        nq = int(rng.integers(0, 8))
        sizes = rng.integers(1, 40, nq)
        firsts = [int(rng.integers(0, s)) for s in sizes]
        q = [(i, f, int(s)) for i, (f, s) in enumerate(zip(firsts, sizes))]
        tick_max = int(rng.integers(1, 80))
        maxp = int(rng.integers(1, 6))
        shares, whole = plan_tick(q, tick_max, maxp)
        # brute force: walk the queue's candidates one by one
        rows, want, done = 0, [], 0
        for rid, f, s in q:
            if rows == tick_max or len(want) == maxp:
                break
            k = min(s - f, tick_max - rows)
            want.append((rid, f, k, rows))
            rows += k
            if f + k < s:
                break
            done += 1
        assert shares == want and whole == done
        assert sum(x[2] for x in shares) <= tick_max


def test_request_mix_shapes():
    s = request_sizes(20000, seed=4)
    assert s.min() >= 1 and s.max() <= 200_000
    # log-uniform: about as many requests in [1, 447) as in [447, 200k]
    assert 0.4 < (s < 447).mean() < 0.6
    a = poisson_arrivals(20000, rate=1000.0, seed=4)
    assert np.all(np.diff(a) > 0)
    assert abs(np.diff(a).mean() - 1e-3) < 5e-5


def test_request_parts_in_request_order():
    torch = pytest.importorskip("torch")
    from paper_2208_14567_amd.serve import Part, Request
    r = Request(0, 100, 20, 0.0)
    # shares of two ticks, the later share finished first
    r.parts.append(Part(60, torch.full((40,), 2, dtype=torch.uint8), torch.zeros(40, dtype=torch.int16),
                        torch.zeros(40, dtype=torch.int16), np.array([61, 70]), torch.full((2, 3, 2), 2.0)))
    r.parts.append(Part(0, torch.full((60,), 1, dtype=torch.uint8), torch.zeros(60, dtype=torch.int16),
                        torch.zeros(60, dtype=torch.int16), np.array([5, 9, 30]), torch.full((3, 3, 2), 1.0)))
    idx, paths = r.valid()
    assert idx.tolist() == [5, 9, 30, 61, 70]
    assert paths[:3].eq(1.0).all() and paths[3:].eq(2.0).all()
    st = r.status
    assert st.shape[0] == 100 and st[:60].eq(1).all() and st[60:].eq(2).all()
