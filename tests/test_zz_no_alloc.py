"""links_simulate_noalloc (workspace in the device's fixed scratch array, no
allocation) against links_simulate (workspace allocated by the context): the
same kernels, so every output must be identical bit for bit.  Calls come in a
row on one context and stream, later ones smaller, so that anything a call
leaves in the shared array would show in the next one's results."""
import sys

import numpy as np
import pytest

from paper_2208_14567_amd import gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("status", "fail_step", "esc_step")


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
    return {k: v.cpu().numpy() for k, v in r.items()}


def _same(a, z, write, L, label):
    for k in KEYS:
        assert np.array_equal(a[k], z[k]), (label, k)
    if write == L.WRITE_VALID:
        n = int(a["n_written"][0])
        assert int(z["n_written"][0]) == n, label
        k = min(n, a["path_index"].shape[0])
        assert np.array_equal(a["path_index"][:k], z["path_index"][:k]), label
        assert np.array_equal(a["path"][:k], z["path"][:k], equal_nan=True), label
    elif write == L.WRITE_ALL:
        assert np.array_equal(a["path"], z["path"], equal_nan=True), label


# (workload, candidates, seed, precision, write, T, T_prefilter, x0 as float)
CALLS = [
    ("dyad_6_20", 30000, 71, 0, 2, 200, 0, False),   # near the array's size at J = 20
    ("dyad_6_20", 5000, 72, 0, 2, 200, 0, False),    # smaller: stale counters or lists would show
    ("dyad_4_20", 3000, 73, 1, 1, 200, 0, False),    # FP64, every path (side bits of the row chunks)
    ("fourbar_u", 1000, 74, 0, 1, 100, 0, True),     # another crank table, single-precision positions
    ("dyad_6_20", 8000, 75, 0, 2, 200, 50, False),   # low-fidelity screen: two passes in one call
    ("dyad_6_20", 700, 76, 0, 0, 200, 0, False),     # decisions only
]


def test_noalloc_matches_simulate(L):
    ctx = L.Context(0)
    for i, (name, B, seed, prec, write, T, Tp, f32) in enumerate(CALLS):
        _say(f"[noalloc] call {i}: {name} B={B} precision={prec} write={write} T={T} T_prefilter={Tp} x0_f32={f32}")
        b = gen.workload(name, B, seed=seed)
        db = L.to_device(b, x0_dtype=np.float32) if f32 else L.to_device(b)
        kw = dict(T=T, precision=prec, write=write, T_prefilter=Tp, cap=B if write == L.WRITE_VALID else None)
        ref = _np(ctx.simulate(db, **kw))
        got = _np(ctx.simulate_noalloc(db, **kw))
        _same(ref, got, write, L, f"call {i}")
        # and the same call again, after the allocating path ran in between
        again = _np(ctx.simulate_noalloc(db, **kw))
        _same(ref, again, write, L, f"call {i} repeated")


def test_noalloc_two_contexts_share_the_array(L):
    """Two contexts on one device use the same array, one after the other on one
    stream: each call's results are its own."""
    c1, c2 = L.Context(0), L.Context(0)
    b1 = L.to_device(gen.workload("dyad_6_20", 12000, seed=81))
    b2 = L.to_device(gen.workload("dyad_skewed", 4000, seed=82))
    r1 = _np(c1.simulate(b1, write=L.WRITE_VALID, cap=12000))
    r2 = _np(c2.simulate(b2, write=L.WRITE_VALID, cap=4000))
    g1 = _np(c1.simulate_noalloc(b1, write=L.WRITE_VALID, cap=12000))
    g2 = _np(c2.simulate_noalloc(b2, write=L.WRITE_VALID, cap=4000))
    _same(r1, g1, L.WRITE_VALID, L, "context 1")
    _same(r2, g2, L.WRITE_VALID, L, "context 2")


def test_noalloc_rejects_what_does_not_fit(L):
    """A call that needs more than the array, or more steps than its table
    holds, fails before any device work: the outputs keep what they held."""
    ctx = L.Context(0)
    b = L.to_device(gen.workload("dyad_6_20", 40000, seed=83))
    out = {"status": torch.full((40000,), 77, dtype=torch.uint8, device="cuda"),
           "fail_step": torch.full((40000,), -7, dtype=torch.int16, device="cuda"),
           "esc_step": torch.full((40000,), -7, dtype=torch.int16, device="cuda")}
    with pytest.raises(L.LinksError, match="scratch"):
        ctx.simulate_noalloc(b, out=out)
    small = L.to_device(gen.workload("dyad_6_20", 100, seed=84))
    out_s = {k: v[:100] for k, v in out.items()}
    with pytest.raises(L.LinksError, match="4096"):
        ctx.simulate_noalloc(small, T=5000, out=out_s)
    torch.cuda.synchronize()
    assert bool((out["status"] == 77).all()) and bool((out["fail_step"] == -7).all())
    # the context still works, both ways
    ref = _np(ctx.simulate(small))
    got = _np(ctx.simulate_noalloc(small))
    _same(ref, got, L.WRITE_NONE, L, "after the rejected calls")
