"""Parity of the retrieval kernels (links_chamfer, links_chamfer_search) with the
FP64 oracle of oracle/retrieval.py.

Bars:
* distances: |gpu - oracle| <= (T + 16) 2^-24 oracle + 1e-9 for every pair.  The
  kernel rounds each squared distance at most three times (difference, product,
  fused add), the square root once, and sums at most T/8 + 6 terms per partial
  sum, so every term carries a relative error below (T/8 + 9) 2^-24;
* searches: the returned positions equal the oracle's where the answer is unique
  under that tolerance (no oracle distance within it of the cut-off or of the
  distance at a rank boundary), which the tests check before comparing; the
  returned distances meet the distance bar.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import retrieval as R
from paper_2208_14567_amd import gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_14567_amd import links
    return links


@pytest.fixture(scope="module")
def ctx(L):
    return L.Context(0)


def _tol(d, T):
    return (T + 16) * U * np.abs(d) + 1e-9


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def _coupler_bank(B, seed, T):
    """Curated DIAMETER-normalised coupler paths (circles and arcs removed, as in
    the paper's curated set) of the valid candidates of a seeded dyad_6_20 batch,
    all computed by the oracle."""
    b = gen.workload("dyad_6_20", B=B, seed=seed)
    r = oracle.simulate(b, T=T, path=True, nthreads=8)
    ok = np.nonzero(r["status"] == oracle.VALID)[0]
    out, _ = oracle.normalize_paths(r["path"][ok], mode=oracle.NORM_DIAMETER)
    flags = oracle.curate(b, out, cand=ok)["flags"]
    return out[flags == 0].astype(np.float32)


def _check_dist(got, queries, bank, T):
    for qi in range(len(queries)):
        want = R.chamfer_bank(queries[qi], bank)
        fin = np.isfinite(want)
        assert np.array_equal(np.isfinite(got[qi]), fin)
        err = np.abs(got[qi][fin].astype(np.float64) - want[fin])
        bad = err > _tol(want[fin], T)
        assert not bad.any(), f"query {qi}: {bad.sum()} pairs off, worst {err.max():.3e}"


@pytest.mark.parametrize("T", [200, 50, 100, 37, 1, 8, 64, 256, 250])
def test_distance_matrix_synthetic(ctx, T):
    _say(f"[chamfer] synthetic T={T}")
    base = gen.closed_curves(300, T, seed=T)
    bank = np.concatenate([base, gen.near_copies(base[:20], 3, 0.003, seed=T + 1)])
    queries = np.concatenate([base[:3], gen.closed_curves(2, T, seed=1000 + T)])
    got = ctx.chamfer(_dev(bank), _dev(queries)).cpu().numpy()
    _check_dist(got, queries, bank, T)


def test_distance_matrix_coupler_paths(ctx):
    _say("[chamfer] coupler paths T=200")
    bank = _coupler_bank(30000, 21, 200)
    queries = _coupler_bank(800, 22, 200)[:4]
    assert len(bank) > 200 and len(queries) == 4
    got = ctx.chamfer(_dev(bank), _dev(queries)).cpu().numpy()
    _check_dist(got, queries, bank, 200)


def test_non_finite_paths(ctx):
    T = 24
    bank = gen.closed_curves(6, T, seed=3)
    bank[1, 4, 0] = np.nan
    bank[2, 7, 1] = np.inf
    bank[3, 0, 0] = -np.inf
    q = bank[[0, 4]].copy()
    got = ctx.chamfer(_dev(bank), _dev(q)).cpu().numpy()
    assert np.isnan(got[:, 1:4]).all()
    _check_dist(got, q, bank, T)
    q[1, 2, 1] = np.nan
    got = ctx.chamfer(_dev(bank), _dev(q)).cpu().numpy()
    assert np.isnan(got[1]).all() and np.isfinite(got[0, [0, 4, 5]]).all()


def _unique(want, k, cutoff, order, T):
    """True when the oracle's answer cannot change within the distance bar."""
    tol = _tol(want, T)
    fin = np.isfinite(want)
    if (fin & (np.abs(want - cutoff) <= tol)).any():
        return False
    if order == R.BEST:
        s = np.sort(want[fin & (want < cutoff)])
        if len(s) > k and s[k] - s[k - 1] <= 2 * _tol(s[k], T):
            return False
        if len(s) > 1 and (np.diff(s[:k + 1]) <= 2 * _tol(s[1:k + 1], T)).any():
            return False
    return True


def _check_search(ctx, L, bank, queries, k, cutoff, order, T):
    idx, dist = ctx.chamfer_search(_dev(bank), _dev(queries), k=k, cutoff=cutoff,
                                   order=L.SEARCH_FIRST if order == R.FIRST else L.SEARCH_BEST)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    for qi in range(len(queries)):
        want = R.chamfer_bank(queries[qi], bank)
        assert _unique(want, k, cutoff, order, T), "test data must have a unique answer"
        widx, wd = R.select(want, k, cutoff, order)
        assert list(idx[qi]) == list(widx), f"query {qi}: {idx[qi]} vs {widx}"
        have = widx >= 0
        assert np.isnan(dist[qi][~have]).all()
        assert (np.abs(dist[qi][have] - wd[have]) <= _tol(wd[have], T)).all()
    return idx


def _planted_bank(P, T, seed, queries, pos, sigma):
    bank = gen.closed_curves(P, T, seed=seed)
    near = gen.near_copies(queries, len(pos[0]), sigma, seed=seed + 1)
    for qi, ps in enumerate(pos):
        bank[ps] = near[qi * len(ps):(qi + 1) * len(ps)]
    return bank


@pytest.mark.parametrize("order", [R.FIRST, R.BEST])
@pytest.mark.parametrize("T", [200, 50])
def test_search_planted(ctx, L, order, T):
    _say(f"[search] planted order={order} T={T}")
    rng = np.random.default_rng(T + order)
    queries = gen.closed_curves(3, T, seed=500 + T)
    P = 20000
    pos = [sorted(rng.choice(P, 6, replace=False)) for _ in range(3)]
    bank = _planted_bank(P, T, 40 + T, queries, pos, 0.004)
    idx = _check_search(ctx, L, bank, queries, 3, R.CUTOFF, order, T)
    if order == R.FIRST:
        assert [list(i) for i in idx] == [p[:3] for p in pos]


def test_search_top_k_without_cutoff(ctx, L):
    _say("[search] plain top 16")
    T = 64
    bank = gen.closed_curves(5000, T, seed=77)
    queries = gen.closed_curves(2, T, seed=78)
    _check_search(ctx, L, bank, queries, 16, float("inf"), R.BEST, T)


def test_search_fewer_matches_than_k(ctx, L):
    T = 40
    queries = gen.closed_curves(2, T, seed=90)
    bank = _planted_bank(3000, T, 91, queries, [[5, 2900], [17, 18]], 0.003)
    for order in (R.FIRST, R.BEST):
        idx = _check_search(ctx, L, bank, queries, 5, R.CUTOFF, order, T)
        assert (idx[:, 2:] == -1).all()


def test_search_coupler_paths(ctx, L):
    _say("[search] coupler paths")
    bank = _coupler_bank(16000, 31, 200)
    queries = _coupler_bank(800, 32, 200)[:3]
    assert len(queries) == 3
    # cut-off at a gap of the first query's distances so that the answer is unique
    d = np.sort(R.chamfer_bank(queries[0], bank))
    cut = float(d[40] + d[41]) / 2
    _check_search(ctx, L, bank, queries[:1], 3, cut, R.FIRST, 200)
    _check_search(ctx, L, bank, queries, 5, float("inf"), R.BEST, 200)


def test_search_edges(ctx, L):
    T = 16
    bank = gen.closed_curves(10, T, seed=5)
    q = bank[:2].copy()
    idx, dist = ctx.chamfer_search(_dev(bank[:0]), _dev(q), k=2, cutoff=0.03)
    assert (idx.cpu().numpy() == -1).all() and np.isnan(dist.cpu().numpy()).all()
    idx, _ = ctx.chamfer_search(_dev(bank), _dev(q[:0]), k=2)
    assert idx.shape == (0, 2)
    idx, _ = ctx.chamfer_search(_dev(bank), _dev(q), k=1, cutoff=1e-9, order=L.SEARCH_FIRST)
    assert list(idx.cpu().numpy()[:, 0]) == [0, 1]  # zero distance to itself
    for bad in (dict(k=0), dict(k=17), dict(cutoff=float("nan")), dict(order=2)):
        with pytest.raises(L.LinksError):
            ctx.chamfer_search(_dev(bank), _dev(q), **{**dict(k=2, cutoff=0.03, order=0), **bad})
    with pytest.raises(L.LinksError):
        ctx.chamfer(_dev(gen.closed_curves(2, 257, seed=1)), _dev(gen.closed_curves(1, 257, seed=2)))


def test_full_size_bank_sampled(ctx, L):
    """400,000 bank paths of 200 points with planted near copies: sampled
    distances against the oracle, and both searches return the planted paths."""
    T, P = 200, 400_000
    _say(f"[search] full size P={P}")
    rng = np.random.default_rng(9)
    queries = gen.closed_curves(3, T, seed=901)
    pos = [sorted(rng.choice(P, 4, replace=False)) for _ in range(3)]
    parts = [gen.closed_curves(50_000, T, seed=902 + i) for i in range(P // 50_000)]
    bank = np.concatenate(parts)
    near = gen.near_copies(queries, 4, 0.004, seed=903)
    for qi, ps in enumerate(pos):
        bank[ps] = near[qi * 4:(qi + 1) * 4]
    bd, qd = _dev(bank), _dev(queries)
    got = ctx.chamfer(bd, qd).cpu().numpy()
    sample = np.concatenate([rng.choice(P, 1500, replace=False), np.concatenate(pos)])
    for qi in range(3):
        want = R.chamfer_bank(queries[qi], bank[sample])
        assert (np.abs(got[qi, sample] - want) <= _tol(want, T)).all()
    # every path under the cut-off is a planted one (a property of the whole matrix)
    for qi in range(3):
        assert set(np.flatnonzero(got[qi] < R.CUTOFF)) == set(pos[qi])
    idx, dist = ctx.chamfer_search(bd, qd, k=3, cutoff=R.CUTOFF, order=L.SEARCH_FIRST)
    assert [list(i) for i in idx.cpu().numpy()] == [p[:3] for p in pos]
    idx, dist = ctx.chamfer_search(bd, qd, k=4, cutoff=R.CUTOFF, order=L.SEARCH_BEST)
    for qi in range(3):
        i = idx.cpu().numpy()[qi]
        assert sorted(i) == list(pos[qi])
        want = R.chamfer_bank(queries[qi], bank[i])
        assert (np.abs(dist.cpu().numpy()[qi] - want) <= _tol(want, T)).all()
        assert (np.diff(dist.cpu().numpy()[qi]) >= 0).all()
