"""Pins of the oracle's path curation (Methodology, "Dataset Curation &
Processing"): arc flags from the four-bar's topology, the radial variance of
closed-form curves, and the reduced mechanism checked by simulating it."""
import numpy as np

import oracle
from paper_2208_14567_amd import gen
from tests import mech


def _norm(paths):
    out, _ = oracle.normalize_paths(paths, oracle.NORM_DIAMETER)
    return out


def test_fourbar_arcs_circles_and_reduction(oracle_lib):
    b = gen.workload("fourbar", 200, seed=71)
    T = 200
    for out, arc, keep in ((1, True, 0b00011), (3, True, 0b01111), (4, False, 0b11111)):
        r = oracle.simulate(b, T=T, out_joint=out, path=True)
        assert np.all(r["status"] == oracle.VALID)
        c = oracle.curate(b, _norm(r["path"]), out_joint=out)
        assert np.all(((c["flags"] & oracle.ARC) != 0) == arc)
        assert np.all(c["keep"] == keep)
        if out == 1:   # the crank tip turns on a circle about the pivot
            assert np.all(c["radial_var"] < 1e-20) and np.all(c["flags"] & oracle.CIRCLE)


def test_radial_variance_of_an_ellipse(oracle_lib):
    """An ellipse with semi-axes 1 and b0 sampled at T angles that include both
    vertices: the diameter rule takes the major axis as the longest chord, so the
    normalised points are (0.5 + cos/2, 0.5 + b0 sin/2) up to a half turn, and the
    distances from the box centre are sqrt(cos^2 + b0^2 sin^2)/2."""
    T = 200
    th = 2 * np.pi * np.arange(T) / T
    b4 = gen.workload("fourbar", 4, seed=1)
    for b0 in (1.0, 0.9, 0.5, 0.2):
        pts = np.stack([3.0 + np.cos(th), -1.0 + b0 * np.sin(th)], -1)[None]
        norm = _norm(pts)
        r = np.sqrt(np.cos(th) ** 2 + (b0 * np.sin(th)) ** 2) / 2
        want = r.var()
        c = oracle.curate(b4, norm, cand=np.array([0], np.int32), out_joint=4)
        assert abs(c["radial_var"][0] - want) <= 1e-12 + 1e-9 * want, (b0, c["radial_var"][0], want)
        assert bool(c["flags"][0] & oracle.CIRCLE) == (want < oracle.CIRCLE_VAR)


def _reduce(b, c, keep):
    """The candidate with only the joints in keep, relabelled in ascending order."""
    js = [j for j in range(int(b.n[c])) if (int(keep) >> j) & 1]
    idx = {j: i for i, j in enumerate(js)}
    J = b.J
    r = gen.empty_batch(1, J)
    r.n[0] = len(js)
    for j in js:
        r.x0[0, idx[j]] = b.x0[c, j]
        row = 0
        for k in js:
            if (int(b.adj[c, j]) >> k) & 1:
                row |= 1 << idx[k]
        r.adj[0, idx[j]] = row
        if (int(b.fixed[c]) >> j) & 1:
            r.fixed[0] |= np.uint32(1 << idx[j])
    r.motor[0] = (idx[int(b.motor[c, 0])], idx[int(b.motor[c, 1])])
    return r, idx


def test_reduced_mechanism_reproduces_the_path(oracle_lib):
    """Simulating only the kept joints gives the path joint bit-identical
    positions: its parents are never outside the kept set, so every kept joint is
    placed from the same parents, lengths and previous positions."""
    b = gen.workload("dyad_6_20", 3000, seed=72)
    T = 200
    r = oracle.simulate(b, T=T, path=True)
    valid = np.nonzero(r["status"] == oracle.VALID)[0][:60]
    assert valid.size >= 30
    order, nd, _, _ = oracle.solve_order(b.take(valid))
    c = oracle.curate(b, _norm(r["path"][valid]), cand=valid.astype(np.int32))
    reduced_some = 0
    for i, cand in enumerate(valid):
        keep = int(c["keep"][i])
        out = int(order[i, nd[i] - 1, 0])
        assert (keep >> out) & 1 and (keep & 0b11) == 0b11
        if keep != (1 << int(b.n[cand])) - 1:
            reduced_some += 1
        rb, idx = _reduce(b, cand, keep)
        rr = oracle.simulate(rb, T=T, out_joint=idx[out], path=True)
        assert rr["status"][0] == oracle.VALID
        assert np.array_equal(rr["path"][0], r["path"][cand])
    assert reduced_some > 0
