"""Pins of the retrieval oracle (chamfer distance and the two searches) against
closed forms, invariants and hand-checked answers, plus planted mistakes that
those pins must catch."""
import math
import os
import types

import numpy as np
import pytest

from oracle import retrieval as R
from paper_2208_14567_amd import gen


def _line(n, y=0.0):
    return np.stack([np.arange(n, dtype=np.float64), np.full(n, y)], axis=1)


def _circle(T, r, c=(0.0, 0.0), phase=0.0):
    th = phase + 2 * np.pi * np.arange(T) / T
    return np.stack([c[0] + r * np.cos(th), c[1] + r * np.sin(th)], axis=1)


# ---- closed forms --------------------------------------------------------------

def test_single_points(mod=R):
    # each direction contributes |a - b| once: CD = 2 |a - b| (3-4-5 triangle)
    assert mod.chamfer(np.array([[1.0, 2.0]]), np.array([[4.0, 6.0]])) == pytest.approx(10.0, abs=1e-12)


def test_collinear_subset(mod=R):
    # A = 7 points on a line, B = its two ends: from A the nearest-end distances
    # are 0,1,2,3,2,1,0 (mean 9/7); from B both distances are 0
    a, b = _line(7), _line(7)[[0, 6]]
    assert mod.chamfer(a, b) == pytest.approx(9.0 / 7.0, abs=1e-12)
    assert mod.chamfer(b, a) == pytest.approx(9.0 / 7.0, abs=1e-12)


def test_ends_lifted_off_the_line(mod=R):
    # B = the two ends moved up by 1: from A the distances are sqrt(1 + m^2) with
    # m the distance to the nearer end; from B both are exactly 1
    a, b = _line(7), _line(7, 1.0)[[0, 6]]
    m = np.array([0, 1, 2, 3, 2, 1, 0], float)
    want = np.sqrt(1 + m * m).mean() + 1.0
    assert mod.chamfer(a, b) == pytest.approx(want, abs=1e-12)


def test_parallel_lines(mod=R):
    # two copies of a point row a distance h apart: every nearest point is the
    # one straight across, CD = 2 h
    assert mod.chamfer(_line(9), _line(9, 0.25)) == pytest.approx(0.5, abs=1e-12)


def test_concentric_circles(mod=R):
    # same angles, radii 1 and 1.1, 8 points: the nearest point is the radial
    # neighbour (0.1) rather than the next angle (about 0.81), so CD = 0.2
    assert mod.chamfer(_circle(8, 1.0), _circle(8, 1.1)) == pytest.approx(0.2, abs=1e-12)


def test_rotated_copy_of_a_sampled_circle(mod=R):
    # a circle sampled at T angles against the same circle turned by half a step:
    # every nearest point is an angular neighbour at chord 2 r sin(pi / 2T)
    T, r = 16, 0.5
    want = 2 * 2 * r * math.sin(math.pi / (2 * T))
    assert mod.chamfer(_circle(T, r), _circle(T, r, phase=math.pi / T)) == pytest.approx(want, abs=1e-12)


def test_bank_form_matches_closed_forms(mod=R):
    # the bank evaluation on circles of several radii: CD = 2 |r - 1| while the
    # radial neighbour stays the nearest point
    T = 12
    radii = [1.0, 1.02, 0.97, 1.1]
    bank = np.stack([_circle(T, r) for r in radii])
    got = mod.chamfer_bank(_circle(T, 1.0), bank)
    np.testing.assert_allclose(got, [2 * abs(r - 1) for r in radii], atol=1e-12)


def test_bank_form_one_sided_sets(mod=R):
    # the collinear example in bank form: a bank path made of the ends repeated
    q = _line(7)
    b = np.concatenate([np.repeat(_line(7)[[0]], 3, 0), np.repeat(_line(7)[[6]], 4, 0)])
    got = mod.chamfer_bank(q, b[None])
    assert got[0] == pytest.approx(9.0 / 7.0, abs=1e-12)


# ---- invariants -------------------------------------------------------------------

def test_invariants(mod=R):
    c = gen.closed_curves(4, 40, seed=7).astype(np.float64)
    a, b = c[0], c[1]
    d = mod.chamfer(a, b)
    assert d > 0
    assert mod.chamfer(a, a) == 0.0
    assert mod.chamfer(b, a) == pytest.approx(d, rel=1e-14)
    rng = np.random.default_rng(3)
    assert mod.chamfer(a[rng.permutation(40)], b[rng.permutation(40)]) == pytest.approx(d, rel=1e-12)
    th = 0.7
    R2 = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    t = np.array([0.3, -1.2])
    assert mod.chamfer(a @ R2.T + t, b @ R2.T + t) == pytest.approx(d, rel=1e-12)
    # scaling both sets scales the distance
    assert mod.chamfer(3 * a, 3 * b) == pytest.approx(3 * d, rel=1e-12)


def test_non_finite_paths_never_match(mod=R):
    c = gen.closed_curves(3, 16, seed=1).astype(np.float64)
    c[1, 5, 0] = np.nan
    c[2, 3, 1] = np.inf
    got = mod.chamfer_bank(c[0], c)
    assert got[0] == 0.0 and np.isnan(got[1]) and np.isnan(got[2])
    idx, _ = mod.select(got, 3, cutoff=np.inf, order=mod.BEST)
    assert list(idx) == [0, -1, -1]


# ---- the searches -------------------------------------------------------------------

D = np.array([0.5, 0.01, np.nan, 0.02, 0.01, 0.029, 0.03, 0.0])


def test_first_search(mod=R):
    idx, dist = mod.select(D, 3, 0.03, mod.FIRST)
    assert list(idx) == [1, 3, 4]
    np.testing.assert_array_equal(dist, [0.01, 0.02, 0.01])
    idx, dist = mod.select(D, 6, 0.03, mod.FIRST)  # 0.03 is not below the cut-off
    assert list(idx) == [1, 3, 4, 5, 7, -1] and np.isnan(dist[-1])


def test_best_search(mod=R):
    idx, dist = mod.select(D, 3, 0.03, mod.BEST)
    assert list(idx) == [7, 1, 4]  # equal distances in bank order
    idx, _ = mod.select(D, 8, np.inf, mod.BEST)
    assert list(idx) == [7, 1, 4, 3, 5, 6, 0, -1]


def test_search_on_planted_matches(mod=R):
    # near copies of query 0 planted at known positions of a bank of unrelated
    # curves: both searches find them, FIRST in bank order
    base = gen.closed_curves(40, 32, seed=11)
    bank = base.copy()
    near = gen.near_copies(base[:1], 4, 0.001, seed=5)
    pos = [31, 7, 22, 13]
    bank[pos] = near
    idx, dist = mod.search(base[:1], bank, 3, 0.03, mod.FIRST)
    assert list(idx[0]) == [0, 7, 13]  # the query itself (position 0) comes first
    idx, _ = mod.search(base[:1], bank, 5, 0.03, mod.BEST)
    assert idx[0, 0] == 0 and sorted(idx[0, 1:]) == sorted(pos)


PINS = [test_single_points, test_collinear_subset, test_ends_lifted_off_the_line, test_parallel_lines,
        test_concentric_circles, test_rotated_copy_of_a_sampled_circle, test_bank_form_matches_closed_forms,
        test_bank_form_one_sided_sets, test_invariants, test_non_finite_paths_never_match, test_first_search,
        test_best_search, test_search_on_planted_matches]

MUTATIONS = {
    "squared_distance": ("d = np.sqrt((diff * diff).sum(axis=-1))  # [Ta, Tb]", "d = (diff * diff).sum(axis=-1)  # [Ta, Tb]"),
    "one_direction": ("return float(d.min(axis=1).mean() + d.min(axis=0).mean())", "return float(2 * d.min(axis=1).mean())"),
    "sum_not_mean": ("return float(d.min(axis=1).mean() + d.min(axis=0).mean())",
                     "return float(d.min(axis=1).sum() + d.min(axis=0).mean())"),
    "bank_same_axis_twice": ("out[lo:lo + block] = d.min(axis=2).mean(axis=1) + d.min(axis=1).mean(axis=1)",
                             "out[lo:lo + block] = 2 * d.min(axis=2).mean(axis=1)"),
    "bank_l1_norm": ("        d = np.sqrt((diff * diff).sum(axis=-1))\n", "        d = np.abs(diff).sum(axis=-1)\n"),
    "cutoff_inclusive": ("under = np.flatnonzero(d < cutoff)", "under = np.flatnonzero(d <= cutoff)"),
    "best_ties_reversed": ("pick = under[np.lexsort((under, d[under]))][:k]", "pick = under[np.lexsort((-under, d[under]))][:k]"),
    "first_by_distance": ("        pick = under[:k]\n", "        pick = under[np.argsort(d[under], kind='stable')][:k]\n"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name):
    src = open(os.path.join(os.path.dirname(R.__file__), "retrieval.py")).read()
    old, new = MUTATIONS[name]
    assert src.count(old) == 1, "mutation anchor must match the source exactly once"
    mod = types.ModuleType(f"retrieval_{name}")
    exec(compile(src.replace(old, new), f"retrieval_{name}.py", "exec"), mod.__dict__)
    caught = 0
    for pin in PINS:
        try:
            pin(mod)
        except AssertionError:
            caught += 1
    assert caught, f"no pin detects the planted mistake '{name}'"
