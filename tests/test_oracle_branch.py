"""The two branch rules of the oracle, pinned by properties of the positions they
produce (not by re-running their own formulas):

* continuity: at every step each placed joint is the intersection nearer its
  previous position (the other intersection is its mirror image in the line
  through its parents);
* orientation: each placed joint stays on the side of its parents' line where it
  starts;
* on Grashof crank-rockers, which never pass through a folded position, the two
  rules coincide; on random dyad mechanisms they do not always."""
import numpy as np

import oracle
from paper_2208_14567_amd import gen


def _sides_and_mirror_gap(b, r, order, nd, c, T):
    """For candidate c: per step and dyad, the side (sign of the cross product of
    a->b with a->k) and whether the chosen point is at least as near the previous
    position as its mirror image."""
    pos = r["pos_all"][c]
    x0 = b.x0[c]
    steps = T if r["status"][c] == 0 else int(r["fail_step"][c])
    sides, nearer = [], []
    for t in range(steps):
        prev = x0 if t == 0 else pos[t - 1]
        row_s, row_n = [], []
        for s in range(int(nd[c])):
            k, a, bb = (int(v) for v in order[c, s])
            pa, pb, pk = pos[t, a], pos[t, bb], pos[t, k]
            u = pb - pa
            row_s.append(u[0] * (pk[1] - pa[1]) - u[1] * (pk[0] - pa[0]) >= 0)
            # mirror of pk in the line a-b
            w = pk - pa
            proj = pa + u * (w @ u) / (u @ u)
            mirror = 2 * proj - pk
            q = prev[k]
            row_n.append(np.sum((q - pk) ** 2) <= np.sum((q - mirror) ** 2) * (1 + 1e-9) + 1e-24)
        sides.append(row_s)
        nearer.append(row_n)
    return np.array(sides, bool), np.array(nearer, bool)


def test_rules_keep_their_invariants():
    T = 60
    b = gen.dyad_batch(400, 17, gen.n_uniform(5, 9), J=10)
    order, nd, _, _ = oracle.solve_order(b)
    rc = oracle.simulate(b, T=T, pos_all=True)
    ro = oracle.simulate(b, T=T, pos_all=True, branch=oracle.BRANCH_ORIENTATION)
    differ = 0
    for c in range(b.B):
        if nd[c] == 0:
            continue
        s_o, _ = _sides_and_mirror_gap(b, ro, order, nd, c, T)
        if s_o.size:
            # orientation: the starting sides at every step
            x0 = b.x0[c]
            start = []
            for s in range(int(nd[c])):
                k, a, bb = (int(v) for v in order[c, s])
                u = x0[bb] - x0[a]
                start.append(u[0] * (x0[k, 1] - x0[a, 1]) - u[1] * (x0[k, 0] - x0[a, 0]) >= 0)
            assert (s_o == np.array(start)[None, :]).all(), c
        _, n_c = _sides_and_mirror_gap(b, rc, order, nd, c, T)
        assert n_c.size == 0 or n_c.all(), c  # continuity: never the farther intersection
        if rc["status"][c] != ro["status"][c] or rc["fail_step"][c] != ro["fail_step"][c]:
            differ += 1
    assert differ > 0  # the rules are different rules


def test_rules_agree_where_continuity_keeps_the_starting_sides():
    """Where the continuity run keeps every placed joint on its starting side of
    its parents' line at every step, the orientation run is the same run, bit for
    bit (checked on crank-rocker four-bars with a coupler point, most of which
    qualify; a coupler point almost on its parents' line may change side under
    continuity)."""
    T = 200
    b = gen.workload("fourbar", 600, seed=9)
    order, nd, _, _ = oracle.solve_order(b)
    rc = oracle.simulate(b, T=T, path=True, pos_all=True)
    ro = oracle.simulate(b, T=T, path=True, branch=oracle.BRANCH_ORIENTATION)
    qualified = 0
    for c in range(b.B):
        sides, _ = _sides_and_mirror_gap(b, rc, order, nd, c, T)
        x0 = b.x0[c]
        start = []
        for s in range(int(nd[c])):
            k, a, bb = (int(v) for v in order[c, s])
            u = x0[bb] - x0[a]
            start.append(u[0] * (x0[k, 1] - x0[a, 1]) - u[1] * (x0[k, 0] - x0[a, 0]) >= 0)
        if sides.size == 0 or (sides == np.array(start)[None, :]).all():
            qualified += 1
            assert rc["status"][c] == ro["status"][c] and rc["fail_step"][c] == ro["fail_step"][c], c
            assert np.array_equal(rc["path"][c], ro["path"][c], equal_nan=True), c
    assert qualified > 0.9 * b.B
