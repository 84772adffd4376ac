"""Pins of the oracle's graphical solve order (Methodology, "Graphical Simulator")."""
import itertools
import json
import os

import numpy as np

import oracle
from paper_2208_14567_amd import gen
from tests import mech

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_fourbar_worked_order(oracle_lib):
    g = json.load(open(os.path.join(GOLD, "fourbar_worked.json")))
    b = gen.fourbar_topology(1)
    order, nd, dp, st = oracle.solve_order(b)
    assert st[0] == oracle.VALID and nd[0] == 2 and dp[0] == g["depth"]
    assert order[0, :2].tolist() == g["solve_order"] and np.all(order[0, 2:] == -1)


def _rounds_brute(n, edges, known0):
    """Earliest round of every joint by exhaustive search over known sets: a joint
    can be placed once two of its neighbours are placed; placing joints only ever
    helps, so the earliest round of each joint is the shortest chain of placements
    (breadth-first over all subsets reachable by placing any placeable subset)."""
    nb = [set() for _ in range(n)]
    for i, j in edges:
        nb[i].add(j); nb[j].add(i)
    best = {k: 0 for k in known0}
    frontier = {frozenset(known0)}
    r = 0
    while frontier:
        r += 1
        nxt = set()
        for K in frontier:
            placeable = [k for k in range(n) if k not in K and len(nb[k] & K) >= 2]
            for size in range(1, len(placeable) + 1):
                for sub in itertools.combinations(placeable, size):
                    K2 = K | frozenset(sub)
                    for k in sub:
                        if k not in best:
                            best[k] = r
                    nxt.add(K2)
        frontier = {K for K in nxt if len(K) < n}
        if r > n:
            break
    return best


def test_order_matches_brute_force_on_small_random_graphs(oracle_lib):
    rng = np.random.default_rng(0)
    mechs = []
    for _ in range(300):
        n = int(rng.integers(3, 8))
        edges = {(0, 1)}
        for i in range(n):
            for j in range(i + 1, n):
                if rng.random() < 0.35:
                    edges.add((i, j))
        fixed = {0} | {int(f) for f in rng.choice(np.arange(2, n), size=int(rng.integers(0, 2)), replace=False)} if n > 2 else {0}
        mechs.append({"n": n, "edges": sorted(edges), "fixed": sorted(fixed), "motor": (0, 1)})
    b = mech.build(mechs, J=8)
    order, nd, dp, st = oracle.solve_order(b)
    for c, m in enumerate(mechs):
        n = m["n"]
        best = _rounds_brute(n, m["edges"], set(m["fixed"]) | {1})
        placed = {int(order[c, s, 0]): s for s in range(nd[c])}
        assert set(placed) == set(best) - set(m["fixed"]) - {1}
        assert (st[c] == oracle.VALID) == (len(best) == n)
        # rounds: entries appear round by round, ascending joint index inside a round,
        # parents are the two smallest neighbours known before the round
        known = set(m["fixed"]) | {1}
        nb = [set() for _ in range(n)]
        for i, j in m["edges"]:
            nb[i].add(j); nb[j].add(i)
        s = 0
        r = 0
        while s < nd[c]:
            r += 1
            this = sorted(k for k in range(n) if k not in known and len(nb[k] & known) >= 2)
            got = [int(order[c, s + q, 0]) for q in range(len(this))]
            assert got == this
            for q, k in enumerate(this):
                assert [int(order[c, s + q, 1]), int(order[c, s + q, 2])] == sorted(nb[k] & known)[:2]
                assert best[k] == r
            known |= set(this)
            s += len(this)
        assert dp[c] == r


def test_dyad_topologies_solve_with_exactly_two_known_neighbours(oracle_lib):
    b = gen.workload("dyad_6_20", 2000, seed=4)
    order, nd, dp, st = oracle.solve_order(b)
    assert np.all(st == oracle.VALID)
    nfix = np.array([bin(int(f)).count("1") for f in b.fixed])
    assert np.array_equal(nd.astype(int), b.n.astype(int) - nfix - 1)
    # counting argument: |E| = 1 + 2 * placed joints, so no joint ever sees a third known neighbour
    for c in range(0, 2000, 7):
        known = int(b.fixed[c]) | 2
        s = 0
        while s < nd[c]:
            batch = []
            while s < nd[c]:
                k = int(order[c, s, 0])
                if bin(int(b.adj[c, k]) & known).count("1") < 2:
                    break
                assert bin(int(b.adj[c, k]) & known).count("1") == 2
                batch.append(k)
                s += 1
            for k in batch:
                known |= 1 << k


def test_relabeling_permutes_order(oracle_lib):
    b = gen.workload("dyad_6_20", 200, seed=8)
    rng = np.random.default_rng(1)
    order, nd, dp, st = oracle.solve_order(b)
    mechs, perms = [], []
    for c in range(b.B):
        n = int(b.n[c])
        rest = rng.permutation(np.arange(2, n)) if n > 2 else []
        perm = [0, 1] + [int(x) for x in rest]
        perms.append(perm)
        mechs.append(mech.permute(b, c, perm))
    p = mech.build(mechs, J=b.J)
    o2, nd2, dp2, st2 = oracle.solve_order(p)
    assert np.array_equal(nd, nd2) and np.array_equal(dp, dp2) and np.array_equal(st, st2)
    for c in range(b.B):
        a = {(perms[c][int(order[c, s, 0])], frozenset((perms[c][int(order[c, s, 1])], perms[c][int(order[c, s, 2])])))
             for s in range(nd[c])}
        bb = {(int(o2[c, s, 0]), frozenset((int(o2[c, s, 1]), int(o2[c, s, 2])))) for s in range(nd2[c])}
        assert a == bb


def test_assur_triad_and_dangling_joint_are_unsolvable(oracle_lib):
    # class-III Assur group: joints 3,4,5 form a ternary triangle, each tied to one known joint
    triad = {"n": 6, "edges": [(0, 1), (1, 3), (2, 4), (0, 5), (3, 4), (4, 5), (3, 5)], "fixed": [0, 2]}
    dangling = {"n": 5, "edges": [(0, 1), (1, 3), (2, 3), (3, 4)], "fixed": [0, 2]}
    ok = {"n": 4, "edges": [(0, 1), (1, 3), (2, 3)], "fixed": [0, 2]}
    b = mech.build([triad, dangling, ok])
    order, nd, dp, st = oracle.solve_order(b)
    assert st.tolist() == [oracle.UNSOLVABLE, oracle.UNSOLVABLE, oracle.VALID]
    assert nd[0] == 0 and nd[1] == 1 and order[1, 0].tolist() == [3, 1, 2]


def test_malformed_inputs_are_bad_mech(oracle_lib):
    base = {"n": 4, "edges": [(0, 1), (1, 3), (2, 3)], "fixed": [0, 2]}
    b = mech.build([base] * 8, J=6)
    b.adj[0, 3] &= ~np.uint32(1 << 1)            # asymmetric
    b.motor[1] = (2, 1); b.fixed[1] = 0b0001     # pivot not fixed
    b.motor[2] = (0, 2)                          # tip fixed
    b.adj[3, 2] |= np.uint32(1 << 2)             # diagonal bit
    b.n[4] = 2                                   # n < 3
    b.adj[5, 3] |= np.uint32(1 << 5); b.adj[5, 5] |= np.uint32(1 << 3)  # link beyond n
    b.motor[6] = (0, 3)                          # pivot-tip not linked
    order, nd, dp, st = oracle.solve_order(b)
    assert st.tolist() == [oracle.BAD_MECH] * 7 + [oracle.VALID]
