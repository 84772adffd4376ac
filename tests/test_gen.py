"""Seeded input generator: counter-based RNG and dyad-built topologies."""
import numpy as np
import pytest

from paper_2208_14567_amd import gen


def test_splitmix64_reference_outputs():
    # first outputs of SplitMix64 seeded with 0 (Steele, Lea, Flood 2014 reference generator)
    out = gen.draw_u64(np.uint64(0), np.arange(3))
    assert [int(x) for x in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_counter_based_and_fp32_exact():
    b1 = gen.workload("dyad_6_20", 1000, seed=5)
    b2 = gen.workload("dyad_6_20", 600, seed=5, first=400)
    assert np.array_equal(b1.adj[400:], b2.adj) and np.array_equal(b1.x0[400:], b2.x0)
    # every coordinate is a multiple of 2^-24 in [0, 1): exact in FP32
    x = b1.x0.ravel()
    assert np.all(x.astype(np.float32).astype(np.float64) == x)
    assert np.all((x * 2 ** 24) == np.floor(x * 2 ** 24)) and x.min() >= 0 and x.max() < 1


@pytest.mark.parametrize("paper,rules", [(False, False), (True, False), (False, True)])
def test_candidates_at_indices_equal_the_batch_rows(paper, rules):
    nd = gen.n_uniform(6, 20)
    b = gen.dyad_batch(3000, 7, nd, 20, paper_mode=paper, first=5000, rules=rules)
    idx = np.random.default_rng(3).integers(5000, 8000, size=500)
    idx[:3] = (7999, 5000, 7999)  # both ends, a repeat
    a = gen.dyad_batch_at(idx, 7, nd, 20, paper_mode=paper, rules=rules, chunk=128)
    r = idx - 5000
    for f in ("n", "adj", "fixed", "motor", "x0"):
        assert np.array_equal(getattr(a, f), getattr(b, f)[r]), f
    assert gen.dyad_batch_at([], 7, nd).B == 0
    with pytest.raises(ValueError):
        gen.dyad_batch_at([-1], 7, nd)


def _mobility(b):
    """Mobility m = 3(N-1) - 2 j1 of the paper's Eq. 1 with every edge a binary link
    plus one ground body; a joint joining k bodies contributes k-1 pin pairs."""
    m = np.zeros(b.B, np.int64)
    for c in range(b.B):
        n = int(b.n[c])
        E = sum(bin(int(b.adj[c, i]) & ((1 << n) - 1)).count("1") for i in range(n)) // 2
        bodies = E + 1
        j1 = 0
        for i in range(n):
            k = bin(int(b.adj[c, i])).count("1") + ((int(b.fixed[c]) >> i) & 1)
            j1 += max(k - 1, 0)
        m[c] = 3 * (bodies - 1) - 2 * j1
    return m


@pytest.mark.parametrize("name", ["dyad_6_20", "dyad_skewed", "dyad_4_20", "paper_8_20", "paper_rules_8_20",
                                  "dyad_rules_6_20"])
def test_dyad_topologies_have_mobility_one(name):
    b = gen.workload(name, 400, seed=9)
    assert np.all(_mobility(b) == 1)
    # symmetric, no self links, nothing beyond n
    for c in range(b.B):
        n = int(b.n[c])
        A = np.array([[(int(b.adj[c, i]) >> j) & 1 for j in range(b.J)] for i in range(b.J)])
        assert np.array_equal(A, A.T) and A.trace() == 0 and A[n:].sum() == 0
        assert (int(b.fixed[c]) >> 0) & 1 and not (int(b.fixed[c]) >> 1) & 1 and A[0, 1] == 1


def test_joint_count_distributions():
    b = gen.workload("dyad_6_20", 60000, seed=2)
    counts = np.bincount(b.n, minlength=21)[6:21]
    assert counts.min() > 0.9 * 60000 / 15 and counts.max() < 1.1 * 60000 / 15
    s = gen.workload("dyad_skewed", 60000, seed=3)
    frac = [np.mean((s.n >= lo) & (s.n <= hi)) for lo, hi in ((6, 8), (9, 14), (15, 20))]
    assert abs(frac[0] - 0.6) < 0.01 and abs(frac[1] - 0.3) < 0.01 and abs(frac[2] - 0.1) < 0.01


def test_fourbar_rejection_gives_grashof_crank_rockers():
    b = gen.workload("fourbar", 2000)
    p = b.x0
    L = lambda i, j: np.hypot(*(p[:, i] - p[:, j]).T)
    crank, coupler, rocker, ground = L(0, 1), L(1, 3), L(2, 3), L(0, 2)
    allL = np.stack([crank, coupler, rocker, ground], 1)
    s, l = allL.min(1), allL.max(1)
    assert np.all(crank == s) and np.all(s + l < allL.sum(1) - s - l)


def test_closed_curves_are_seeded_and_closed():
    a = gen.closed_curves(50, 64, seed=3)
    b = gen.closed_curves(50, 64, seed=3)
    c = gen.closed_curves(50, 64, seed=4)
    assert a.shape == (50, 64, 2) and a.dtype == np.float32
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert np.isfinite(a).all()
    # a Fourier series without a constant term: the points average to the centre,
    # which lies near (0.5, 0.5)
    centre = a.astype(np.float64).mean(axis=1)
    assert np.all(np.abs(centre - 0.5) < 0.3)


def test_near_copies_shift_the_start_and_add_noise():
    base = gen.closed_curves(4, 40, seed=8)
    near = gen.near_copies(base, 3, 0.0, seed=9)
    assert near.shape == (12, 40, 2)
    for i in range(12):
        # without noise each copy is its curve with the start point moved
        src = base[i // 3]
        assert any(np.array_equal(near[i], np.roll(src, -k, axis=0)) for k in range(40))
    noisy = gen.near_copies(base, 2, 0.01, seed=9)
    assert not np.array_equal(noisy, gen.near_copies(base, 2, 0.0, seed=9))


def _rule_violations(b):
    """Per candidate: (not every joint lies in the dependency closure of the last
    joint of the graphical solver's order, the last joint is linked to a fixed
    joint).  The closure follows each placed joint to its two solve-order parents
    and the tip to the pivot."""
    import oracle
    order, nd, _, st = oracle.solve_order(b)
    assert np.all(st == 0)
    red, fix = np.zeros(b.B, bool), np.zeros(b.B, bool)
    for c in range(b.B):
        n, D, fx = int(b.n[c]), int(nd[c]), int(b.fixed[c])
        par = {int(e[0]): (int(e[1]), int(e[2])) for e in order[c, :D]}
        par[1] = (0,)
        last = int(order[c, D - 1, 0])
        seen, todo = set(), [last]
        while todo:
            j = todo.pop()
            if j not in seen:
                seen.add(j)
                todo.extend(par.get(j, ()))
        red[c] = len(seen) != n
        fix[c] = any((int(b.adj[c, last]) >> f) & 1 and (fx >> f) & 1 for f in range(n))
    return red, fix


@pytest.mark.parametrize("paper", [False, True])
def test_topology_rules(paper):
    """The paper's topology rules ("Generating Valid Topologies"): with them every
    candidate's last solved joint depends on all other joints and touches no fixed
    joint; without them many candidates break both rules."""
    lo = 8 if paper else 5
    b = gen.dyad_batch(3000, 31, gen.n_uniform(lo, 20), J=20, paper_mode=paper, rules=True)
    red, fix = _rule_violations(b)
    assert not red.any() and not fix.any()
    b0 = gen.dyad_batch(3000, 31, gen.n_uniform(lo, 20), J=20, paper_mode=paper, rules=False)
    red0, fix0 = _rule_violations(b0)
    assert red0.mean() > 0.5 and fix0.mean() > 0.05
    # the rules cannot be met below five joints
    with pytest.raises(ValueError):
        gen.dyad_batch(10, 1, gen.n_uniform(4, 6), rules=True)
