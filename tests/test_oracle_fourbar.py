"""Four-bar pins of the FP64 oracle: values fixed by closed forms, not by the oracle.

* a hand-derived worked example (tests/golden/fourbar_worked.json),
* Freudenstein's equation for the rocker angle (half-angle quadratic),
* grid-exact prediction of the first locking step from the law of cosines,
* Grashof's criterion for full crank rotation.
"""
import json
import math
import os

import numpy as np

import oracle
from paper_2208_14567_amd import gen
from tests import mech

GOLD = os.path.join(os.path.dirname(__file__), "golden")
ENV = {"sqrt": math.sqrt}


def _ev(s):
    return float(eval(str(s), {"__builtins__": {}}, ENV))


def test_worked_example_positions(oracle_lib):
    g = json.load(open(os.path.join(GOLD, "fourbar_worked.json")))
    x0 = np.array([[_ev(v) for v in p] for p in g["x0"]])
    b = gen.fourbar_topology(1)
    b.x0[0] = x0
    r = oracle.simulate(b, T=g["T"], pos_all=True, path=True)
    assert r["status"][0] == oracle.VALID and r["fail_step"][0] == -1
    P = r["pos_all"][0]
    for t, joints in g["expected"].items():
        t = int(t)
        for j, xy in joints.items():
            want = np.array([_ev(v) for v in xy])
            assert np.allclose(P[t, int(j)], want, atol=1e-12), (t, j, P[t, int(j)], want)
        A, B = P[t, 1], P[t, 3]
        v = B - A
        want4 = A + v / 2 + np.array([-v[1], v[0]]) / 2
        assert np.allclose(P[t, 4], want4, atol=1e-12)
    # the default output joint is the last placed joint (the coupler point)
    assert np.array_equal(r["path"][0], P[:, 4])


def _frame(x0):
    """Rotate so the ground link O2->O4 lies on +x with O2 at the origin."""
    g = x0[2] - x0[0]
    ang = math.atan2(g[1], g[0])
    c, s = math.cos(-ang), math.sin(-ang)
    R = np.array([[c, -s], [s, c]])
    return lambda p: (np.asarray(p) - x0[0]) @ R.T, ang


def _freudenstein_roots(a, b, c, d, th2):
    """Rocker angles theta4 with K1 cos th4 - K2 cos th2 + K3 = cos(th2 - th4),
    K1 = d/a, K2 = d/c, K3 = (a^2 - b^2 + c^2 + d^2)/(2ac), via u = tan(th4/2):
    (R - P) u^2 - 2 Q u + (P + R) = 0 with P = K1 - cos th2, Q = sin th2, R = K3 - K2 cos th2."""
    K1, K2, K3 = d / a, d / c, (a * a - b * b + c * c + d * d) / (2 * a * c)
    P, Q, R = K1 - math.cos(th2), math.sin(th2), K3 - K2 * math.cos(th2)
    disc = Q * Q + P * P - R * R
    if disc < 0:
        return []
    if abs(R - P) < 1e-14:
        return [2 * math.atan(-(P + R) / (-2 * Q))] if Q != 0 else []
    return [2 * math.atan((Q + sg * math.sqrt(disc)) / (R - P)) for sg in (1, -1)]


def test_freudenstein_rocker_angle(oracle_lib):
    b = gen.workload("fourbar", 300, seed=21)
    T = 200
    r = oracle.simulate(b, T=T, pos_all=True, margins=True)
    assert np.all(r["status"] == oracle.VALID)
    for c in range(b.B):
        x0 = b.x0[c, :5]
        to, ang = _frame(x0)
        L = lambda i, j: float(np.hypot(*(x0[i] - x0[j])))
        a, bb, cc, d = L(0, 1), L(1, 3), L(2, 3), L(0, 2)
        q1 = to(x0[1]); q3 = to(x0[3])
        th2_0 = math.atan2(q1[1], q1[0])
        th4 = math.atan2(q3[1], q3[0] - d)
        for t in range(T):
            th2 = th2_0 + 2 * math.pi * t / T
            roots = _freudenstein_roots(a, bb, cc, d, th2)
            assert roots
            # continuity of the rocker angle from its initial value
            th4 = min(roots, key=lambda r4: abs(math.remainder(r4 - th4, 2 * math.pi)))
            p3 = to(r["pos_all"][c, t, 3])
            want = np.array([d + cc * math.cos(th4), cc * math.sin(th4)])
            assert np.allclose(p3, want, atol=1e-9 * max(a, bb, cc, d)), (c, t)


def _lock_prediction(b, T):
    """First grid step where joint 3 (parents 1 and 2) cannot be placed:
    |p1(t) - x0_2| outside [|r1 - r2|, r1 + r2]; joint 4 sits on the rigid
    triangle 1-3-4 and never locks.  Returns (status, fail_step, margin)."""
    st = np.zeros(b.B, np.uint8)
    fs = np.full(b.B, -1, np.int16)
    margin = np.full(b.B, np.inf)
    t = np.arange(T)
    for c in range(b.B):
        x0 = b.x0[c]
        z1 = complex(*(x0[1] - x0[0]))
        p1 = complex(*x0[0]) + z1 * np.exp(2j * np.pi * t / T)
        dist = np.abs(p1 - complex(*x0[2]))
        r1 = np.hypot(*(x0[3] - x0[1])); r2 = np.hypot(*(x0[3] - x0[2]))
        lo, hi = abs(r1 - r2), r1 + r2
        bad = (dist < lo) | (dist > hi)
        m = np.minimum(np.abs(dist - lo), np.abs(dist - hi))
        if bad.any():
            t0 = int(np.argmax(bad))
            st[c], fs[c] = oracle.LOCKED, t0
            margin[c] = m[: t0 + 1].min()
        else:
            margin[c] = m.min()
    return st, fs, margin


def test_grid_exact_lock_prediction(oracle_lib):
    T = 200
    b = gen.workload("fourbar_u", 4000, seed=31)
    r = oracle.simulate(b, T=T)
    st, fs, margin = _lock_prediction(b, T)
    clear = margin > 1e-9
    assert clear.mean() > 0.99
    assert np.array_equal(r["status"][clear], st[clear])
    assert np.array_equal(r["fail_step"][clear], fs[clear])
    assert 0.1 < (st == oracle.VALID).mean() < 0.5  # both outcomes are well represented
    # the low-fidelity grid: the same prediction at T = 50
    r50 = oracle.simulate(b, T=50)
    st50, fs50, m50 = _lock_prediction(b, 50)
    c50 = m50 > 1e-9
    assert np.array_equal(r50["status"][c50], st50[c50]) and np.array_equal(r50["fail_step"][c50], fs50[c50])


def test_grashof_full_rotation(oracle_lib):
    T = 200
    b = gen.workload("fourbar_u", 4000, seed=41)
    r = oracle.simulate(b, T=T)
    valid = r["status"] == oracle.VALID
    x0 = b.x0
    L = lambda i, j: np.hypot(*(x0[:, i] - x0[:, j]).T)
    crank, coupler, rocker, ground = L(0, 1), L(1, 3), L(2, 3), L(0, 2)
    allL = np.stack([crank, coupler, rocker, ground], 1)
    s, l = allL.min(1), allL.max(1)
    pq = allL.sum(1) - s - l
    grashof = s + l < pq - 1e-6
    crank_turns = grashof & ((crank == s) | (ground == s))
    assert crank_turns.sum() > 200 and np.all(valid[crank_turns])
    # the crank cannot turn fully: invalid whenever the forbidden arc of crank angles
    # is wider than the grid spacing (then some grid angle falls inside it)
    th = np.linspace(0, 2 * np.pi, 20000, endpoint=False)
    checked = 0
    for c in np.nonzero(~crank_turns)[0][:600]:
        z1 = complex(*(x0[c, 1] - x0[c, 0]))
        dist = np.abs(complex(*x0[c, 0]) + z1 * np.exp(1j * th) - complex(*x0[c, 2]))
        lo, hi = abs(rocker[c] - coupler[c]), rocker[c] + coupler[c]
        forbidden = (dist < lo) | (dist > hi)
        if forbidden.mean() * 2 * np.pi > 2 * (2 * np.pi / T):
            assert not valid[c]
            checked += 1
    assert checked > 100


def test_discriminant_and_distance_margins_closed_form(oracle_lib):
    """The band margins the oracle reports (used to split candidates into
    decided-outside-the-band and in-band) against closed forms for crank-rocker
    four-bars: joint 3 hangs between the crank tip 1 and pivot 2, so its parent
    distance is |p1(t) - x0_2| and its discriminant the Heron product of the two
    link lengths and that distance; the coupler joint 4 sits on the rigid triangle
    1-3-4, whose parent distance and discriminant never change."""
    T = 200
    b = gen.workload("fourbar", 300, seed=51)
    r = oracle.simulate(b, T=T, margins=True)
    assert np.all(r["status"] == oracle.VALID)
    t = np.arange(T)
    for c in range(b.B):
        x0 = b.x0[c]
        L = lambda i, j: float(np.hypot(*(x0[i] - x0[j])))
        scale = max(L(0, 1), L(1, 3), L(2, 3), L(1, 4), L(3, 4))
        p1 = complex(*x0[0]) + complex(*(x0[1] - x0[0])) * np.exp(2j * np.pi * t / T)
        d3 = np.abs(p1 - complex(*x0[2]))
        ra, rb = L(1, 3), L(2, 3)
        K3 = ((ra + rb) ** 2 - d3 ** 2) * (d3 ** 2 - (ra - rb) ** 2)
        ra4, rb4, d4 = L(1, 4), L(3, 4), L(1, 3)
        K4 = ((ra4 + rb4) ** 2 - d4 ** 2) * (d4 ** 2 - (ra4 - rb4) ** 2)
        want_disc = min(np.abs(K3).min(), abs(K4)) / (4 * scale ** 4)
        want_deg = min((d3 ** 2).min(), d4 ** 2) / scale ** 2
        m = r["margins"][c]
        assert abs(m[0] - want_disc) <= 1e-9 * max(want_disc, 1e-12), (c, m[0], want_disc)
        assert abs(m[1] - want_deg) <= 1e-9 * want_deg, (c, m[1], want_deg)
        assert np.isinf(m[3])   # no redundant link, no drift check


def test_low_fidelity_screen_on_the_coarse_grid(oracle_lib):
    """The 50-position screen is the 200-position rule evaluated on every fourth
    angle: for four-bars, whose only lockable joint is decided by the law of
    cosines at each angle independently of the branch history, a candidate
    rejected on the coarse grid fails at the first coarse angle where the fine
    grid also fails (same status), and every survivor gets the full 200-step
    decision."""
    T = 200
    b = gen.workload("fourbar_u", 3000, seed=61)
    full = oracle.simulate(b, T=T)
    pre = oracle.simulate_prefiltered(b, T=T, T_low=50)
    st50, fs50, m50 = _lock_prediction(b, 50)
    clear = m50 > 1e-9
    rej = pre["status"] != oracle.VALID
    # rejected on the coarse grid: the law-of-cosines prediction at T = 50, mapped to the fine grid
    coarse_bad = clear & (st50 != oracle.VALID)
    assert np.array_equal(rej[clear] & coarse_bad[clear], coarse_bad[clear])
    assert np.array_equal(pre["fail_step"][coarse_bad], fs50[coarse_bad].astype(np.int16) * 4)
    # survivors of the screen carry the full simulation's decision
    surv = pre["status"] == oracle.VALID
    assert np.all(full["status"][surv] == oracle.VALID)
    keep = ~coarse_bad & clear
    assert np.array_equal(pre["status"][keep], full["status"][keep])
    assert np.array_equal(pre["fail_step"][keep], full["fail_step"][keep])
