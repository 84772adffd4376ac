"""Closed-form pins of the oracle's band margins.

The margins decide which candidates are in-band (a decision within the stated
band of its threshold, so a lower-precision evaluation may take it either way)
and therefore excused from bit-exact FP32 parity.  Each margin is checked here
against values computed from the geometry alone, never by re-running the
oracle's formulas:

* margins[2], the branch distance: at every step each placed joint's previous
  position (the initial one at t = 0) measured from the line through its two
  parents' current positions.  On crank-rocker four-bars the rocker joint's
  positions come from Freudenstein's equation and the coupler point's from its
  rigid triangle; on a joint carried rigidly by the crank the distance is
  r |sin(psi - 2 pi / T)|.
* margins[3], the drift distance: |(length now - initial length) - tau scale| /
  scale, minimised over the steps evaluated up to the failing one, for a link
  outside the solve order whose length is a law-of-cosines function of the
  crank angle (crank tip to a fixed joint, crank-carried joint to a fixed joint)
  or of the rocker angle (rocker joint to a fixed joint near the rocker's pivot).
  The DRIFT step is pinned at the same time.
* margins[0] and margins[1] on the crank-carried joint: its triangle with the
  pivot and the tip is rigid, so 16 area^2 = 4 a^2 r^2 sin^2 psi and d^2 = a^2.

Paper: "Finding Valid Initial Positions" (a mechanism is kept only if a full
rotation completes) and "Background -- Simulation of Kinematics" (the branch is
resolved from the initial positions).
"""
import math

import numpy as np

import oracle
from paper_2208_14567_amd import gen
from tests import mech
from tests.test_oracle_fourbar import _frame, _freudenstein_roots

TAU = oracle.TAU_DRIFT


def _cross(u, v):
    return u[0] * v[1] - u[1] * v[0]


def _line_distance(p, a, b):
    """Distance of point p from the line through a and b."""
    u = b - a
    return abs(_cross(u, p - a)) / math.hypot(*u)


def _fourbar_track(x0, T):
    """Ground-frame positions (x0_0 at the origin, x0_2 on +x) of the crank tip 1,
    the rocker joint 3 (Freudenstein's equation, root continuous from x0) and
    the coupler point 4 (fixed in the frame of 1 -> 3, on the side of the line
    1 -> 3 nearer its previous position) at every step, plus the initial
    positions in that frame."""
    to, _ = _frame(x0)
    L = lambda i, j: float(np.hypot(*(x0[i] - x0[j])))
    a, bb, cc, d = L(0, 1), L(1, 3), L(2, 3), L(0, 2)
    q = {k: np.asarray(to(x0[k]), float) for k in range(len(x0))}
    th2_0 = math.atan2(q[1][1], q[1][0])
    th4 = math.atan2(q[3][1], q[3][0] - d)
    u0 = (q[3] - q[1]) / math.hypot(*(q[3] - q[1]))
    n0 = np.array([-u0[1], u0[0]])
    along4, perp4 = float((q[4] - q[1]) @ u0), float((q[4] - q[1]) @ n0)
    p1 = np.empty((T, 2))
    p3 = np.empty((T, 2))
    p4 = np.empty((T, 2))
    for t in range(T):
        th2 = th2_0 + 2 * math.pi * t / T
        roots = _freudenstein_roots(a, bb, cc, d, th2)
        assert roots
        th4 = min(roots, key=lambda r4: abs(math.remainder(r4 - th4, 2 * math.pi)))
        p1[t] = (a * math.cos(th2), a * math.sin(th2))
        p3[t] = (d + cc * math.cos(th4), cc * math.sin(th4))
        u = (p3[t] - p1[t]) / math.hypot(*(p3[t] - p1[t]))
        n = np.array([-u[1], u[0]])
        # the triangle 1-3-4 or its mirror image in the line 1-3: the one nearer
        # the previous position (a thin triangle can change side)
        prev4 = q[4] if t == 0 else p4[t - 1]
        c4 = [p1[t] + along4 * u + s * perp4 * n for s in (1.0, -1.0)]
        p4[t] = min(c4, key=lambda z: float(np.sum((z - prev4) ** 2)))
    return q, p1, p3, p4


def test_branch_margin_fourbar_closed_form(oracle_lib=None):
    """margins[2] on crank-rocker four-bars with a coupler point: the rocker
    joint 3 (parents 1, 2) measured from the line p1(t) -- x0_2 and the coupler
    point 4 (parents 1, 3) from the line p1(t) -- p3(t), each from its previous
    position; positions from Freudenstein's equation and the rigid coupler
    triangle (and checked against the oracle's positions on the way)."""
    T = 200
    b = gen.workload("fourbar", 150, seed=71)
    r = oracle.simulate(b, T=T, margins=True, pos_all=True)
    assert np.all(r["status"] == oracle.VALID)
    to_min_at_later_step = 0
    for c in range(b.B):
        x0 = b.x0[c, :5]
        scale = max(float(np.hypot(*(x0[i] - x0[j]))) for i, j in mech.edges_of(b, c))
        q, p1, p3, p4 = _fourbar_track(x0, T)
        to, _ = _frame(x0)
        # the closed-form positions are the oracle's (to 1e-9 of the scale)
        assert np.allclose(np.asarray(to(r["pos_all"][c, :, 3])), p3, atol=1e-9 * scale), c
        assert np.allclose(np.asarray(to(r["pos_all"][c, :, 4])), p4, atol=1e-9 * scale), c
        d3 = np.array([_line_distance(q[3] if t == 0 else p3[t - 1], p1[t], q[2]) for t in range(T)])
        d4 = np.array([_line_distance(q[4] if t == 0 else p4[t - 1], p1[t], p3[t]) for t in range(T)])
        per_step = np.minimum(d3, d4)
        want = per_step.min() / scale
        got = r["margins"][c, 2]
        assert abs(got - want) <= 1e-9, (c, got, want)
        to_min_at_later_step += int(np.argmin(per_step) > 0)
    # the minimum is usually taken where the previous position has moved along
    # the parents' line (a step after the first), so the pin sees that component
    assert to_min_at_later_step > b.B // 4


def _crank_carried(B, seed):
    """Pivot 0, crank tip 1, fixed joint 2, and joint 3 linked to 0, 1 and 2:
    joint 3 is placed from (0, 1), so it turns rigidly with the crank, and the
    link 2-3 lies outside the solve order.  Joint 3 starts near the line through
    0 and 2 (where its distance to 2 is extremal), so the link drifts slowly.
    Returns the batch and the closed-form parameters."""
    rng = np.random.default_rng(seed)
    ms, par = [], []
    while len(ms) < B:
        p0 = rng.uniform(0.2, 0.8, 2)
        a = rng.uniform(0.05, 0.3)
        al = rng.uniform(-math.pi, math.pi)
        g = rng.uniform(0.5, 1.0)
        be = rng.uniform(-math.pi, math.pi)
        rr = rng.uniform(0.1, 0.4)
        om = be + math.pi * rng.integers(0, 2) + rng.normal(0, 0.03)
        psi = om - al
        # keep the joint well off the crank's line: with |psi| (mod pi) above
        # 17 degrees and steps of at most 7.2 degrees the continuity rule never
        # swaps it for its mirror image, so it turns rigidly with the crank
        if abs(math.sin(psi)) < 0.3:
            continue
        x0 = np.array([p0, p0 + a * np.array([math.cos(al), math.sin(al)]),
                       p0 + g * np.array([math.cos(be), math.sin(be)]),
                       p0 + rr * np.array([math.cos(om), math.sin(om)])])
        ms.append({"n": 4, "edges": [(0, 1), (0, 3), (1, 3), (2, 3)], "fixed": [0, 2], "x0": x0})
        par.append((a, g, rr, be, om, psi))
    return mech.build(ms, J=6), par


def _drift_decision(length, L0, scale, T, tau=TAU):
    """First step where |length(t) - L0| exceeds tau scale (-1: none), the drift
    margin over the steps evaluated up to it, and whether any evaluated step is
    too close to the threshold to call."""
    drift = np.abs(length - L0)
    over = drift > tau * scale
    t_fail = int(np.argmax(over)) if over.any() else -1
    last = t_fail if t_fail >= 0 else T - 1
    gap = np.abs(drift[: last + 1] - tau * scale)
    return t_fail, gap.min() / scale, gap.min() < 1e-9 * scale


def test_margins_of_a_crank_carried_joint_closed_form(oracle_lib=None):
    """The crank-carried joint 3: status and failing step of the drifting link
    2-3 (law of cosines in the crank angle), its drift margin, its branch
    distance r |sin(psi - 2 pi / T)| (r |sin psi| at t = 0), and its constant
    discriminant and parent distance."""
    checked = {T: 0 for T in (50, 200, 1000)}
    fails = 0
    for T in checked:
        b, par = _crank_carried(120, seed=T)
        r = oracle.simulate(b, T=T, margins=True)
        t = np.arange(T)
        for c, (a, g, rr, be, om, psi) in enumerate(par):
            x0 = b.x0[c, :4]
            L = lambda i, j: float(np.hypot(*(x0[i] - x0[j])))
            scale = max(L(0, 1), L(0, 3), L(1, 3), L(2, 3))
            length = np.sqrt(rr * rr + g * g - 2 * rr * g * np.cos(om - be + 2 * np.pi * t / T))
            t_fail, m3, close = _drift_decision(length, L(2, 3), scale, T)
            if close:
                continue
            want_status = oracle.DRIFT if t_fail >= 0 else oracle.VALID
            assert r["status"][c] == want_status and r["fail_step"][c] == t_fail, (T, c, r["fail_step"][c], t_fail)
            m = r["margins"][c]
            assert abs(m[3] - m3) <= 1e-12, (T, c, m[3], m3)
            evaluated_later = t_fail != 0 and T > 1
            dist = rr * min(abs(math.sin(psi)), abs(math.sin(psi - 2 * math.pi / T)) if evaluated_later else 9.0)
            assert abs(m[2] - dist / scale) <= 1e-12, (T, c, m[2], dist / scale)
            assert abs(m[0] - (a * rr * math.sin(psi)) ** 2 / scale ** 4) <= 1e-12 * m[0], (T, c)
            assert abs(m[1] - a * a / scale ** 2) <= 1e-13, (T, c)
            checked[T] += 1
            fails += t_fail > 0
    assert min(checked.values()) > 100 and fails > 100, (checked, fails)


def test_drift_margin_of_the_crank_tip_closed_form(oracle_lib=None):
    """No placed joint: pivot 0, tip 1, fixed joint 2 and the link 1-2 outside
    the solve order, whose length follows the law of cosines in the crank
    angle.  The tip starts near the line through 0 and 2 and the turn has 2000
    steps, so the link drifts past the threshold over a range of steps; no dyad is evaluated, so the other margins stay
    infinite."""
    rng = np.random.default_rng(81)
    T = 2000
    ms, par = [], []
    for _ in range(300):
        p0 = rng.uniform(0.2, 0.8, 2)
        a, g = rng.uniform(0.05, 0.4), rng.uniform(0.5, 1.0)
        be = rng.uniform(-math.pi, math.pi)
        al = be + math.pi * rng.integers(0, 2) + rng.normal(0, 0.005)
        x0 = np.array([p0, p0 + a * np.array([math.cos(al), math.sin(al)]),
                       p0 + g * np.array([math.cos(be), math.sin(be)])])
        ms.append({"n": 3, "edges": [(0, 1), (1, 2)], "fixed": [0, 2], "x0": x0})
        par.append((a, g, al, be))
    b = mech.build(ms, J=4)
    r = oracle.simulate(b, T=T, margins=True)
    t = np.arange(T)
    seen_steps = set()
    for c, (a, g, al, be) in enumerate(par):
        x0 = b.x0[c, :3]
        L12 = float(np.hypot(*(x0[1] - x0[2])))
        scale = max(float(np.hypot(*(x0[1] - x0[0]))), L12)
        length = np.sqrt(a * a + g * g - 2 * a * g * np.cos(al - be + 2 * np.pi * t / T))
        t_fail, m3, close = _drift_decision(length, L12, scale, T)
        if close:
            continue
        assert r["fail_step"][c] == t_fail and r["status"][c] == (oracle.DRIFT if t_fail >= 0 else oracle.VALID), c
        assert abs(r["margins"][c, 3] - m3) <= 1e-12, (c, r["margins"][c, 3], m3)
        assert np.all(np.isinf(r["margins"][c, :3]))
        seen_steps.add(t_fail)
    assert len(seen_steps) > 5


def test_drift_margin_through_the_rocker_closed_form(oracle_lib=None):
    """Crank-rocker four-bars whose coupler point is replaced by a fixed joint 4
    near the rocker's pivot 2, linked to the rocker joint 3.  Joint 3 keeps its
    parents (1, 2), so the link 3-4 lies outside the solve order and its length
    |p3(t) - x0_4| follows from Freudenstein's rocker angle; the branch distance
    of joint 3 is pinned on the way."""
    T = 200
    base = gen.workload("fourbar", 160, seed=91)
    rng = np.random.default_rng(92)
    ms = []
    for c in range(base.B):
        x0 = base.x0[c, :5].copy()
        delta = rng.uniform(2e-5, 2e-3) * float(np.hypot(*(x0[3] - x0[2])))
        ang = rng.uniform(-math.pi, math.pi)
        x0[4] = x0[2] + delta * np.array([math.cos(ang), math.sin(ang)])
        ms.append({"n": 5, "edges": [(0, 1), (1, 3), (2, 3), (3, 4)], "fixed": [0, 2, 4], "x0": x0})
    b = mech.build(ms, J=6)
    r = oracle.simulate(b, T=T, margins=True)
    checked, fails = 0, 0
    for c in range(b.B):
        x0 = b.x0[c, :5]
        scale = max(float(np.hypot(*(x0[i] - x0[j]))) for i, j in mech.edges_of(b, c))
        q, p1, p3, _ = _fourbar_track(x0, T)
        length = np.hypot(*(p3 - q[4]).T)
        t_fail, m3, close = _drift_decision(length, float(np.hypot(*(x0[3] - x0[4]))), scale, T)
        if close:
            continue
        assert r["fail_step"][c] == t_fail and r["status"][c] == (oracle.DRIFT if t_fail >= 0 else oracle.VALID), c
        assert abs(r["margins"][c, 3] - m3) <= 1e-9, (c, r["margins"][c, 3], m3)
        last = t_fail if t_fail >= 0 else T - 1
        d3 = [_line_distance(q[3] if t == 0 else p3[t - 1], p1[t], q[2]) for t in range(last + 1)]
        assert abs(r["margins"][c, 2] - min(d3) / scale) <= 1e-9, c
        checked += 1
        fails += t_fail > 0
    assert checked > 150 and fails > 50, (checked, fails)
