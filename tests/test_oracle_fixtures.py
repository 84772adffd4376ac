"""Status codes of the FP64 oracle on hand-built inputs (every code forced from the host)."""
import numpy as np

import oracle
from tests import mech

FB = [(0, 1), (1, 3), (2, 3)]
X_FB = [[0, 0], [1, 0], [4, 0], [11 / 3, 4 * 5 ** 0.5 / 3]]


def run(mechs, T=200, J=None):
    return oracle.simulate(mech.build(mechs, J=J), T=T, margins=True)


def test_redundant_links_drift(oracle_lib):
    # tip also tied to the second ground joint: a rigid structure turned by the motor
    tip_ground = {"n": 4, "edges": FB + [(1, 2)], "fixed": [0, 2], "x0": X_FB}
    # a consistent redundant link (a braced triangle that moves rigidly) never drifts
    braced = {"n": 5, "edges": FB + [(0, 4), (1, 4), (3, 4)], "fixed": [0, 2],
              "x0": X_FB + [[0.5, 0.8]]}
    r = run([tip_ground, braced])
    assert r["status"][0] == oracle.DRIFT and r["fail_step"][0] == 1
    # joint 4 is placed from (0, 1); the link 3-4 is redundant and must drift once the
    # four-bar moves, since 3 and 4 move on different curves
    assert r["status"][1] == oracle.DRIFT and r["fail_step"][1] >= 1
    rigid = {"n": 4, "edges": [(0, 1), (0, 3), (1, 3), (2, 3)], "fixed": [0, 2],
             "x0": [[0, 0], [1, 0], [3, 0], [0.5, 1.0]]}
    r = run([rigid])
    assert r["status"][0] == oracle.DRIFT and r["fail_step"][0] == 1


def test_consistent_redundancy_is_valid(oracle_lib):
    # a triangle with an extra joint braced to all three of its corners keeps every length
    tri = {"n": 4, "edges": [(0, 1), (0, 3), (1, 3)], "fixed": [0, 2],
           "x0": [[0, 0], [1, 0], [5, 5], [0.3, 0.9]]}
    four = {"n": 5, "edges": [(0, 1), (0, 3), (1, 3), (0, 4), (1, 4), (3, 4)], "fixed": [0, 2],
            "x0": [[0, 0], [1, 0], [5, 5], [0.3, 0.9], [0.8, -0.6]]}
    r = run([tri, four])
    assert r["status"].tolist() == [oracle.VALID, oracle.VALID]


def test_coincident_parents_are_degenerate(oracle_lib):
    # joint 3's parents are 1 and 2; the crank tip passes exactly through ground joint 2
    m = {"n": 4, "edges": FB, "fixed": [0, 2], "x0": [[0, 0], [1, 0], [0, 1], [0.5, 0.5]]}
    r = run([m], T=4)
    assert r["status"][0] == oracle.DEGENERATE and r["fail_step"][0] == 1


def test_locking_step(oracle_lib):
    # crank 1, coupler 1, rocker 1, ground 2.5: joint 3 reachable only while |p1 - O4| <= 2
    m = {"n": 4, "edges": FB, "fixed": [0, 2], "x0": [[0, 0], [1, 0], [2.5, 0], [1.75, 0.6614378277661477]]}
    r = run([m], T=8)
    # |p1 - O4| = |e^{i theta} - 2.5|: 1.5 at t=0, 1.93 at t=1 (45 deg), 2.69 at t=2 (90 deg)
    assert r["status"][0] == oracle.LOCKED and r["fail_step"][0] == 2


def test_bad_inputs(oracle_lib):
    ok = {"n": 4, "edges": FB, "fixed": [0, 2], "x0": X_FB}
    zero_link = dict(ok, x0=[[0, 0], [1, 0], [4, 0], [1, 0]])
    nan_pos = dict(ok, x0=[[0, 0], [1, 0], [4, 0], [np.nan, 1]])
    r = run([ok, zero_link, nan_pos])
    assert r["status"].tolist() == [oracle.VALID, oracle.BAD_MECH, oracle.BAD_MECH]
    assert r["fail_step"].tolist() == [-1, -1, -1]
    b = mech.build([ok])
    b.adj[0, 1] = 0
    assert oracle.simulate(b)["status"][0] == oracle.BAD_MECH
    triad = {"n": 6, "edges": [(0, 1), (1, 3), (2, 4), (0, 5), (3, 4), (4, 5), (3, 5)], "fixed": [0, 2],
             "x0": np.random.default_rng(0).random((6, 2))}
    assert run([triad])["status"][0] == oracle.UNSOLVABLE


def test_explicit_output_joint_and_nan_padding(oracle_lib):
    m = {"n": 4, "edges": FB, "fixed": [0, 2], "x0": [[0, 0], [1, 0], [2.5, 0], [1.75, 0.6614378277661477]]}
    b = mech.build([m])
    r = oracle.simulate(b, T=8, out_joint=1, path=True)
    h = 0.5 ** 0.5
    assert np.allclose(r["path"][0, :2], [[1, 0], [h, h]]) and np.all(np.isnan(r["path"][0, 2:]))
