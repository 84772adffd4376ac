"""The oracle's pins are strong enough to catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (on the CPU),
builds it, and requires that at least one pin test fails against it.
"""
import os

import pytest

import oracle
from tests import test_oracle_fixtures as fx
from tests import test_oracle_fourbar as fb
from tests import test_oracle_curate as cu
from tests import test_oracle_order as od
from tests import test_oracle_branch as br
from tests import test_oracle_margins as mg

MUTATIONS = {
    "offset_sign": ("double ox = -(h / d) * dy;", "double ox = (h / d) * dy;"),
    "swapped_radii": ("double along = (d2 + ra2 - rb2) / (2.0 * d);", "double along = (d2 - ra2 + rb2) / (2.0 * d);"),
    "foot_over_d2": ("double along = (d2 + ra2 - rb2) / (2.0 * d);", "double along = (d2 + ra2 - rb2) / (2.0 * d2);"),
    "branch_inverted": ("left = dp2 <= dm2;", "left = dp2 > dm2;"),
    "orientation_flipped": ("left0[s] = cr >= 0.0;", "left0[s] = cr < 0.0;"),
    "clockwise_crank": ("double theta = 2.0 * M_PI * (double)t / (double)T;",
                        "double theta = -2.0 * M_PI * (double)t / (double)T;"),
    "tip_y_sign": ("pos[tip][1] = x0[2 * pivot + 1] + (st * vx + ct * vy);",
                   "pos[tip][1] = x0[2 * pivot + 1] + (st * vx - ct * vy);"),
    "discriminant_term": ("double K = (sum * sum - d2) * (d2 - dif * dif);",
                          "double K = (sum * sum - d2) * (d2 + dif * dif);"),
    "lock_threshold": ("if (K < 0.0) {", "if (K < -1e-4 * scale2 * scale2) {"),
    "height_factor": ("double h = sqrt(K) / (2.0 * d);", "double h = sqrt(K) / d;"),
    "no_depth_count": ("    rounds++;\n", "\n"),
    "largest_parent": ("int a = lowest_bit(kn);", "int a = 31 - __builtin_clz(kn);"),
    "descending_round": ("for (int k = 0; k < n; k++) {\n      if ((known >> k) & 1u) continue;",
                         "for (int k = n - 1; k >= 0; k--) {\n      if ((known >> k) & 1u) continue;"),
    "drift_ignored": ("if (drift > A->tau_drift * scale) {", "if (drift > 1e9 * A->tau_drift * scale) {"),
    "skip_last_step": ("for (int t = 0; t < T; t++) {\n    /* actuator", "for (int t = 0; t < T - 1; t++) {\n    /* actuator"),
    "radial_not_squared": ("      var += e * e;", "      var += fabs(e);"),
    "ancestors_forward": ("for (int s = nd - 1; s >= 0; s--) {\n      int k = order[3 * s];",
                          "for (int s = 0; s < nd; s++) {\n      int k = order[3 * s];"),
    "arc_any_link": ("if (a[out] & fixed[c]) f |= LREF_CUR_ARC;", "if (a[out]) f |= LREF_CUR_ARC;"),
    # the band margins that decide which candidates are excused from bit-exact parity
    "branch_margin_x10": ("if (side / scale < m_branch) m_branch = side / scale;",
                          "if (10.0 * side / scale < m_branch) m_branch = 10.0 * side / scale;"),
    "branch_margin_to_base": (
        "double side = fabs((prev[k][0] - bx) * (-dy) + (prev[k][1] - by) * dx) / d;",
        "double side = sqrt((prev[k][0] - bx) * (prev[k][0] - bx) + (prev[k][1] - by) * (prev[k][1] - by));"),
    "branch_margin_not_over_d": ("double side = fabs((prev[k][0] - bx) * (-dy) + (prev[k][1] - by) * dx) / d;",
                                 "double side = fabs((prev[k][0] - bx) * (-dy) + (prev[k][1] - by) * dx);"),
    "drift_margin_without_tau": ("double md = fabs(drift - A->tau_drift * scale) / scale;",
                                 "double md = fabs(drift) / scale;"),
    "drift_margin_unscaled": ("double md = fabs(drift - A->tau_drift * scale) / scale;",
                              "double md = fabs(drift - A->tau_drift * scale);"),
    "disc_margin_unscaled": ("if (fabs(disc) / scale2 < m_disc) m_disc = fabs(disc) / scale2;",
                             "if (fabs(disc) < m_disc) m_disc = fabs(disc);"),
    "deg_margin_unscaled": ("if (d2 / scale2 < m_deg) m_deg = d2 / scale2;", "if (d2 < m_deg) m_deg = d2;"),
}

PINS = [
    lambda: fb.test_worked_example_positions(None),
    lambda: fb.test_grid_exact_lock_prediction(None),
    lambda: fb.test_freudenstein_rocker_angle(None),
    lambda: od.test_fourbar_worked_order(None),
    lambda: od.test_order_matches_brute_force_on_small_random_graphs(None),
    lambda: fx.test_redundant_links_drift(None),
    lambda: fx.test_locking_step(None),
    lambda: cu.test_fourbar_arcs_circles_and_reduction(None),
    lambda: cu.test_radial_variance_of_an_ellipse(None),
    lambda: cu.test_reduced_mechanism_reproduces_the_path(None),
    br.test_rules_keep_their_invariants,
    br.test_rules_agree_where_continuity_keeps_the_starting_sides,
    lambda: fb.test_discriminant_and_distance_margins_closed_form(None),
    mg.test_branch_margin_fourbar_closed_form,
    mg.test_margins_of_a_crank_carried_joint_closed_form,
    mg.test_drift_margin_of_the_crank_tip_closed_form,
    mg.test_drift_margin_through_the_rocker_closed_form,
]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path, oracle_lib):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "links_ref.c")).read()
    old, new = MUTATIONS[name]
    assert src.count(old) == 1, "mutation anchor must match the source exactly once"
    lib = oracle.build_variant(src.replace(old, new), str(tmp_path / f"liblinks_ref_{name}.so"))
    oracle.use_library(lib)
    try:
        caught = []
        for i, pin in enumerate(PINS):
            try:
                pin()
            except AssertionError:
                caught.append(i)
        assert caught, f"no pin detects the planted mistake '{name}'"
    finally:
        oracle.use_library(None)


def test_unmodified_source_passes_all_pins(oracle_lib):
    for pin in PINS:
        pin()
