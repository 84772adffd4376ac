"""The oracle's input validation against the contract's rules: every way of
breaking a candidate gives BAD_MECH, and what the contract ignores (positions
beyond the joint count) changes nothing."""
import numpy as np

import oracle
from paper_2208_14567_amd import gen
from tests import mech


def test_each_break_is_bad_mech():
    b = gen.dyad_batch(600, 91, gen.n_uniform(4, 12), J=16)
    ref = oracle.simulate(b, T=8)
    m, kinds = mech.malform(b, seed=5)
    r = oracle.simulate(m, T=8)
    _, _, _, so = oracle.solve_order(m)
    seen = set()
    for c in range(b.B):
        name = mech.MALFORM_KINDS[kinds[c]]
        seen.add(name)
        if name in mech.MALFORM_EITHER:
            continue
        if name in mech.MALFORM_BENIGN:
            assert r["status"][c] == ref["status"][c] and r["fail_step"][c] == ref["fail_step"][c], name
        else:
            assert r["status"][c] == oracle.BAD_MECH, (c, name)
            assert r["fail_step"][c] == -1
            # the solve order checks structure only: broken positions pass it
            if name not in ("nan_position", "inf_position", "zero_length_link"):
                assert so[c] == oracle.BAD_MECH, (c, name)
    assert seen >= set(mech.MALFORM_KINDS) - {"untouched"}
