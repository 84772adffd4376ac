"""The configuration table: its bands are the library's defaults and its host
workloads exist (CPU; the library is loaded but no device is used)."""
import ctypes

import pytest

from paper_2208_14567_amd import gen
from paper_2208_14567_amd.configs import BANDS, CONFIGS, T


def test_bands_are_the_library_defaults():
    from paper_2208_14567_amd import links
    L = links.load()
    o = links.SimOpts()
    L.links_sim_opts_default(ctypes.byref(o))
    assert o.T == T
    assert (o.eps_disc, o.eps_branch, o.tau_drift) == (BANDS["eps_disc"], BANDS["eps_branch"], BANDS["tau_drift"])


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "cfg2_rules", "cfg3", "cfg4"])
def test_workloads_exist(name):
    c = CONFIGS[name]
    b = gen.workload(c["workload"], 3, seed=c["seed"])
    assert b.B == 3 and c["T"] == T
