"""On-device candidate generation against the host generator: the same seed and
candidate indices give bit-identical batches (joint counts, adjacency, fixed
masks, motor pairs and positions)."""
import sys

import numpy as np
import pytest

from paper_2208_14567_amd import gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed,first,B,J,lo,hi,paper,rules", [
    (2, 0, 5000, 20, 6, 20, False, False),
    (5, 99_990_000, 4133, 20, 6, 20, False, False),   # deep into a 100M stream, ragged size
    (4, 12345, 3001, 20, 4, 20, False, False),
    (6, 777, 2500, 20, 8, 20, True, False),           # paper mode: ground joints and standard arm
    (9, 0, 1000, 32, 20, 32, False, False),           # widest stride
    (3, 5, 1, 7, 3, 7, False, False),
    (12, 0, 5000, 20, 5, 20, False, True),            # the paper's topology rules
    (13, 4242, 3000, 20, 8, 20, True, True),          # paper mode with the rules
    (14, 0, 1000, 32, 5, 32, True, True),
])
def test_device_generator_matches_host(seed, first, B, J, lo, hi, paper, rules):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_14567_amd import links as L
    print(f"[gen] seed={seed} first={first} B={B} J={J} n={lo}..{hi} paper={paper} rules={rules}", flush=True)
    sys.stdout.flush()
    ctx = L.Context(0)
    d = ctx.generate_dyads(B, seed, first=first, J=J, n_lo=lo, n_hi=hi, paper_mode=paper, rules=rules)
    h = gen.dyad_batch(B, seed, gen.n_uniform(lo, hi), J=J, paper_mode=paper, first=first, rules=rules)
    if paper:
        h = gen.standardize_paper(h)
    assert np.array_equal(d.n.cpu().numpy(), h.n)
    assert np.array_equal(d.adj.cpu().numpy().view(np.uint32), h.adj)
    assert np.array_equal(d.fixed.cpu().numpy().view(np.uint32), h.fixed)
    assert np.array_equal(d.motor.cpu().numpy(), h.motor)
    assert np.array_equal(d.x0.cpu().numpy(), h.x0)
    ctx.close()


def test_device_generator_rejects_bad_arguments():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_14567_amd import links as L
    ctx = L.Context(0)
    for kw in ({"n_lo": 2}, {"n_lo": 10, "n_hi": 9}, {"n_hi": 21}, {"J": 33, "n_hi": 20}, {"n_lo": 4, "rules": True}):
        with pytest.raises(L.LinksError):
            ctx.generate_dyads(10, 1, **kw)
    ctx.close()
