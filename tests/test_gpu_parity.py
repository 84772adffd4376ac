"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars (element by element, same seeded inputs):
* solve order, n_dyads, depth, status of links_solve_order: bit-exact;
* FP64 precision: status and fail_step bit-exact for every candidate, paths
  bit-exact (the FP64 pass evaluates the same correctly rounded operations);
* FP32 with escalation: status and fail_step bit-exact for every candidate whose
  oracle margins are outside the bands (|disc| >= 1e-6 scale^2, d^2 >= 1e-6
  scale^2, branch distance >= 1e-5 scale, drift margin >= 0.9e-4 scale); paths
  within 1e-5 scale at every written step.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2208_14567_amd import gen
from tests import mech

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NTH = min(16, os.cpu_count() or 1)

# Upper bound on the share of candidates the oracle calls in-band.  On the
# workloads of up to 20 joints here it is 0 (Grashof four-bars) to 8.4%
# (paper-mode positions), almost all of it the discriminant band at the grid step
# before a lock; it grows with the number of placed joints (14.1% for 20 to 32
# joints, which get their own bound).  A margin that reports too small a distance
# would move candidates in band and out of the bit-exact comparison; the bound
# keeps that from emptying a test.
IN_BAND_MAX = 0.10


def _check_in_band(ib, label="", bound=IN_BAND_MAX):
    assert ib.mean() <= bound, f"{label}: {ib.mean():.3%} of candidates in band"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_14567_amd import links
    return links


@pytest.fixture(scope="module")
def ctx(L):
    return L.Context(0)


def _np(r):
    return {k: v.cpu().numpy() for k, v in r.items()}


def _scale(b):
    return mech.scale_of(b)


WORKLOADS = [("fourbar", 4000, 1), ("fourbar_u", 4000, 11), ("dyad_6_20", 20000, 2), ("dyad_skewed", 20000, 3),
             ("dyad_4_20", 8000, 4), ("paper_8_20", 6000, 6)]


@pytest.mark.parametrize("name,B,seed", WORKLOADS)
def test_solve_order_bit_exact(ctx, L, name, B, seed):
    _say(f"[solve_order] {name} B={B}")
    b = gen.workload(name, B, seed=seed)
    o, nd, dp, st = ctx.solve_order(L.to_device(b))
    ro, rnd, rdp, rst = oracle.solve_order(b)
    assert np.array_equal(o.cpu().numpy(), ro)
    assert np.array_equal(nd.cpu().numpy(), rnd) and np.array_equal(dp.cpu().numpy(), rdp)
    assert np.array_equal(st.cpu().numpy(), rst)


def _fixtures():
    rng = np.random.default_rng(0)
    FB = [(0, 1), (1, 3), (2, 3)]
    X = [[0, 0], [1, 0], [4, 0], [11 / 3, 4 * 5 ** 0.5 / 3]]
    ms = [
        {"n": 4, "edges": FB + [(1, 2)], "fixed": [0, 2], "x0": X},                       # drift at step 1
        {"n": 5, "edges": FB + [(0, 4), (1, 4), (3, 4)], "fixed": [0, 2], "x0": X + [[0.5, 0.8]]},
        {"n": 4, "edges": FB, "fixed": [0, 2], "x0": [[0, 0], [1, 0], [0, 1], [0.5, 0.5]]},  # degenerate
        {"n": 4, "edges": FB, "fixed": [0, 2], "x0": [[0, 0], [1, 0], [2.5, 0], [1.75, 0.6614378277661477]]},
        {"n": 6, "edges": [(0, 1), (1, 3), (2, 4), (0, 5), (3, 4), (4, 5), (3, 5)], "fixed": [0, 2],
         "x0": rng.random((6, 2))},                                                      # unsolvable
        {"n": 4, "edges": FB, "fixed": [0, 2], "x0": [[0, 0], [1, 0], [4, 0], [1, 0]]},   # zero-length link
        {"n": 5, "edges": [(0, 1), (0, 3), (1, 3), (0, 4), (1, 4), (3, 4)], "fixed": [0, 2],
         "x0": [[0, 0], [1, 0], [5, 5], [0.3, 0.9], [0.8, -0.6]]},                       # consistent redundancy
        {"n": 3, "edges": [(0, 1)], "fixed": [0, 2], "x0": [[0, 0], [1, 0], [2, 2]]},     # no placed joints
    ]
    b = mech.build(ms, J=8)
    b.adj[5] = b.adj[5]
    return b


@pytest.mark.parametrize("precision", [0, 1])
def test_status_fixtures(ctx, L, precision):
    _say(f"[fixtures] precision={precision}")
    b = _fixtures()
    for T in (4, 8, 200):
        r = _np(ctx.simulate(L.to_device(b), T=T, precision=precision, write=L.WRITE_ALL, path_dtype=L.F64))
        ref = oracle.simulate(b, T=T, path=True)
        assert np.array_equal(r["status"], ref["status"]), (T, r["status"], ref["status"])
        assert np.array_equal(r["fail_step"], ref["fail_step"])
        assert np.array_equal(np.isnan(r["path"]), np.isnan(ref["path"]))
        tol = 1e-12 if precision == 1 else 1e-5 * _scale(b).max()
        assert np.allclose(r["path"], ref["path"], rtol=0, atol=tol, equal_nan=True)


def test_parallel_in_time_fp64_passes(ctx, L):
    """Every FP64 pass computed parallel in time gives the step-by-step results
    bit for bit (statuses, steps and paths), in both precisions."""
    _say("[par64]")
    b = gen.workload("dyad_4_20", 20000, seed=21)
    db = L.to_device(b)
    res = {}
    try:
        for mode in (0, 1, 2):
            ctx.set_option("par64", mode)
            for precision in (L.FP64, L.FP32_RECHECK):
                r = _np(ctx.simulate(db, T=200, precision=precision, write=L.WRITE_ALL, path_dtype=L.F64))
                res[mode, precision] = r
    finally:
        ctx.set_option("par64", 1)
    for precision in (L.FP64, L.FP32_RECHECK):
        for mode in (1, 2):
            a, z = res[0, precision], res[mode, precision]
            for k in ("status", "fail_step", "esc_step"):
                assert np.array_equal(a[k], z[k]), (precision, mode, k)
            assert np.array_equal(a["path"], z["path"], equal_nan=True), (precision, mode)
    try:
        for seg in (4, 16):   # hand-over segment widths besides the default 8
            ctx.set_option("seg64", seg)
            z = _np(ctx.simulate(db, T=200, precision=L.FP32_RECHECK, write=L.WRITE_ALL, path_dtype=L.F64))
            a = res[0, L.FP32_RECHECK]
            for k in ("status", "fail_step", "esc_step"):
                assert np.array_equal(a[k], z[k]), (seg, k)
            assert np.array_equal(a["path"], z["path"], equal_nan=True), seg
    finally:
        ctx.set_option("seg64", 8)
    ref = oracle.simulate(b, T=200, path=True, nthreads=NTH)
    z = res[2, L.FP64]
    assert np.array_equal(z["status"], ref["status"]) and np.array_equal(z["fail_step"], ref["fail_step"])
    assert np.array_equal(z["path"], ref["path"], equal_nan=True)


@pytest.mark.parametrize("name,B,seed", [("dyad_6_20", 40000, 23), ("dyad_skewed", 40000, 24),
                                         ("fourbar_u", 8000, 25)])
def test_drain_handed_to_parallel_pass(ctx, L, name, B, seed):
    """Once the work list is exhausted, nearly empty waves of the step-by-step FP32
    pass hand their candidates (columns, error bounds, next step) to the
    parallel-in-time pass: every decision, hand-over step and path equals the
    pass without the hand-off, in both FP32 precisions and whatever the
    threshold."""
    _say(f"[drain] {name} B={B}")
    b = gen.workload(name, B, seed=seed)
    db = L.to_device(b)
    prev = ctx.get_option("drain32")
    try:
        for precision in (L.FP32_RECHECK, L.FP32_ONLY):
            ctx.set_option("drain32", 0)
            base = _np(ctx.simulate(db, T=200, precision=precision, write=L.WRITE_ALL))
            for thr in (1, 16, 48, 65):
                ctx.set_option("drain32", thr)
                r = _np(ctx.simulate(db, T=200, precision=precision, write=L.WRITE_ALL))
                for k in ("status", "fail_step", "esc_step"):
                    diff = np.nonzero(r[k] != base[k])[0]
                    assert diff.size == 0, (precision, thr, k, diff[:5])
                assert np.array_equal(r["path"], base["path"], equal_nan=True), (precision, thr)
            for T in (1, 15, 16, 17, 1500):   # short rotations, one segment pass, a global crank table
                ctx.set_option("drain32", 0)
                base = _np(ctx.simulate(db, T=T, precision=precision))
                ctx.set_option("drain32", 65)
                r = _np(ctx.simulate(db, T=T, precision=precision))
                for k in ("status", "fail_step", "esc_step"):
                    assert np.array_equal(r[k], base[k]), (precision, T, k)
    finally:
        ctx.set_option("drain32", prev)


@pytest.mark.parametrize("name,B,seed,T", [("dyad_6_20", 30000, 29, 200), ("dyad_skewed", 30000, 30, 200),
                                           ("fourbar_u", 6000, 31, 200), ("dyad_4_20", 10000, 32, 77),
                                           ("paper_8_20", 10000, 33, 1500)])
def test_path_rows_in_chunks(ctx, L, name, B, seed, T):
    """Path rows computed in 32-step chunks from the sides the FP32 pass and the
    FP64 hand-over pass record at chunk ends equal rows computed whole, bit for
    bit, with either hand-over pass and both write modes (FP32 decisions with
    escalation; without escalation rows are always computed whole)."""
    _say(f"[row chunks] {name} B={B} T={T}")
    b = gen.workload(name, B, seed=seed)
    db = L.to_device(b)
    prev = (ctx.get_option("path_chunks"), ctx.get_option("par64"))
    try:
        for precision in (L.FP32_RECHECK, L.FP32_ONLY):
            for par in (0, 1):
                ctx.set_option("par64", par)
                res = {}
                for ck in (0, 1):
                    ctx.set_option("path_chunks", ck)
                    res[ck] = _np(ctx.simulate(db, T=T, precision=precision, write=L.WRITE_ALL, path_dtype=L.F64))
                for k in ("status", "fail_step", "esc_step"):
                    assert np.array_equal(res[0][k], res[1][k]), (precision, par, k)
                diff = ~((res[0]["path"] == res[1]["path"]) | (np.isnan(res[0]["path"]) & np.isnan(res[1]["path"])))
                assert not diff.any(), (precision, par, np.nonzero(diff.any(axis=(1, 2)))[0][:5])
            ctx.set_option("path_chunks", 1)
            v = _np(ctx.simulate(db, T=T, precision=precision, write=L.WRITE_VALID, cap=B))
            k = int(v["n_written"][0])
            assert np.array_equal(v["path"][:k], res[0]["path"][v["path_index"][:k]].astype(np.float32),
                                  equal_nan=True)
    finally:
        ctx.set_option("path_chunks", prev[0])
        ctx.set_option("par64", prev[1])


def test_handover_queue_order(ctx, L):
    """The FP64 hand-over pass takes its queue as handed over or ordered by
    hand-over step: the same decisions and paths either way (and with the
    step-by-step or parallel-in-time hand-over pass)."""
    _say("[hand-over order]")
    b = gen.workload("dyad_6_20", 40000, seed=28)
    db = L.to_device(b)
    prev = (ctx.get_option("sort_esc"), ctx.get_option("par64"))
    res = {}
    try:
        for sort in (0, 1):
            for par in (0, 1):
                ctx.set_option("sort_esc", sort)
                ctx.set_option("par64", par)
                res[sort, par] = _np(ctx.simulate(db, T=200, write=L.WRITE_ALL))
    finally:
        ctx.set_option("sort_esc", prev[0])
        ctx.set_option("par64", prev[1])
    a = res[0, 1]
    assert (a["esc_step"] >= 0).sum() > 1000
    for key, z in res.items():
        for k in ("status", "fail_step", "esc_step"):
            assert np.array_equal(a[k], z[k]), (key, k)
        assert np.array_equal(a["path"], z["path"], equal_nan=True), key


@pytest.mark.parametrize("name,B,seed,T,branch", [("dyad_6_20", 30000, 41, 200, 0), ("dyad_4_20", 20000, 42, 77, 0),
                                                  ("paper_8_20", 8000, 43, 200, 0), ("dyad_skewed", 20000, 44, 1500, 0),
                                                  ("dyad_6_20", 20000, 45, 200, 1), ("fourbar_u", 5000, 46, 200, 0),
                                                  ("dyad_4_20", 5000, 48, 1, 0), ("dyad_4_20", 5000, 49, 2, 0),
                                                  ("dyad_4_20", 5000, 50, 63, 0), ("dyad_4_20", 5000, 51, 64, 0),
                                                  ("dyad_4_20", 5000, 52, 127, 1)])
def test_wave_per_candidate_fp64_passes(ctx, L, name, B, seed, T, branch):
    """The FP64 passes with one candidate per wave (positions in registers, 63
    steps per round) take every decision of the segmented and step-by-step passes:
    statuses, failure and hand-over steps and path rows equal bit for bit, for the
    hand-over pass, the path pass and the FP64 decision pass, alone and together."""
    _say(f"[wave64] {name} B={B} T={T} branch={branch}")
    b = gen.workload(name, B, seed=seed)
    db = L.to_device(b)
    prev = ctx.get_option("wave64")
    res = {}
    try:
        for precision in (L.FP32_RECHECK, L.FP64):
            for mode in (0, 1, 2, 4, 7):
                ctx.set_option("wave64", mode)
                res[precision, mode] = _np(ctx.simulate(db, T=T, precision=precision, branch=branch,
                                                        write=L.WRITE_ALL, path_dtype=L.F64))
    finally:
        ctx.set_option("wave64", prev)
    for precision in (L.FP32_RECHECK, L.FP64):
        a = res[precision, 0]
        assert (a["status"] == 0).sum() > 20
        if precision == L.FP32_RECHECK:
            assert (a["esc_step"] >= 0).sum() > 20
        for mode in (1, 2, 4, 7):
            z = res[precision, mode]
            for k in ("status", "fail_step", "esc_step"):
                assert np.array_equal(a[k], z[k]), (precision, mode, k)
            assert np.array_equal(a["path"], z["path"], equal_nan=True), (precision, mode)
    ref = oracle.simulate(b, T=T, branch=branch, path=True, nthreads=NTH)
    z = res[L.FP64, 7]
    assert np.array_equal(z["status"], ref["status"]) and np.array_equal(z["fail_step"], ref["fail_step"])
    assert np.array_equal(z["path"], ref["path"], equal_nan=True)


@pytest.mark.parametrize("precision", [0, 1])
def test_wave_per_candidate_status_fixtures(ctx, L, precision):
    """The wave-per-candidate FP64 passes on the fixtures (a drifting link, a
    consistent redundant link, degenerate and locking mechanisms, no placed
    joints): statuses, failure steps and paths equal to the oracle's."""
    b = _fixtures()
    prev = ctx.get_option("wave64")
    try:
        ctx.set_option("wave64", 7)
        for T in (4, 8, 200):
            r = _np(ctx.simulate(L.to_device(b), T=T, precision=precision, write=L.WRITE_ALL, path_dtype=L.F64))
            ref = oracle.simulate(b, T=T, path=True)
            assert np.array_equal(r["status"], ref["status"]), (T, r["status"], ref["status"])
            assert np.array_equal(r["fail_step"], ref["fail_step"])
            assert np.array_equal(np.isnan(r["path"]), np.isnan(ref["path"]))
            tol = 1e-12 if precision == 1 else 1e-5 * _scale(b).max()
            assert np.allclose(r["path"], ref["path"], rtol=0, atol=tol, equal_nan=True)
    finally:
        ctx.set_option("wave64", prev)


def test_wave_per_candidate_falls_back_above_20_joints(ctx, L):
    """Above 20 joints the wave-per-candidate kernels do not apply and the other
    passes run: results equal with the option on or off."""
    b = gen.Batch.concat([gen.dyad_batch(3000, 47, gen.n_uniform(6, 24), J=24)])
    db = L.to_device(b)
    prev = ctx.get_option("wave64")
    try:
        ctx.set_option("wave64", 7)
        z = _np(ctx.simulate(db, T=200, write=L.WRITE_ALL, path_dtype=L.F64))
        ctx.set_option("wave64", 0)
        a = _np(ctx.simulate(db, T=200, write=L.WRITE_ALL, path_dtype=L.F64))
    finally:
        ctx.set_option("wave64", prev)
    for k in ("status", "fail_step", "esc_step"):
        assert np.array_equal(a[k], z[k]), k
    assert np.array_equal(a["path"], z["path"], equal_nan=True)


@pytest.mark.parametrize("precision,T,branch", [(0, 200, 0), (2, 200, 0), (0, 77, 0), (0, 200, 1)])
def test_parallel_in_time_fp32_pass(ctx, L, precision, T, branch):
    """The FP32 pass computed parallel in time takes every decision of the
    step-by-step pass: statuses, failure and hand-over steps and paths equal (with
    FP32 decisions and escalation the rows are computed in chunks from the sides
    either pass records)."""
    _say(f"[par32] precision={precision} T={T} branch={branch}")
    b = gen.workload("dyad_6_20", 30000, seed=22)
    db = L.to_device(b)
    res = {}
    prev = ctx.get_option("par32")
    try:
        for mode in (0, 1):
            ctx.set_option("par32", mode)
            res[mode] = _np(ctx.simulate(db, T=T, precision=precision, branch=branch, write=L.WRITE_ALL,
                                         path_dtype=L.F64))
    finally:
        ctx.set_option("par32", prev)
    a, z = res[0], res[1]
    for k in ("status", "fail_step", "esc_step"):
        diff = np.nonzero(a[k] != z[k])[0]
        assert diff.size == 0, (k, diff[:10], a[k][diff[:10]], z[k][diff[:10]])
    assert np.array_equal(a["path"], z["path"], equal_nan=True)


ORIENT_WORKLOADS = [("fourbar_u", 4000, 31), ("dyad_6_20", 20000, 32), ("paper_8_20", 6000, 33)]


@pytest.mark.parametrize("name,B,seed", ORIENT_WORKLOADS)
def test_orientation_rule_parity(ctx, L, name, B, seed):
    """The orientation branch rule: FP64 bit-exact with the oracle's orientation
    rule (statuses, steps, paths); FP32 with escalation equal to it outside the
    bands, paths within 1e-5 of the scale."""
    _say(f"[orientation] {name} B={B}")
    b = gen.workload(name, B, seed=seed)
    r = _np(ctx.simulate(L.to_device(b), T=200, precision=L.FP64, write=L.WRITE_ALL, path_dtype=L.F64,
                         branch=L.BRANCH_ORIENTATION))
    ref = oracle.simulate(b, T=200, path=True, nthreads=NTH, branch=oracle.BRANCH_ORIENTATION)
    assert np.array_equal(r["status"], ref["status"]) and np.array_equal(r["fail_step"], ref["fail_step"])
    assert np.array_equal(r["path"], ref["path"], equal_nan=True)
    cont = oracle.simulate(b, T=200, nthreads=NTH)
    _say(f"   statuses differing from the continuity rule: {(cont['status'] != ref['status']).mean():.4f}")
    _fp32_parity(ctx, L, b, label=f"{name} orientation", branch=L.BRANCH_ORIENTATION)


def test_orientation_rule_parallel_passes(ctx, L):
    """Under the orientation rule the parallel-in-time passes (no side changes to
    restart on) give the step-by-step results."""
    b = gen.workload("dyad_4_20", 20000, seed=34)
    db = L.to_device(b)
    p32, p64 = ctx.get_option("par32"), ctx.get_option("par64")
    res = {}
    try:
        for m32, m64 in ((0, 0), (1, 2)):
            ctx.set_option("par32", m32)
            ctx.set_option("par64", m64)
            for precision in (L.FP64, L.FP32_RECHECK):
                res[m32, precision] = _np(ctx.simulate(db, T=200, precision=precision, write=L.WRITE_ALL,
                                                       path_dtype=L.F64, branch=L.BRANCH_ORIENTATION))
    finally:
        ctx.set_option("par32", p32)
        ctx.set_option("par64", p64)
    for precision in (L.FP64, L.FP32_RECHECK):
        a, z = res[0, precision], res[1, precision]
        for k in ("status", "fail_step", "esc_step"):
            assert np.array_equal(a[k], z[k]), (precision, k)
        assert np.array_equal(a["path"], z["path"], equal_nan=True), precision


@pytest.mark.parametrize("J", [7, 10, 13, 20, 22, 32])
def test_malformed_candidates(ctx, L, J):
    """Every way of breaking the input contract, mixed into valid batches of each
    joint-stride class: statuses and failure steps as the oracle's."""
    _say(f"[malformed] J={J}")
    b = gen.dyad_batch(3000, 300 + J, gen.n_uniform(4, J), J=J)
    m, kinds = mech.malform(b, seed=J)
    ref = oracle.simulate(m, T=50, nthreads=NTH)
    for precision in (L.FP64, L.FP32_RECHECK):
        r = _np(ctx.simulate(L.to_device(m), T=50, precision=precision))
        # the set-up decides UNSOLVABLE and BAD_MECH exactly in both precisions
        pre = np.isin(ref["status"], (oracle.UNSOLVABLE, oracle.BAD_MECH)) | np.isin(r["status"], (4, 5))
        bad = pre & (r["status"] != ref["status"])
        if precision == L.FP64:
            bad |= r["status"] != ref["status"]
        assert not bad.any(), (precision, [mech.MALFORM_KINDS[k] for k in kinds[bad][:5]])
        if precision == L.FP64:
            assert np.array_equal(r["fail_step"], ref["fail_step"])
    _, _, _, st = ctx.solve_order(L.to_device(m))
    assert np.array_equal(st.cpu().numpy(), oracle.solve_order(m)[3])


@pytest.mark.parametrize("name,B,seed", WORKLOADS)
def test_fp64_bit_exact(ctx, L, name, B, seed):
    _say(f"[fp64] {name} B={B}")
    b = gen.workload(name, B, seed=seed)
    r = _np(ctx.simulate(L.to_device(b), T=200, precision=L.FP64, write=L.WRITE_ALL, path_dtype=L.F64))
    ref = oracle.simulate(b, T=200, path=True, nthreads=NTH)
    assert np.array_equal(r["status"], ref["status"])
    assert np.array_equal(r["fail_step"], ref["fail_step"])
    assert np.all(r["esc_step"] == -1)          # FP64 throughout: nothing handed over
    same = (r["path"] == ref["path"]) | (np.isnan(r["path"]) & np.isnan(ref["path"]))
    assert same.all(), f"{(~same.all(axis=(1, 2))).sum()} paths differ in some bit"


def _fp32_parity(ctx, L, b, T=200, write=None, label="", branch=0, in_band_max=IN_BAND_MAX):
    write = L.WRITE_ALL if write is None else write
    r = _np(ctx.simulate(L.to_device(b), T=T, precision=L.FP32_RECHECK, write=write, branch=branch))
    ref = oracle.simulate(b, T=T, path=True, margins=True, nthreads=NTH, branch=branch)
    ib = oracle.in_band(ref["margins"])
    _check_in_band(ib, label, in_band_max)
    clear = ~ib
    bad = clear & ((r["status"] != ref["status"]) | (r["fail_step"] != ref["fail_step"]))
    agree_in = ((r["status"] == ref["status"]) & (r["fail_step"] == ref["fail_step"]))[ib].mean() if ib.any() else 1.0
    esc = (r["esc_step"] >= 0).mean()
    _say(f"   {label}: out-of-band {clear.sum()} mismatches {bad.sum()}; in-band {ib.sum()} agree {agree_in:.3f}; "
         f"handed to FP64 {esc:.3%}")
    assert bad.sum() == 0, np.nonzero(bad)[0][:10]
    if write == L.WRITE_ALL:
        sc = _scale(b)
        ok = clear & (ref["status"] == r["status"]) & (ref["fail_step"] == r["fail_step"])
        nan_r, nan_o = np.isnan(r["path"][ok]), np.isnan(ref["path"][ok])
        assert np.array_equal(nan_r, nan_o)
        err = np.where(nan_o, 0.0, np.abs(r["path"][ok] - ref["path"][ok])).max(axis=(1, 2))
        assert np.all(err <= 1e-5 * sc[ok]), (err / sc[ok]).max()
        _say(f"   {label}: max path error / scale {(err / sc[ok]).max():.2e}")
    return r, ref


@pytest.mark.parametrize("name,B,seed", WORKLOADS)
def test_fp32_recheck_parity(ctx, L, name, B, seed):
    _say(f"[fp32r] {name} B={B}")
    b = gen.workload(name, B, seed=seed)
    _fp32_parity(ctx, L, b, label=name)


def test_fp32_recheck_narrow_bands(ctx, L):
    """Bands far below the defaults (eps_disc = 1e-9, no branch band): the FP32
    pass may then take a decision in FP32 only where its tracked error bound,
    including the rounding of the discriminant and of the placement themselves,
    keeps it away from the threshold; everything outside these bands must equal
    the oracle."""
    _say("[fp32r narrow bands]")
    b = gen.Batch.concat([gen.workload("dyad_6_20", 20000, seed=26), gen.workload("fourbar_u", 4000, seed=27)])
    r = _np(ctx.simulate(L.to_device(b), T=200, precision=L.FP32_RECHECK, eps_disc=1e-9, eps_branch=0.0))
    ref = oracle.simulate(b, T=200, margins=True, nthreads=NTH)
    ib = oracle.in_band(ref["margins"], eps_disc=1e-9, eps_branch=0.0)
    clear = ~ib
    bad = clear & ((r["status"] != ref["status"]) | (r["fail_step"] != ref["fail_step"]))
    _say(f"   out-of-band {clear.sum()} mismatches {bad.sum()}; in-band {ib.sum()}; "
         f"handed to FP64 {(r['esc_step'] >= 0).mean():.3%}")
    assert ib.mean() < 0.01
    assert bad.sum() == 0, np.nonzero(bad)[0][:10]


def test_fp32_recheck_parity_exact_handover(ctx, L):
    """The same bar with the hand-over pass evaluating the correctly rounded FP64
    sequence instead of reciprocal square roots with Newton steps."""
    _say("[fp32r exact hand-over]")
    b = gen.workload("dyad_6_20", 20000, seed=12)
    ctx.set_option("exact_handover", 1)
    try:
        _fp32_parity(ctx, L, b, label="exact hand-over")
    finally:
        ctx.set_option("exact_handover", 0)


@pytest.mark.parametrize("T", [1, 2, 50, 333])
def test_step_counts(ctx, L, T):
    _say(f"[T] {T}")
    b = gen.Batch.concat([gen.workload("fourbar_u", 1000, seed=5), gen.workload("dyad_6_20", 3000, seed=5)])
    _fp32_parity(ctx, L, b, T=T, label=f"T={T}")


@pytest.mark.parametrize("T", [1500, 4096])
def test_long_rotations(ctx, L, T):
    """More than 1024 actuator positions: the FP32 passes read the crank table
    from global memory instead of LDS.  FP64 bit-exact with the oracle; FP32 with
    escalation to the FP32 bar, step by step and parallel in time."""
    _say(f"[long T] {T}")
    b = gen.Batch.concat([gen.workload("fourbar_u", 1000, seed=51), gen.workload("dyad_6_20", 2000, seed=52)])
    db = L.to_device(b)
    ref = oracle.simulate(b, T=T, path=True, nthreads=NTH)
    r = _np(ctx.simulate(db, T=T, precision=L.FP64, write=L.WRITE_ALL, path_dtype=L.F64))
    assert np.array_equal(r["status"], ref["status"]) and np.array_equal(r["fail_step"], ref["fail_step"])
    assert np.array_equal(r["path"], ref["path"], equal_nan=True)
    prev = ctx.get_option("par32")
    try:
        for par in (0, 1):
            ctx.set_option("par32", par)
            # a finer grid puts the step before a lock nearer to it: 7.4% of this
            # batch is in band at T = 1500, 10.6% at T = 4096
            _fp32_parity(ctx, L, b, T=T, label=f"T={T} par32={par}", in_band_max=0.15)
    finally:
        ctx.set_option("par32", prev)


@pytest.mark.parametrize("T", [1, 7, 8, 13, 200, 201])
def test_small_mechanism_path_rows(ctx, L, T):
    """Path rows of small mechanisms (written in 64-byte groups): every row,
    including rows that end in a lock (NaN from the failing step) and step counts
    that are not a multiple of the group, equal the oracle's in f64 and its
    rounding in f32."""
    _say(f"[rows] T={T}")
    b = gen.workload("fourbar_u", 3000, seed=61)
    db = L.to_device(b)
    ref = oracle.simulate(b, T=T, path=True, nthreads=NTH)
    r64 = _np(ctx.simulate(db, T=T, precision=L.FP64, write=L.WRITE_ALL, path_dtype=L.F64))
    assert np.array_equal(r64["status"], ref["status"])
    assert np.array_equal(r64["path"], ref["path"], equal_nan=True)
    r32 = _np(ctx.simulate(db, T=T, precision=L.FP64, write=L.WRITE_ALL, path_dtype=L.F32))
    assert np.array_equal(r32["path"], ref["path"].astype(np.float32), equal_nan=True)
    assert np.isnan(ref["path"]).any() or T < 8


@pytest.mark.parametrize("T", [7, 13, 200, 201])
def test_path_rows_every_joint_count(ctx, L, T):
    """Path rows of mechanisms of every size class (written in staged groups of
    steps, or a store per step): FP64 rows equal the oracle's bit for bit in f64
    and f32; with FP32 decisions the path pass's rows are within 1e-5 scale of the
    oracle's and its f32 rows are its f64 rows rounded."""
    _say(f"[rows, all sizes] T={T}")
    b = gen.Batch.concat([gen.dyad_batch(1500, 90 + T, gen.n_uniform(4, 20), J=20),
                          gen.dyad_batch(500, 91 + T, gen.n_uniform(20, 32), J=32)])
    db = L.to_device(b)
    ref = oracle.simulate(b, T=T, path=True, nthreads=NTH)
    for precision in (L.FP64, L.FP32_RECHECK):
        r64 = _np(ctx.simulate(db, T=T, precision=precision, write=L.WRITE_ALL, path_dtype=L.F64))
        r32 = _np(ctx.simulate(db, T=T, precision=precision, write=L.WRITE_ALL, path_dtype=L.F32))
        for k in ("status", "fail_step", "esc_step"):
            assert np.array_equal(r64[k], r32[k]), (precision, k)
        assert np.array_equal(r32["path"], r64["path"].astype(np.float32), equal_nan=True), precision
        if precision == L.FP64:
            assert np.array_equal(r64["status"], ref["status"])
            assert np.array_equal(r64["path"], ref["path"], equal_nan=True)
        else:
            ok = (r64["status"] == ref["status"]) & (r64["fail_step"] == ref["fail_step"])
            assert ok.mean() > 0.97
            sc = _scale(b)[ok]
            err = np.where(np.isnan(ref["path"][ok]), 0.0, np.abs(r64["path"][ok] - ref["path"][ok]))
            assert np.array_equal(np.isnan(r64["path"][ok]), np.isnan(ref["path"][ok]))
            assert np.all(err.max(axis=(1, 2)) <= 1e-5 * sc)
    assert (ref["status"] == 0).sum() > 50


def test_ragged_and_wide_strides(ctx, L):
    _say("[strides]")
    for J, lo, hi in ((7, 4, 7), (13, 6, 13), (32, 20, 32)):
        b = gen.dyad_batch(3000, 77 + J, gen.n_uniform(lo, hi), J=J)
        _fp32_parity(ctx, L, b, label=f"J={J}", in_band_max=IN_BAND_MAX if J <= 20 else 0.20)
        r = _np(ctx.simulate(L.to_device(b), precision=L.FP64))
        ref = oracle.simulate(b, nthreads=NTH)
        assert np.array_equal(r["status"], ref["status"]) and np.array_equal(r["fail_step"], ref["fail_step"])


def test_empty_and_single(ctx, L):
    b = gen.workload("dyad_6_20", 1, seed=1)
    _fp32_parity(ctx, L, b, label="B=1")
    e = gen.workload("dyad_6_20", 1, seed=1).take(np.arange(0))
    r = ctx.simulate(L.to_device(e), write=L.WRITE_VALID, cap=0)
    assert int(r["n_written"].cpu()[0]) == 0


def test_output_joint_choices(ctx, L):
    b = gen.workload("dyad_6_20", 3000, seed=12)
    for out_joint in (0, 1, 2, 5, 19):
        r = _np(ctx.simulate(L.to_device(b), out_joint=out_joint, write=L.WRITE_ALL, precision=L.FP64,
                             path_dtype=L.F64))
        ref = oracle.simulate(b, out_joint=out_joint, path=True, nthreads=NTH)
        same = (r["path"] == ref["path"]) | (np.isnan(r["path"]) & np.isnan(ref["path"]))
        assert same.all(), out_joint


def test_write_valid_compaction(ctx, L):
    _say("[compaction]")
    b = gen.workload("dyad_6_20", 20000, seed=21)
    db = L.to_device(b)
    full = _np(ctx.simulate(db, write=L.WRITE_ALL))
    valid_idx = np.nonzero(full["status"] == 0)[0]
    for cap in (len(valid_idx) + 10, len(valid_idx), 37, 0):
        r = _np(ctx.simulate(db, write=L.WRITE_VALID, cap=cap))
        assert int(r["n_written"][0]) == len(valid_idx)
        k = min(cap, len(valid_idx))
        assert np.array_equal(r["path_index"][:k], valid_idx[:k])
        assert np.array_equal(r["path"][:k], full["path"][valid_idx[:k]])


def test_deterministic_across_tunings(ctx, L):
    _say("[determinism]")
    b = gen.workload("dyad_skewed", 30000, seed=31)
    db = L.to_device(b)
    base = _np(ctx.simulate(db, write=L.WRITE_ALL))
    saved = ctx.get_tuning()
    try:
        for w32, rmin, w64, spread, r64 in ((1, 1, 1, 1, 1), (4, 32, 2, 0, 8), (2, 64, 4, 1, 64), (1, 8, 1, 0, 32)):
            ctx.set_tuning(w32, rmin, w64)
            ctx.set_option("spread", spread)
            ctx.set_option("refill64", r64)
            r = _np(ctx.simulate(db, write=L.WRITE_ALL))
            for k in ("status", "fail_step", "esc_step"):
                assert np.array_equal(r[k], base[k]), (k, w32, rmin, w64, spread, r64)
            assert np.array_equal(np.nan_to_num(r["path"], nan=7.0), np.nan_to_num(base["path"], nan=7.0))
    finally:
        ctx.set_tuning(saved["waves32"], saved["refill_min"], saved["waves64"])
        ctx.set_option("spread", 1)
        ctx.set_option("refill64", 32)
    # a candidate gives the same result alone and in the mix
    for c in (0, 17, 4242):
        one = _np(ctx.simulate(L.to_device(b.take([c])), write=L.WRITE_ALL))
        for k in ("status", "fail_step", "esc_step"):
            assert one[k][0] == base[k][c]
        assert np.array_equal(np.nan_to_num(one["path"][0], nan=7.0), np.nan_to_num(base["path"][c], nan=7.0))


def test_full_size_sampled(ctx, L):
    """The benchmark's workload and launch (1M dyad-built candidates, n ~ U{6..20},
    FP32 with escalation, no path output), checked on a sample the oracle computes."""
    _say("[full size] 1M")
    b = gen.workload("dyad_6_20", 1_000_000, seed=2)
    r = _np(ctx.simulate(L.to_device(b), T=200))
    idx = np.random.default_rng(0).choice(b.B, 40000, replace=False)
    sb = b.take(idx)
    ref = oracle.simulate(sb, T=200, margins=True, nthreads=NTH)
    ib = oracle.in_band(ref["margins"])
    _check_in_band(ib, "1M sample")
    clear = ~ib
    st, fs = r["status"][idx], r["fail_step"][idx]
    assert np.array_equal(st[clear], ref["status"][clear]) and np.array_equal(fs[clear], ref["fail_step"][clear])
    assert abs((r["status"] == 0).mean() - (ref["status"] == 0).mean()) < 0.01
    assert np.all(r["status"] <= 5)


def test_full_size_skewed_sampled(ctx, L):
    """4M candidates with skewed joint counts (60% of 6-8, 30% of 9-14, 10% of
    15-20 joints), FP32 with escalation in the default bucketed launch, checked on
    a sample the oracle computes."""
    _say("[full size] 4M skewed")
    b = gen.workload("dyad_skewed", 4_000_000, seed=3)
    r = _np(ctx.simulate(L.to_device(b), T=200))
    idx = np.random.default_rng(1).choice(b.B, 40000, replace=False)
    sb = b.take(idx)
    ref = oracle.simulate(sb, T=200, margins=True, nthreads=NTH)
    ib = oracle.in_band(ref["margins"])
    _check_in_band(ib, "4M skewed sample")
    clear = ~ib
    st, fs = r["status"][idx], r["fail_step"][idx]
    assert np.array_equal(st[clear], ref["status"][clear]) and np.array_equal(fs[clear], ref["fail_step"][clear])
    assert abs((r["status"] == 0).mean() - (ref["status"] == 0).mean()) < 0.01
    assert np.all(r["status"] <= 5)


def test_normalize_parity(ctx, L):
    """Both sides normalise the same FP32 paths: coordinates within 1e-5 where
    neither side raises a flag; flags agree on almost every path (they are
    threshold decisions); flagged paths agree on the rotation-invariant part
    (centroid, scale, sorted radii)."""
    _say("[normalize]")
    b = gen.workload("dyad_6_20", 20000, seed=41)
    ref = oracle.simulate(b, path=True, nthreads=NTH)
    v = ref["status"] == 0
    paths32 = ref["path"][v].astype(np.float32)
    for mode in (L.NORM_PCA, L.NORM_DIAMETER):
        out, xf = ctx.normalize_paths(torch.from_numpy(paths32).cuda(), mode)
        out, xf = out.cpu().numpy(), xf.cpu().numpy()
        ro, rxf = oracle.normalize_paths(paths32.astype(np.float64), mode)
        fo, fg = rxf[:, 4].astype(int), xf[:, 4].astype(int)
        agree = (fo == fg).mean()
        plain = (fo == 0) & (fg == 0)
        assert plain.sum() > 200 and agree > 0.99, (plain.sum(), agree)
        err = np.abs(out[plain] - ro[plain]).max(axis=(1, 2))
        _say(f"   mode {mode}: {plain.sum()} unflagged paths, flag agreement {agree:.4f}, max error {err.max():.2e}")
        assert np.all(err <= 1e-5)
        flagged = (fo != 0) & (fo == fg) & ((fo & L.NF_CONSTANT) == 0)
        if mode == L.NORM_PCA and flagged.any():
            assert np.allclose(xf[flagged, :3], rxf[flagged, :3], rtol=1e-5, atol=1e-6)
            rg = np.sort(np.hypot(*out[flagged].transpose(2, 0, 1)), axis=1)
            rr = np.sort(np.hypot(*ro[flagged].transpose(2, 0, 1)), axis=1)
            assert np.abs(rg - rr).max() <= 1e-5


def test_normalize_closed_forms(ctx, L):
    t = 2 * np.pi * np.arange(200) / 200
    circle = np.stack([0.3 + 0.1 * np.cos(t), 0.6 + 0.1 * np.sin(t)], -1)
    seg = np.stack([np.linspace(2, 5, 200), np.linspace(1, -3, 200)], -1)
    const = np.ones((200, 2))
    p = torch.from_numpy(np.stack([circle, seg, const]).astype(np.float32)).cuda()
    out, xf = ctx.normalize_paths(p, L.NORM_PCA)
    xf = xf.cpu().numpy()
    assert int(xf[0, 4]) & L.NF_ISOTROPIC and int(xf[2, 4]) == L.NF_CONSTANT
    out, xf = ctx.normalize_paths(p, L.NORM_DIAMETER)
    o = out.cpu().numpy()
    assert np.allclose(o[1, 0], [0, 0.5], atol=1e-6) and np.allclose(o[1, -1], [1, 0.5], atol=1e-6)


@pytest.mark.parametrize("T,P", [(7, 37), (200, 1001), (512, 50), (513, 50), (3000, 9)])
def test_normalize_pca_lengths(ctx, L, T, P):
    """PCA normalisation of random-walk paths of several lengths (the grouped
    kernel up to 512 points, one wave per path above) against the oracle."""
    rng = np.random.default_rng(T)
    steps = rng.normal(size=(P, T, 2)) * rng.uniform(0.01, 1.0, size=(P, 1, 2))
    paths = (np.cumsum(steps, axis=1) + rng.uniform(-5, 5, size=(P, 1, 2))).astype(np.float32)
    out, xf = ctx.normalize_paths(torch.from_numpy(paths).cuda(), L.NORM_PCA)
    out, xf = out.cpu().numpy(), xf.cpu().numpy()
    ro, rxf = oracle.normalize_paths(paths.astype(np.float64), L.NORM_PCA)
    plain = (rxf[:, 4] == 0) & (xf[:, 4] == 0)
    assert plain.mean() > 0.9
    assert np.abs(out[plain] - ro[plain]).max() <= 1e-5
    assert np.allclose(xf[plain, :3], rxf[plain, :3], rtol=1e-5, atol=1e-6)


def test_bad_arguments_raise(ctx, L):
    b = L.to_device(gen.workload("fourbar", 4))
    with pytest.raises(L.LinksError):
        ctx.simulate(b, T=0)
    with pytest.raises(L.LinksError):
        ctx.simulate(b, out_joint=99)
    with pytest.raises(L.LinksError):
        ctx.normalize_paths(torch.zeros((2, 5000, 2), device="cuda"), L.NORM_PCA)


def test_single_precision_positions_give_identical_results(ctx, L):
    """The generator's positions are 24-bit uniforms, exact in FP32, so x0 passed
    as float must give exactly the results of the same numbers passed as double."""
    _say("[x0 f32]")
    b = gen.workload("dyad_6_20", 20000, seed=13)
    assert np.array_equal(b.x0.astype(np.float32).astype(np.float64), b.x0)
    for prec in (L.FP32_RECHECK, L.FP64):
        r64 = _np(ctx.simulate(L.to_device(b), precision=prec, write=L.WRITE_ALL))
        r32 = _np(ctx.simulate(L.to_device(b, x0_dtype=np.float32), precision=prec, write=L.WRITE_ALL))
        for k in ("status", "fail_step", "esc_step"):
            assert np.array_equal(r64[k], r32[k]), (prec, k)
        assert np.array_equal(np.nan_to_num(r64["path"], nan=7.0), np.nan_to_num(r32["path"], nan=7.0))


@pytest.mark.parametrize("precision", [0, 1])
def test_low_fidelity_prefilter(ctx, L, precision):
    """T_prefilter = 50 (the paper's low-fidelity screen) against the oracle's
    composition of a 50-position and a 200-position run: bit-exact for FP64, and
    outside the bands for FP32 with escalation; valid paths are the full run's."""
    _say(f"[prefilter] precision={precision}")
    b = gen.workload("dyad_6_20", 20000, seed=14)
    r = _np(ctx.simulate(L.to_device(b), T=200, precision=precision, T_prefilter=50, write=L.WRITE_VALID,
                         cap=20000))
    ref = oracle.simulate_prefiltered(b, T=200, T_low=50, margins=True, nthreads=NTH)
    if precision == L.FP64:
        assert np.array_equal(r["status"], ref["status"]) and np.array_equal(r["fail_step"], ref["fail_step"])
    else:
        ib = oracle.in_band(ref["margins"])
        _check_in_band(ib, "prefilter")
        clear = ~ib
        assert np.array_equal(r["status"][clear], ref["status"][clear])
        assert np.array_equal(r["fail_step"][clear], ref["fail_step"][clear])
    k = int(r["n_written"][0])
    assert k == int((r["status"] == 0).sum())
    full = oracle.simulate(b.take(r["path_index"][:k]), T=200, path=True, nthreads=NTH)
    tol = 1e-5 * mech.scale_of(b.take(r["path_index"][:k]))
    ok = full["status"] == 0          # in-band candidates may differ; they are excluded above
    assert ok.mean() > 0.99
    err = np.abs(r["path"][:k][ok] - full["path"][ok]).max(axis=(1, 2))
    assert np.all(err <= tol[ok])


def test_prefilter_argument_checks(ctx, L):
    db = L.to_device(gen.workload("dyad_6_20", 100, seed=15))
    for tp in (200, 33, -1):
        with pytest.raises(L.LinksError):
            ctx.simulate(db, T=200, T_prefilter=tp)


def test_curation_parity(ctx, L):
    """links_curate against the oracle's curation of the same DIAMETER-normalised
    paths: arc flags and reduced-mechanism masks bit-exact, radial variances to
    float rounding, circle flags exact away from the threshold."""
    _say("[curate]")
    b = gen.Batch.concat([gen.workload("dyad_6_20", 20000, seed=16), gen.workload("fourbar", 2000, seed=17)])
    db = L.to_device(b)
    r = ctx.simulate(db, write=L.WRITE_VALID, cap=b.B)
    k = int(r["n_written"].cpu()[0])
    norm, _ = ctx.normalize_paths(r["path"][:k].contiguous(), L.NORM_DIAMETER)
    cu = ctx.curate(db, norm, path_index=r["path_index"][:k], count=r["n_written"])
    got = {key: v.cpu().numpy() for key, v in cu.items()}
    idx = r["path_index"][:k].cpu().numpy()
    ref = oracle.curate(b, norm.cpu().numpy().astype(np.float64), cand=idx)
    assert k > 2000
    assert np.array_equal(got["keep"].view(np.uint32), ref["keep"])
    assert np.array_equal(got["flags"] & 1, ref["flags"] & 1)
    far = np.abs(ref["radial_var"] - oracle.CIRCLE_VAR) > 1e-9
    assert np.array_equal(got["flags"][far] & 2, ref["flags"][far] & 2)
    assert np.allclose(got["radial_var"], ref["radial_var"], rtol=1e-6, atol=1e-12)
    arcs, circles = (ref["flags"] & 1).mean(), ((ref["flags"] & 2) != 0).mean()
    _say(f"   {k} paths: arcs {arcs:.3f}, circles {circles:.3f}")
    # the crank tip of a four-bar: an arc and a circle
    fb = gen.workload("fourbar", 500, seed=18)
    dfb = L.to_device(fb)
    rr = ctx.simulate(dfb, out_joint=1, write=L.WRITE_ALL)
    nf, _ = ctx.normalize_paths(rr["path"], L.NORM_DIAMETER)
    cf = ctx.curate(dfb, nf, out_joint=1)
    assert np.all(cf["flags"].cpu().numpy() == 3)
    assert np.all(cf["keep"].cpu().numpy() == 3)


@pytest.mark.parametrize("deesc", [1, 4, 8])
def test_return_to_fp32_after_handover(ctx, L, deesc):
    """The same bar whatever the number of FP64 steps before a handed-over
    candidate returns to FP32 (0: never returns)."""
    _say(f"[deesc] {deesc}")
    b = gen.workload("dyad_6_20", 20000, seed=19)
    ctx.set_option("deesc", deesc)
    try:
        _fp32_parity(ctx, L, b, label=f"deesc={deesc}")
    finally:
        ctx.set_option("deesc", 0)
