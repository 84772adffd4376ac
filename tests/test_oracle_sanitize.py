"""The FP64 oracle under sanitizers (CPU only).

The oracle is multithreaded C with fixed-size stack arrays.  It is built twice
more, once with AddressSanitizer + UndefinedBehaviorSanitizer and once with
ThreadSanitizer (both halting at the first report), and every entry point is run
through a small driver on fixtures, malformed candidates and a dyad-built batch
with several threads and both branch rules.  The run must be clean and its
outputs must equal those of the ordinary build bit for bit.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2208_14567_amd import gen
from tests import mech

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "oracle_sanitize_driver.c")
ORACLE_DIR = os.path.dirname(oracle.__file__)
T = 200

SANITIZERS = {
    "address_undefined": (["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"],
                          {"ASAN_OPTIONS": "halt_on_error=1:detect_leaks=1:abort_on_error=0",
                           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}),
    "thread": (["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1"}),
}


def _inputs():
    b = gen.workload("dyad_4_20", 2000, seed=101)
    broken, _ = mech.malform(gen.dyad_batch(400, 102, gen.n_uniform(4, 20), J=20), seed=103)
    fb = gen.workload("fourbar_u", 300, seed=104)
    fb20 = gen.Batch(fb.n, np.zeros((fb.B, 20), np.uint32), fb.fixed, fb.motor, np.zeros((fb.B, 20, 2)))
    fb20.adj[:, :fb.J] = fb.adj
    fb20.x0[:, :fb.J] = fb.x0
    return gen.Batch.concat([b, broken, fb20])


def _build(kind, out):
    flags, _ = SANITIZERS[kind]
    cmd = ["gcc", "-O1", "-g", "-ffp-contract=off", "-fno-fast-math", "-fno-builtin-sin", "-fno-builtin-cos",
           "-fno-builtin-sincos", *flags, "-I", ORACLE_DIR, "-o", out, DRIVER, os.path.join(ORACLE_DIR, "links_ref.c"),
           "-lm", "-lpthread"]
    subprocess.check_call(cmd)


def _read(d, name, dtype, shape):
    return np.fromfile(os.path.join(d, name + ".bin"), dtype=dtype).reshape(shape)


@pytest.mark.parametrize("kind", sorted(SANITIZERS))
def test_oracle_is_clean_under_sanitizer(kind, tmp_path, oracle_lib):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    b = _inputs()
    B, J = b.B, b.J
    d = str(tmp_path)
    for name, arr, dt in (("n", b.n, np.uint8), ("adj", b.adj, np.uint32), ("fixed", b.fixed, np.uint32),
                          ("motor", b.motor, np.uint8), ("x0", b.x0, np.float64)):
        np.ascontiguousarray(arr, dt).tofile(os.path.join(d, name + ".bin"))
    exe = os.path.join(d, f"driver_{kind}")
    _build(kind, exe)
    env = dict(os.environ)
    env.update(SANITIZERS[kind][1])
    r = subprocess.run([exe, d, str(B), str(J), str(T), "6"], env=env, capture_output=True, text=True, timeout=600)
    report = (r.stderr or "")[-4000:]
    assert r.returncode == 0, f"{kind} run failed (rc {r.returncode}):\n{report}"
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, report

    # the ordinary build gives the same results, bit for bit
    ref = oracle.simulate(b, T=T, path=True, pos_all=True, margins=True, nthreads=3)
    assert np.array_equal(_read(d, "status", np.uint8, B), ref["status"])
    assert np.array_equal(_read(d, "fail", np.int16, B), ref["fail_step"])
    assert np.array_equal(_read(d, "path", np.float64, (B, T, 2)), ref["path"], equal_nan=True)
    assert np.array_equal(_read(d, "pos_all", np.float64, (B, T, J, 2)), ref["pos_all"], equal_nan=True)
    assert np.array_equal(_read(d, "margins", np.float64, (B, 4)), ref["margins"], equal_nan=True)
    ro = oracle.simulate(b, T=T, nthreads=2, branch=oracle.BRANCH_ORIENTATION)
    assert np.array_equal(_read(d, "status_o", np.uint8, B), ro["status"])
    assert np.array_equal(_read(d, "fail_o", np.int16, B), ro["fail_step"])
    order, nd, dp, so = oracle.solve_order(b)
    assert np.array_equal(_read(d, "order", np.int8, (B, J, 3)), order)
    assert np.array_equal(_read(d, "n_dyads", np.uint8, B), nd)
    assert np.array_equal(_read(d, "depth", np.uint8, B), dp)
    assert np.array_equal(_read(d, "st_order", np.uint8, B), so)
    for mode, tag in ((oracle.NORM_PCA, "pca"), (oracle.NORM_DIAMETER, "diam")):
        no, xf = oracle.normalize_paths(ref["path"], mode)
        assert np.array_equal(_read(d, f"norm_{tag}", np.float64, (B, T, 2)), no, equal_nan=True)
        assert np.array_equal(_read(d, f"xf_{tag}", np.float64, (B, 5)), xf, equal_nan=True)
    cu = oracle.curate(b, no)
    assert np.array_equal(_read(d, "cur_flags", np.uint8, B), cu["flags"])
    assert np.array_equal(_read(d, "cur_var", np.float64, B), cu["radial_var"], equal_nan=True)
    assert np.array_equal(_read(d, "cur_keep", np.uint32, B), cu["keep"])
    # the batch exercises every outcome
    assert set(np.unique(ref["status"])) >= {oracle.VALID, oracle.LOCKED, oracle.BAD_MECH}
