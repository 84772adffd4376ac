"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never calls into it, and it shares no
code with the HIP path (its own C sources, its own header, its own build line).

The C code lives in ``links_ref.c``; this module builds it with gcc
(``-O2 -ffp-contract=off``, no fast-math) into ``liblinks_ref.so`` and wraps it
for numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "links_ref.c")
LIB = os.path.join(HERE, "liblinks_ref.so")

VALID, LOCKED, DEGENERATE, DRIFT, UNSOLVABLE, BAD_MECH = range(6)
BRANCH_CONTINUITY, BRANCH_ORIENTATION = 0, 1
NORM_PCA, NORM_DIAMETER = 0, 1
NF_CONSTANT, NF_ISOTROPIC, NF_SIGN_TIE, NF_DIAM_TIE = 1, 2, 4, 8

# band widths used to call a candidate's decisions robust (see margins())
EPS_DISC = 1e-6
EPS_BRANCH = 1e-5
TAU_DRIFT = 1e-4

_lib = None

# every operation as written: no fused multiply-adds, no fast-math, and cos / sin
# called as such (not merged into one sincos call by the compiler)
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fno-builtin-sin", "-fno-builtin-cos",
          "-fno-builtin-sincos", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle library with gcc (always, when ``force``)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-Wall", "-o", tmp, SRC, "-lm", "-lpthread"])
        os.replace(tmp, LIB)
    return LIB


def build_variant(src_text: str, out_path: str) -> str:
    """Compile a modified copy of the oracle source (used to plant mistakes in tests)."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", *CFLAGS, "-I", HERE, "-o", out_path, src, "-lm", "-lpthread"])
    return out_path


def use_library(path: Optional[str]):
    """Point the wrappers at another build of the oracle (None: the default one).
    Returns the previously loaded handle's path."""
    global _lib, _lib_path
    prev = _lib_path
    _lib = None
    _lib_path = path
    return prev


_lib_path: Optional[str] = None


def lib():
    global _lib
    if _lib is None:
        path = _lib_path or LIB
        if path == LIB and not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32 = ctypes.c_int32
        L.links_ref_solve_order.argtypes = [i32, i32, P, P, P, P, P, P, P, P]
        L.links_ref_solve_order.restype = ctypes.c_int
        L.links_ref_simulate.argtypes = [i32, i32, P, P, P, P, P, i32, i32, ctypes.c_double, P, P, P, P, P, i32]
        L.links_ref_simulate.restype = ctypes.c_int
        L.links_ref_simulate_branch.argtypes = [i32, i32, P, P, P, P, P, i32, i32, ctypes.c_double, P, P, P, P, P,
                                                i32, i32]
        L.links_ref_simulate_branch.restype = ctypes.c_int
        L.links_ref_normalize_paths.argtypes = [P, i32, i32, i32, P, P]
        L.links_ref_normalize_paths.restype = ctypes.c_int
        L.links_ref_curate.argtypes = [i32, P, P, P, P, i32, P, i32, P, i32, ctypes.c_double, P, P, P]
        L.links_ref_curate.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def solve_order(batch):
    """Returns (order int8[B,J,3], n_dyads u8[B], depth u8[B], status u8[B])."""
    B, J = batch.B, batch.J
    order = np.empty((B, J, 3), np.int8)
    nd = np.empty(B, np.uint8)
    dp = np.empty(B, np.uint8)
    st = np.empty(B, np.uint8)
    n, adj, fx, mo = _c(batch.n, np.uint8), _c(batch.adj, np.uint32), _c(batch.fixed, np.uint32), _c(batch.motor, np.uint8)
    rc = lib().links_ref_solve_order(B, J, _p(n), _p(adj), _p(fx), _p(mo), _p(order), _p(nd), _p(dp), _p(st))
    if rc != 0:
        raise ValueError("links_ref_solve_order: bad argument")
    return order, nd, dp, st


def simulate(batch, T: int = 200, out_joint: int = -1, tau_drift: float = TAU_DRIFT, path: bool = False,
             pos_all: bool = False, margins: bool = False, nthreads: int = 1, x0=None,
             branch: int = BRANCH_CONTINUITY):
    """FP64 full-rotation simulation.  Returns a dict with status, fail_step and the
    optional path [B,T,2], pos_all [B,T,J,2] and margins [B,4].  branch selects the
    rule for the side of each placed joint (continuity or starting orientation)."""
    B, J = batch.B, batch.J
    st = np.empty(B, np.uint8)
    fs = np.empty(B, np.int16)
    pa = np.empty((B, T, 2), np.float64) if path else None
    al = np.empty((B, T, J, 2), np.float64) if pos_all else None
    mg = np.empty((B, 4), np.float64) if margins else None
    n, adj, fx, mo = _c(batch.n, np.uint8), _c(batch.adj, np.uint32), _c(batch.fixed, np.uint32), _c(batch.motor, np.uint8)
    xx = _c(batch.x0 if x0 is None else x0, np.float64)
    rc = lib().links_ref_simulate_branch(B, J, _p(n), _p(adj), _p(fx), _p(mo), _p(xx), T, out_joint, tau_drift,
                                         _p(st), _p(fs), _p(pa), _p(al), _p(mg), nthreads, branch)
    if rc != 0:
        raise ValueError("links_ref_simulate: bad argument")
    return {"status": st, "fail_step": fs, "path": pa, "pos_all": al, "margins": mg}


def simulate_prefiltered(batch, T: int = 200, T_low: int = 50, nthreads: int = 1, margins: bool = False):
    """The low-fidelity screen of "Scale of Infeasibilities": every candidate is
    simulated at T_low equally spaced actuator positions; those that lock there
    are rejected (their failure kept, at the same angle on the T grid), and only
    the survivors are simulated at T positions.  Returns status, fail_step and,
    with margins, the margins of the run that decided each candidate."""
    if T % T_low != 0 or not 0 < T_low < T:
        raise ValueError("T_low must divide T and be smaller")
    low = simulate(batch, T=T_low, nthreads=nthreads, margins=margins)
    keep = np.nonzero(low["status"] == VALID)[0]
    st = low["status"].copy()
    fs = np.where(low["fail_step"] >= 0, low["fail_step"].astype(np.int32) * (T // T_low), -1).astype(np.int16)
    mg = low["margins"].copy() if margins else None
    if keep.size:
        hi = simulate(batch.take(keep), T=T, nthreads=nthreads, margins=margins)
        st[keep] = hi["status"]
        fs[keep] = hi["fail_step"]
        if margins:
            mg[keep] = np.minimum(mg[keep], hi["margins"])
    return {"status": st, "fail_step": fs, "margins": mg}


ARC, CIRCLE = 1, 2
CIRCLE_VAR = 5e-4


def curate(batch, norm_paths: np.ndarray, cand=None, out_joint: int = -1, circle_var: float = CIRCLE_VAR):
    """Arc and circle flags, radial variances and reduced-mechanism joint masks of
    DIAMETER-normalised paths [P,T,2]; path i belongs to candidate cand[i]."""
    p = _c(norm_paths, np.float64)
    P, T = p.shape[0], p.shape[1]
    cd = None if cand is None else _c(cand, np.int32)
    fl = np.empty(P, np.uint8)
    rv = np.empty(P, np.float64)
    kp = np.empty(P, np.uint32)
    n, adj, fx, mo = _c(batch.n, np.uint8), _c(batch.adj, np.uint32), _c(batch.fixed, np.uint32), _c(batch.motor, np.uint8)
    rc = lib().links_ref_curate(batch.J, _p(n), _p(adj), _p(fx), _p(mo), out_joint, _p(cd), P, _p(p), T,
                                circle_var, _p(fl), _p(rv), _p(kp))
    if rc != 0:
        raise ValueError("links_ref_curate: bad argument")
    return {"flags": fl, "radial_var": rv, "keep": kp}


def in_band(margins: np.ndarray, eps_disc: float = EPS_DISC, eps_branch: float = EPS_BRANCH,
            tau_drift: float = TAU_DRIFT) -> np.ndarray:
    """True where some evaluated decision of the candidate lies within the stated
    band of its threshold, so that a correctly rounded lower-precision path may
    decide it either way."""
    m = margins
    return (m[:, 0] < eps_disc) | (m[:, 1] < eps_disc) | (m[:, 2] < eps_branch) | (m[:, 3] < 0.9 * tau_drift)


def normalize_paths(paths: np.ndarray, mode: int = NORM_PCA):
    """Returns (out [P,T,2], xform [P,5])."""
    p = _c(paths, np.float64)
    P, T = p.shape[0], p.shape[1]
    out = np.empty_like(p)
    xf = np.empty((P, 5), np.float64)
    rc = lib().links_ref_normalize_paths(_p(p), P, T, mode, _p(out), _p(xf))
    if rc != 0:
        raise ValueError("links_ref_normalize_paths: bad argument")
    return out, xf
