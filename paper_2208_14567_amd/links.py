"""Python binding of liblinks.so (argument marshalling only).

Every step of the simulation runs in the HIP library; this module only moves
torch device tensors' pointers and the current HIP stream across the C ABI of
``include/links.h``.  It raises if the library is not built -- there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblinks.so")

OK, ERR_ARG, ERR_DEVICE, ERR_OOM = 0, -1, -2, -3
VALID, LOCKED, DEGENERATE, DRIFT, UNSOLVABLE, BAD_MECH = range(6)
FP32_RECHECK, FP64, FP32_ONLY = 0, 1, 2
BRANCH_CONTINUITY, BRANCH_ORIENTATION = 0, 1
WRITE_NONE, WRITE_ALL, WRITE_VALID = 0, 1, 2
F32, F64 = 0, 1
NORM_PCA, NORM_DIAMETER = 0, 1
NF_CONSTANT, NF_ISOTROPIC, NF_SIGN_TIE, NF_DIAM_TIE = 1, 2, 4, 8
CURATE_ARC, CURATE_CIRCLE = 1, 2
SEARCH_FIRST, SEARCH_BEST = 0, 1

P = ctypes.c_void_p
i32 = ctypes.c_int32


# links_piece of include/links.h
PIECE_DTYPE = np.dtype([("src", np.int64), ("dst", np.int32), ("first", np.int32), ("size", np.int32),
                        ("J", np.int32)], align=True)


class Batch(ctypes.Structure):
    _fields_ = [("B", i32), ("J", i32), ("n", P), ("adj", P), ("fixed", P), ("motor", P), ("x0", P),
                ("x0_f32", P)]


class SimOpts(ctypes.Structure):
    _fields_ = [("T", i32), ("precision", i32), ("eps_disc", ctypes.c_double), ("eps_branch", ctypes.c_double),
                ("tau_drift", ctypes.c_double), ("out_joint", i32), ("write", i32), ("path_dtype", i32),
                ("T_prefilter", i32), ("branch", i32)]


class SimOut(ctypes.Structure):
    _fields_ = [("status", P), ("fail_step", P), ("esc_step", P), ("path", P), ("path_index", P),
                ("n_written", P), ("cap", i32)]


EXPORTS = ["links_create", "links_destroy", "links_last_error", "links_version", "links_solve_order",
           "links_sim_opts_default", "links_simulate", "links_normalize_paths", "links_set_tuning",
           "links_get_tuning", "links_set_option", "links_normalize_paths_n", "links_profile", "links_last_timings",
           "links_mean_timings", "links_simulate_noalloc",
           "links_graph_create", "links_graph_launch", "links_graph_destroy", "links_get_option",
           "links_generate_dyads", "links_curate", "links_gather"]
TIMING_PASSES = ["prep_count", "prep_fill", "fp32_pass", "fp64_pass", "compaction", "path_pass"]

_lib = None


def load() -> ctypes.CDLL:
    """Loads liblinks.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                           "python -m paper_2208_14567_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    L.links_create.argtypes = [ctypes.c_int, ctypes.POINTER(P)]
    L.links_create.restype = ctypes.c_int
    L.links_destroy.argtypes = [P]
    L.links_destroy.restype = None
    L.links_last_error.argtypes = []
    L.links_last_error.restype = ctypes.c_char_p
    L.links_version.argtypes = []
    L.links_version.restype = ctypes.c_char_p
    L.links_solve_order.argtypes = [P, ctypes.POINTER(Batch), P, P, P, P, P]
    L.links_solve_order.restype = ctypes.c_int
    L.links_sim_opts_default.argtypes = [ctypes.POINTER(SimOpts)]
    L.links_sim_opts_default.restype = None
    L.links_simulate.argtypes = [P, ctypes.POINTER(Batch), ctypes.POINTER(SimOpts), ctypes.POINTER(SimOut), P]
    L.links_simulate.restype = ctypes.c_int
    L.links_normalize_paths.argtypes = [P, P, i32, i32, i32, P, P, P]
    L.links_normalize_paths.restype = ctypes.c_int
    L.links_set_tuning.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.links_set_tuning.restype = ctypes.c_int
    L.links_get_tuning.argtypes = [P] + [ctypes.POINTER(ctypes.c_int)] * 5
    L.links_get_tuning.restype = ctypes.c_int
    L.links_set_option.argtypes = [P, ctypes.c_char_p, ctypes.c_int]
    L.links_set_option.restype = ctypes.c_int
    L.links_get_option.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)]
    L.links_get_option.restype = ctypes.c_int
    L.links_normalize_paths_n.argtypes = [P, P, P, i32, i32, i32, P, P, P]
    L.links_normalize_paths_n.restype = ctypes.c_int
    L.links_chamfer.argtypes = [P, P, i32, i32, P, i32, P, P]
    L.links_chamfer.restype = ctypes.c_int
    L.links_chamfer_search.argtypes = [P, P, i32, i32, P, i32, i32, ctypes.c_float, i32, P, P, P]
    L.links_chamfer_search.restype = ctypes.c_int
    L.links_profile.argtypes = [P, ctypes.c_int]
    L.links_profile.restype = ctypes.c_int
    L.links_last_timings.argtypes = [P, ctypes.POINTER(ctypes.c_float), ctypes.c_int]
    L.links_last_timings.restype = ctypes.c_int
    L.links_simulate_noalloc.argtypes = L.links_simulate.argtypes
    L.links_simulate_noalloc.restype = ctypes.c_int
    L.links_mean_timings.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_float), ctypes.c_int]
    L.links_mean_timings.restype = ctypes.c_int
    L.links_generate_dyads.argtypes = [P, ctypes.c_uint64, ctypes.c_int64, i32, i32, i32, i32, i32, P, P, P, P, P, P]
    L.links_generate_dyads.restype = ctypes.c_int
    L.links_curate.argtypes = [P, ctypes.POINTER(Batch), P, P, i32, i32, P, i32, ctypes.c_double, P, P, P, P]
    L.links_curate.restype = ctypes.c_int
    L.links_graph_create.argtypes = [P, ctypes.POINTER(Batch), ctypes.POINTER(SimOpts), ctypes.POINTER(SimOut),
                                     ctypes.POINTER(P)]
    L.links_graph_create.restype = ctypes.c_int
    L.links_graph_launch.argtypes = [P, P]
    L.links_graph_launch.restype = ctypes.c_int
    L.links_graph_destroy.argtypes = [P]
    L.links_graph_destroy.restype = None
    L.links_gather.argtypes = [P, P, P, i32, i32, ctypes.POINTER(Batch), P]
    L.links_gather.restype = ctypes.c_int
    _lib = L
    return L


class LinksError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != OK:
        msg = load().links_last_error().decode(errors="replace")
        raise LinksError(f"{what} failed ({rc}): {msg}")


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _paths_arg(t: torch.Tensor, name: str) -> torch.Tensor:
    if t.dtype != torch.float32 or t.dim() != 3 or t.shape[2] != 2:
        raise ValueError(f"{name} must be a float32 [n, T, 2] tensor")
    return t


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


@dataclass
class DeviceBatch:
    """Device copies of a batch (layout of include/links.h)."""
    n: torch.Tensor
    adj: torch.Tensor
    fixed: torch.Tensor
    motor: torch.Tensor
    x0: torch.Tensor

    @property
    def B(self) -> int:
        return int(self.n.shape[0])

    @property
    def J(self) -> int:
        return int(self.adj.shape[1]) if self.adj.dim() == 2 else 1

    def cstruct(self) -> Batch:
        f32 = self.x0.dtype == torch.float32
        return Batch(self.B, self.J, _ptr(self.n), _ptr(self.adj), _ptr(self.fixed), _ptr(self.motor),
                     None if f32 else _ptr(self.x0), _ptr(self.x0) if f32 else None)

    def slice(self, lo: int, hi: int) -> "DeviceBatch":
        return DeviceBatch(self.n[lo:hi], self.adj[lo:hi], self.fixed[lo:hi], self.motor[lo:hi], self.x0[lo:hi])


def to_device(batch, device="cuda", non_blocking=False, x0_dtype=np.float64) -> DeviceBatch:
    """Copies a host batch (paper_2208_14567_amd.gen.Batch) to the device; x0 in
    double (default) or single precision (np.float32)."""
    def t(a, dtype):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to(device, non_blocking=non_blocking)
    return DeviceBatch(t(batch.n, np.uint8), t(batch.adj.view(np.int32), np.int32), t(batch.fixed.view(np.int32), np.int32),
                       t(batch.motor, np.uint8), t(batch.x0, x0_dtype))


class Context:
    """A library context bound to one HIP device."""

    def __init__(self, device: int = 0):
        L = load()
        h = P()
        _check(L.links_create(device, ctypes.byref(h)), "links_create")
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            load().links_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tuning(self, waves32: int, refill_min: int, waves64: int):
        _check(load().links_set_tuning(self._h, waves32, refill_min, waves64), "links_set_tuning")

    def set_option(self, name: str, value: int):
        _check(load().links_set_option(self._h, name.encode(), int(value)), "links_set_option")

    def get_option(self, name: str) -> int:
        v = ctypes.c_int()
        _check(load().links_get_option(self._h, name.encode(), ctypes.byref(v)), "links_get_option")
        return v.value

    def get_tuning(self) -> dict:
        v = [ctypes.c_int() for _ in range(5)]
        _check(load().links_get_tuning(self._h, *[ctypes.byref(x) for x in v]), "links_get_tuning")
        return dict(zip(["waves32", "refill_min", "waves64", "grid32", "grid64"], [x.value for x in v]))

    def profile(self, enable: bool = True):
        _check(load().links_profile(self._h, 1 if enable else 0), "links_profile")

    def last_timings(self) -> dict:
        """Milliseconds of each pass of the last profiled simulate call."""
        n = len(TIMING_PASSES)
        buf = (ctypes.c_float * n)()
        k = load().links_last_timings(self._h, buf, n)
        if k < 0:
            _check(k, "links_last_timings")
        return {name: float(buf[i]) for i, name in enumerate(TIMING_PASSES[:k])}

    def mean_timings(self, calls: int) -> dict:
        """Mean milliseconds of each pass over the last `calls` profiled simulate calls."""
        n = len(TIMING_PASSES)
        buf = (ctypes.c_float * n)()
        k = load().links_mean_timings(self._h, calls, buf, n)
        if k < 0:
            _check(k, "links_mean_timings")
        return {name: float(buf[i]) for i, name in enumerate(TIMING_PASSES[:k])}

    # ------------------------------------------------------------------ solve order
    def solve_order(self, b: DeviceBatch, stream=None):
        dev = b.n.device
        order = torch.empty((b.B, b.J, 3), dtype=torch.int8, device=dev)
        nd = torch.empty(b.B, dtype=torch.uint8, device=dev)
        dp = torch.empty(b.B, dtype=torch.uint8, device=dev)
        st = torch.empty(b.B, dtype=torch.uint8, device=dev)
        cb = b.cstruct()
        _check(load().links_solve_order(self._h, ctypes.byref(cb), _ptr(order), _ptr(nd), _ptr(dp), _ptr(st),
                                        _stream(stream)), "links_solve_order")
        return order, nd, dp, st

    # ------------------------------------------------------------------ simulation
    def _sim_args(self, b: DeviceBatch, T, precision, write, out_joint, path_dtype, cap, eps_disc, eps_branch,
                  tau_drift, out, T_prefilter=0, branch=BRANCH_CONTINUITY):
        dev = b.n.device
        B = b.B
        o = out or {}
        status = o.get("status") if o.get("status") is not None else torch.empty(B, dtype=torch.uint8, device=dev)
        fail = o.get("fail_step") if o.get("fail_step") is not None else torch.empty(B, dtype=torch.int16, device=dev)
        esc = o.get("esc_step") if o.get("esc_step") is not None else torch.empty(B, dtype=torch.int16, device=dev)
        pdt = torch.float64 if path_dtype == F64 else torch.float32
        path = idx = nw = None
        cap_v = 0
        if write == WRITE_ALL:
            path = o.get("path") if o.get("path") is not None else torch.empty((B, T, 2), dtype=pdt, device=dev)
        elif write == WRITE_VALID:
            cap_v = B if cap is None else int(cap)
            path = o.get("path") if o.get("path") is not None else torch.empty((max(cap_v, 1), T, 2), dtype=pdt, device=dev)
            idx = o.get("path_index") if o.get("path_index") is not None else torch.empty(max(cap_v, 1), dtype=torch.int32, device=dev)
            nw = o.get("n_written") if o.get("n_written") is not None else torch.empty(1, dtype=torch.int32, device=dev)
        opts = SimOpts(T, precision, eps_disc, eps_branch, tau_drift, out_joint, write, path_dtype, T_prefilter,
                       branch)
        so = SimOut(_ptr(status), _ptr(fail), _ptr(esc), _ptr(path), _ptr(idx), _ptr(nw), cap_v)
        res = {"status": status, "fail_step": fail, "esc_step": esc}
        if path is not None:
            res["path"] = path
        if idx is not None:
            res["path_index"] = idx
            res["n_written"] = nw
        return b.cstruct(), opts, so, res

    def simulate(self, b: DeviceBatch, T: int = 200, precision: int = FP32_RECHECK, write: int = WRITE_NONE,
                 out_joint: int = -1, path_dtype: int = F32, cap: Optional[int] = None, eps_disc: float = 1e-6,
                 eps_branch: float = 1e-5, tau_drift: float = 1e-4, out: Optional[dict] = None, stream=None,
                 T_prefilter: int = 0, branch: int = BRANCH_CONTINUITY):
        """Returns a dict of device tensors: status, fail_step, esc_step and, by write
        mode, path ([B,T,2] or [cap,T,2]), path_index and n_written.  T_prefilter > 0
        runs the low-fidelity check at that many positions first; branch selects the
        side rule (continuity or starting orientation)."""
        cb, opts, so, res = self._sim_args(b, T, precision, write, out_joint, path_dtype, cap, eps_disc, eps_branch,
                                           tau_drift, out, T_prefilter, branch)
        _check(load().links_simulate(self._h, ctypes.byref(cb), ctypes.byref(opts), ctypes.byref(so), _stream(stream)),
               "links_simulate")
        return res

    def simulate_noalloc(self, b: DeviceBatch, T: int = 200, precision: int = FP32_RECHECK, write: int = WRITE_NONE,
                         out_joint: int = -1, path_dtype: int = F32, cap: Optional[int] = None,
                         eps_disc: float = 1e-6, eps_branch: float = 1e-5, tau_drift: float = 1e-4,
                         out: Optional[dict] = None, stream=None, T_prefilter: int = 0,
                         branch: int = BRANCH_CONTINUITY):
        """``simulate`` through links_simulate_noalloc: the library's workspace is the
        device's fixed scratch array (the output tensors are still the caller's;
        pass ``out`` to allocate nothing here either)."""
        cb, opts, so, res = self._sim_args(b, T, precision, write, out_joint, path_dtype, cap, eps_disc, eps_branch,
                                           tau_drift, out, T_prefilter, branch)
        _check(load().links_simulate_noalloc(self._h, ctypes.byref(cb), ctypes.byref(opts), ctypes.byref(so),
                                             _stream(stream)), "links_simulate_noalloc")
        return res

    def generate_dyads(self, B: int, seed: int, first: int = 0, J: int = 20, n_lo: int = 6, n_hi: int = 20,
                       paper_mode: bool = False, device=None, out: Optional[DeviceBatch] = None,
                       stream=None, rules: bool = False) -> DeviceBatch:
        """Generates candidates first .. first+B-1 of the seed's sequence on the
        device (the same candidates as gen.dyad_batch with n ~ U{n_lo..n_hi}, the
        same paper_mode and rules)."""
        dev = torch.device("cuda", self.device) if device is None else device
        if out is None:
            out = DeviceBatch(torch.empty(B, dtype=torch.uint8, device=dev),
                              torch.empty((B, J), dtype=torch.int32, device=dev),
                              torch.empty(B, dtype=torch.int32, device=dev),
                              torch.empty((B, 2), dtype=torch.uint8, device=dev),
                              torch.empty((B, J, 2), dtype=torch.float64, device=dev))
        _check(load().links_generate_dyads(self._h, seed & 0xFFFFFFFFFFFFFFFF, first, B, J, n_lo, n_hi,
                                           (1 if paper_mode else 0) | (2 if rules else 0), _ptr(out.n), _ptr(out.adj), _ptr(out.fixed),
                                           _ptr(out.motor), _ptr(out.x0), _stream(stream)), "links_generate_dyads")
        return out

    def curate(self, b: DeviceBatch, norm_paths: torch.Tensor, path_index: Optional[torch.Tensor] = None,
               count: Optional[torch.Tensor] = None, out_joint: int = -1, circle_var: float = 5e-4,
               stream=None) -> dict:
        """Arc / circle flags, radial variances and reduced-mechanism joint masks of
        DIAMETER-normalised paths (links_curate)."""
        cap, T = int(norm_paths.shape[0]), int(norm_paths.shape[1])
        dev = norm_paths.device
        flags = torch.empty(max(cap, 1), dtype=torch.uint8, device=dev)
        rv = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
        keep = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        cb = b.cstruct()
        _check(load().links_curate(self._h, ctypes.byref(cb), _ptr(path_index), _ptr(count), cap, out_joint,
                                   _ptr(norm_paths), T, circle_var, _ptr(flags), _ptr(rv), _ptr(keep),
                                   _stream(stream)), "links_curate")
        return {"flags": flags[:cap], "radial_var": rv[:cap], "keep": keep[:cap]}

    def graph(self, b: DeviceBatch, T: int = 200, precision: int = FP32_RECHECK, write: int = WRITE_NONE,
              out_joint: int = -1, path_dtype: int = F32, cap: Optional[int] = None, eps_disc: float = 1e-6,
              eps_branch: float = 1e-5, tau_drift: float = 1e-4, out: Optional[dict] = None,
              T_prefilter: int = 0, branch: int = BRANCH_CONTINUITY) -> "Graph":
        """Records the launch sequence of ``simulate`` with these arguments into a HIP
        graph; ``Graph.launch`` replays it on the current stream.  The returned
        graph holds the batch and output tensors (``Graph.out``)."""
        cb, opts, so, res = self._sim_args(b, T, precision, write, out_joint, path_dtype, cap, eps_disc, eps_branch,
                                           tau_drift, out, T_prefilter, branch)
        g = P()
        _check(load().links_graph_create(self._h, ctypes.byref(cb), ctypes.byref(opts), ctypes.byref(so),
                                         ctypes.byref(g)), "links_graph_create")
        return Graph(g, self, b, res)

    def gather(self, buf: torch.Tensor, pieces: torch.Tensor, npieces: int, count: int, out: DeviceBatch,
               stream=None):
        """Fills rows 0 .. count-1 of ``out`` (f64 x0) from request blocks in the byte
        buffer ``buf`` as described by ``npieces`` links_piece records in the device
        tensor ``pieces`` (PIECE_DTYPE bytes); rows count .. out.B-1 get n = 0."""
        cb = out.cstruct()
        _check(load().links_gather(self._h, _ptr(buf), _ptr(pieces), int(npieces), int(count), ctypes.byref(cb),
                                   _stream(stream)), "links_gather")

    # ------------------------------------------------------------------ normalisation
    def normalize_paths(self, paths: torch.Tensor, mode: int = NORM_PCA, out: Optional[torch.Tensor] = None,
                        xform: Optional[torch.Tensor] = None, stream=None):
        if paths.dtype != torch.float32:
            raise ValueError("paths must be float32")
        Pn, T = int(paths.shape[0]), int(paths.shape[1])
        out = torch.empty_like(paths) if out is None else out
        xform = torch.empty((Pn, 5), dtype=torch.float32, device=paths.device) if xform is None else xform
        _check(load().links_normalize_paths(self._h, _ptr(paths), Pn, T, mode, _ptr(out), _ptr(xform), _stream(stream)),
               "links_normalize_paths")
        return out, xform

    def normalize_paths_n(self, paths: torch.Tensor, count: torch.Tensor, mode: int = NORM_PCA,
                          out: Optional[torch.Tensor] = None, xform: Optional[torch.Tensor] = None, stream=None):
        """Normalises the first min(count[0], len(paths)) rows; count is a device int32."""
        cap, T = int(paths.shape[0]), int(paths.shape[1])
        out = torch.empty_like(paths) if out is None else out
        xform = torch.empty((cap, 5), dtype=torch.float32, device=paths.device) if xform is None else xform
        _check(load().links_normalize_paths_n(self._h, _ptr(paths), _ptr(count), cap, T, mode, _ptr(out), _ptr(xform),
                                              _stream(stream)), "links_normalize_paths_n")
        return out, xform


    def chamfer(self, bank: torch.Tensor, queries: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
        """Bidirectional chamfer distance of every query [Q,T,2] against every bank
        path [P,T,2] (float32, on the device) -> [Q,P] float32."""
        bank, queries = _paths_arg(bank, "bank"), _paths_arg(queries, "queries")
        Pn, T, Q = int(bank.shape[0]), int(bank.shape[1]), int(queries.shape[0])
        if int(queries.shape[1]) != T:
            raise ValueError("bank and queries need the same number of points")
        out = torch.empty((Q, Pn), dtype=torch.float32, device=bank.device) if out is None else out
        _check(load().links_chamfer(self._h, _ptr(bank), Pn, T, _ptr(queries), Q, _ptr(out), _stream(stream)),
               "links_chamfer")
        return out

    def chamfer_search(self, bank: torch.Tensor, queries: torch.Tensor, k: int = 3, cutoff: float = 0.03,
                       order: int = SEARCH_FIRST, stream=None):
        """Retrieval of k bank paths per query (see links_chamfer_search) ->
        (idx [Q,k] int64, dist [Q,k] float32); returns once the search is done."""
        bank, queries = _paths_arg(bank, "bank"), _paths_arg(queries, "queries")
        Pn, T, Q = int(bank.shape[0]), int(bank.shape[1]), int(queries.shape[0])
        if int(queries.shape[1]) != T:
            raise ValueError("bank and queries need the same number of points")
        idx = torch.empty((Q, k), dtype=torch.int64, device=bank.device)
        dist = torch.empty((Q, k), dtype=torch.float32, device=bank.device)
        _check(load().links_chamfer_search(self._h, _ptr(bank), Pn, T, _ptr(queries), Q, k, float(cutoff), order,
                                           _ptr(idx), _ptr(dist), _stream(stream)), "links_chamfer_search")
        return idx, dist

class Graph:
    """A recorded links_simulate launch sequence (see links_graph_create)."""

    def __init__(self, handle, ctx: "Context", batch: DeviceBatch, out: dict):
        self._h = handle
        self._ctx = ctx      # the context outlives the graph
        self.batch = batch   # inputs and outputs stay alive with the graph
        self.out = out

    def launch(self, stream=None):
        _check(load().links_graph_launch(self._h, _stream(stream)), "links_graph_launch")
        return self.out

    def close(self):
        if getattr(self, "_h", None):
            load().links_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
