"""Seeded synthetic candidate generator.

This module produces the inputs that both the FP64 oracle and the HIP path consume.
It holds none of the simulation's arithmetic: it only draws topologies and initial
positions.  Every random number is a pure function of ``(seed, candidate, draw)``:

* SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014): state advances by the golden gamma
  ``0x9E3779B97F4A7C15`` and each output is the state passed through the
  finaliser ``mix64``.
* Candidate ``c`` owns the stream whose state is the ``c``-th output of
  SplitMix64 seeded with ``seed``; draw ``k`` of that candidate is the ``k``-th
  output of SplitMix64 seeded with that state.
* A uniform float takes the top 24 bits of a draw, so every coordinate is a
  multiple of 2^-24 in [0, 1) and is exactly representable in FP32 and FP64 --
  the FP32 and FP64 paths therefore see identical inputs.

Topologies follow the paper's dyadic J operator (Methodology, "1-DOF Operator"
and "Generating Valid Topologies"): the initial mechanism is ground joint 0,
actuator tip 1 (link 0-1) and a floating ground joint 2; each further joint is
linked to two existing joints that are not both fixed (N_s).  In ``paper`` mode a
new fixed joint with no links (N_g) is added instead with probability 1/4, the
N_g : N_s ratio of one to three.

Draw numbering inside a candidate's stream:
  0                      joint count
  1 + 2j, 2 + 2j         x and y of joint j (j < 32)
  65 + 64(k-3) + 3a + r  topology draws for joint k, attempt a (r: 0 op, 1 i, 2 j)
  (four-bar rejection)   1 + 10a + 2j, 2 + 10a + 2j for attempt a, joint j < 5
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional, Sequence

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_INV24 = 1.0 / float(1 << 24)

DRAW_N = 0
DRAW_POS = 1
DRAW_TOPO = 65
TOPO_ATTEMPTS = 21


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output finaliser (variant 13 of Stafford's mixers)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_state(seed: int, cand: np.ndarray) -> np.ndarray:
    """State of candidate ``cand``'s stream: output ``cand`` of SplitMix64(seed)."""
    cand = np.asarray(cand, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (cand + np.uint64(1)) * GAMMA)


def draw_u64(state: np.ndarray, k) -> np.ndarray:
    """Draw ``k`` (scalar or array) of the streams with the given states."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(state + (k + np.uint64(1)) * GAMMA)


def draw_u24(state: np.ndarray, k) -> np.ndarray:
    """Uniform float64 in [0, 1) with 24 random bits (exact in FP32)."""
    return (draw_u64(state, k) >> np.uint64(40)).astype(np.float64) * _INV24


@dataclasses.dataclass
class Batch:
    """A batch of candidate mechanisms in the library's input layout.

    n      uint8  [B]        joint count
    adj    uint32 [B, J]     row bitmasks of the symmetric adjacency matrix
    fixed  uint32 [B]        bitmask of ground (fixed) joints
    motor  uint8  [B, 2]     (pivot, tip) of the actuator arm
    x0     float64[B, J, 2]  initial joint positions (zero beyond n)
    """

    n: np.ndarray
    adj: np.ndarray
    fixed: np.ndarray
    motor: np.ndarray
    x0: np.ndarray

    @property
    def B(self) -> int:
        return int(self.n.shape[0])

    @property
    def J(self) -> int:
        return int(self.adj.shape[1])

    def take(self, idx) -> "Batch":
        idx = np.asarray(idx)
        return Batch(self.n[idx].copy(), self.adj[idx].copy(), self.fixed[idx].copy(),
                     self.motor[idx].copy(), self.x0[idx].copy())

    def slice(self, lo: int, hi: int) -> "Batch":
        return Batch(self.n[lo:hi], self.adj[lo:hi], self.fixed[lo:hi], self.motor[lo:hi], self.x0[lo:hi])

    @staticmethod
    def concat(parts: Sequence["Batch"]) -> "Batch":
        J = max(p.J for p in parts)
        def pad(p: "Batch"):
            if p.J == J:
                return p
            adj = np.zeros((p.B, J), np.uint32); adj[:, :p.J] = p.adj
            x0 = np.zeros((p.B, J, 2), np.float64); x0[:, :p.J] = p.x0
            return Batch(p.n, adj, p.fixed, p.motor, x0)
        ps = [pad(p) for p in parts]
        return Batch(np.concatenate([p.n for p in ps]), np.concatenate([p.adj for p in ps]),
                     np.concatenate([p.fixed for p in ps]), np.concatenate([p.motor for p in ps]),
                     np.concatenate([p.x0 for p in ps]))


def empty_batch(B: int, J: int) -> Batch:
    return Batch(np.zeros(B, np.uint8), np.zeros((B, J), np.uint32), np.zeros(B, np.uint32),
                 np.zeros((B, 2), np.uint8), np.zeros((B, J, 2), np.float64))


# --------------------------------------------------------------------------- joint counts

def n_uniform(lo: int, hi: int) -> Callable[[np.ndarray], np.ndarray]:
    """n ~ U{lo..hi} from a single 24-bit draw."""
    def f(u: np.ndarray) -> np.ndarray:
        return (lo + np.floor(u * (hi - lo + 1))).astype(np.int64).clip(lo, hi)
    return f


def n_mixture(bands: Sequence[tuple], weights: Sequence[float]) -> Callable[[np.ndarray], np.ndarray]:
    """n from a mixture of uniform bands, e.g. ((6,8),(9,14),(15,20)) with (.6,.3,.1)."""
    w = np.asarray(weights, dtype=np.float64)
    cum = np.cumsum(w / w.sum())
    def f(u: np.ndarray) -> np.ndarray:
        band = np.searchsorted(cum, u, side="right").clip(0, len(bands) - 1)
        lo_b = np.array([b[0] for b in bands])[band]
        hi_b = np.array([b[1] for b in bands])[band]
        c_lo = np.concatenate([[0.0], cum[:-1]])[band]
        c_hi = cum[band]
        v = ((u - c_lo) / np.maximum(c_hi - c_lo, 1e-300)).clip(0.0, np.nextafter(1.0, 0.0))
        return (lo_b + np.floor(v * (hi_b - lo_b + 1))).astype(np.int64).clip(lo_b, hi_b)
    return f


# --------------------------------------------------------------------------- dyad-built topologies

def dyad_batch(B: int, seed: int, n_dist: Callable[[np.ndarray], np.ndarray], J: int = 20,
               paper_mode: bool = False, first: int = 0, chunk: int = 1 << 20, rules: bool = False) -> Batch:
    """Random 1-DOF candidates built by repeated dyad addition (J operator).

    Joint 0 is the fixed pivot, joint 1 the actuated tip (link 0-1), joint 2 a fixed
    joint; joints 3..n-1 are each linked to two existing joints that are not both
    fixed.  All positions are uniform in [0,1)^2.  ``first`` offsets the candidate
    index so a large batch can be produced in independent chunks.

    ``rules`` applies the paper's two topology rules ("Generating Valid
    Topologies"): the last joint depends on every other joint (the mechanism is
    not reducible), and it is linked to no fixed joint.  Each operator draw is
    kept only if the rules can still be met by the joints left to add (see
    ``_rules_feasible``); after the attempt budget a deterministic choice that
    uses up the most pending joints is taken.  Needs n >= 5.
    """
    out = empty_batch(B, J)
    for lo in range(0, B, chunk):
        hi = min(B, lo + chunk)
        cand = np.arange(first + lo, first + hi, dtype=np.uint64)
        _dyad_chunk(out, lo, hi, seed, n_dist, J, paper_mode, cand, rules)
    return out


def dyad_batch_at(index, seed: int, n_dist: Callable[[np.ndarray], np.ndarray], J: int = 20,
                  paper_mode: bool = False, rules: bool = False, chunk: int = 1 << 20) -> Batch:
    """The candidates of ``dyad_batch`` at the given indices of the seed's sequence
    (any order, repeats allowed): row i equals row index[i] - first of a
    ``dyad_batch`` that covers it, since every draw depends only on (seed,
    candidate index, draw number)."""
    idx = np.asarray(index, dtype=np.int64).reshape(-1)
    if idx.size and idx.min() < 0:
        raise ValueError("candidate indices must be non-negative")
    out = empty_batch(idx.size, J)
    for lo in range(0, idx.size, chunk):
        hi = min(idx.size, lo + chunk)
        _dyad_chunk(out, lo, hi, seed, n_dist, J, paper_mode, idx[lo:hi].astype(np.uint64), rules)
    return out


def _popcount(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.uint64)
    c = np.zeros(x.shape, np.int64)
    for b in range(32):
        c += ((x >> np.uint64(b)) & np.uint64(1)).astype(np.int64)
    return c


def _lowest(mask: np.ndarray) -> np.ndarray:
    """Index of the lowest set bit of each mask (32 where none)."""
    m = mask.astype(np.uint64)
    out = np.full(m.shape, 32, np.int64)
    for b in range(31, -1, -1):
        out = np.where(((m >> np.uint64(b)) & np.uint64(1)) == 1, b, out)
    return out


def _rules_feasible(U: np.ndarray, fixed: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Whether the topology rules can still be met with r joints left to add after
    the current one.  U holds the pending joints: placed or fixed joints that no
    later joint uses yet (each must still lead to the last joint).  Every further
    joint except the last can use up at most two pending joints, at most one of
    them fixed (two fixed parents are not allowed), and adds itself; the last one
    must use up all that remain, at most two, none fixed.  So: |U| <= r + 1 and
    at most r - 1 pending fixed joints."""
    return (_popcount(U) <= r + 1) & (_popcount(U & fixed) <= r - 1)


def _dyad_chunk(out: Batch, lo: int, hi: int, seed: int, n_dist, J: int, paper_mode: bool, cand: np.ndarray,
                rules: bool = False):
    """Rows lo..hi of out: the candidates with the global indices cand."""
    m = hi - lo
    st = stream_state(seed, cand)
    n = n_dist(draw_u24(st, DRAW_N)).astype(np.int64)
    if n.min() < 3 or n.max() > J:
        raise ValueError("joint count distribution outside [3, J]")
    if rules and n.min() < 5:
        raise ValueError("the topology rules need at least 5 joints")
    adj = np.zeros((m, J), np.uint32)
    fixed = np.full(m, 0b101, np.uint32)
    one = np.uint32(1)
    adj[:, 0] |= one << np.uint32(1)
    adj[:, 1] |= one << np.uint32(0)
    rows = np.arange(m)
    U = np.full(m, 0b110, np.uint32)     # pending joints (rules): the tip and fixed joint 2
    for k in range(3, J):
        act = n > k
        if not act.any():
            break
        base = DRAW_TOPO + 64 * (k - 3)
        bit = one << np.uint32(k)
        r = n - 1 - k                     # joints still to add after this one
        last = act & (r == 0)
        if paper_mode:
            is_g = act & (draw_u24(st, base) < 0.25)
            if rules:
                is_g &= ~last & _rules_feasible(U | bit, fixed | bit, r)
            fixed = np.where(is_g, fixed | bit, fixed)
            if rules:
                U = np.where(is_g, U | bit, U)
        else:
            is_g = np.zeros(m, bool)
        need = act & ~is_g
        pi = np.zeros(m, np.int64)
        pj = np.zeros(m, np.int64)
        done = ~need
        for a in range(TOPO_ATTEMPTS):
            if done.all():
                break
            ui = draw_u24(st, base + 3 * a + 1)
            uj = draw_u24(st, base + 3 * a + 2)
            i = np.floor(ui * k).astype(np.int64).clip(0, k - 1)
            j = np.floor(uj * (k - 1)).astype(np.int64).clip(0, k - 2)
            j = np.where(j >= i, j + 1, j)
            fi = ((fixed >> i.astype(np.uint32)) & one) == one
            fj = ((fixed >> j.astype(np.uint32)) & one) == one
            both_fixed = fi & fj
            take = ~done & ~both_fixed
            if rules:
                # the last joint's parents are fixed by the rules (below); any other
                # draw is kept if the rules can still be met afterwards
                pair = (one << i.astype(np.uint32)) | (one << j.astype(np.uint32))
                take &= ~last & _rules_feasible((U & ~pair) | bit, fixed, r)
            pi = np.where(take, i, pi)
            pj = np.where(take, j, pj)
            done |= take
        if rules:
            nonfixed = ((one << np.uint32(k)) - one) & ~fixed
            uf, un = U & fixed, U & ~fixed
            # no draw kept: the choice that uses up the most pending joints, a
            # pending fixed one first, then pending non-fixed ones, then the lowest
            # non-fixed joint
            g1 = np.where(uf != 0, _lowest(uf), np.where(un != 0, _lowest(un), _lowest(nonfixed)))
            m1 = one << np.minimum(g1, 31).astype(np.uint32)
            g2 = np.where((un & ~m1) != 0, _lowest(un & ~m1), _lowest(nonfixed & ~m1))
            # the last joint: the one or two pending joints (never fixed by then);
            # with one, a partner among the other non-fixed joints, the q-th in
            # index order with q from the draw of the first attempt's first partner
            l1 = _lowest(un)
            ml = one << np.minimum(l1, 31).astype(np.uint32)
            others = nonfixed & ~ml
            q = np.floor(draw_u24(st, base + 1) * np.maximum(_popcount(others), 1)).astype(np.int64)
            partner = np.full(m, 32, np.int64)
            seen = np.zeros(m, np.int64)
            for bb in range(32):
                has = ((others >> np.uint32(bb)) & one) == one
                partner = np.where(has & (seen == q), bb, partner)
                seen += has
            l2 = np.where((un & ~ml) != 0, _lowest(un & ~ml), partner)
            pi = np.where(done, pi, np.where(last, l1, g1))
            pj = np.where(done, pj, np.where(last, l2, g2))
            if np.any(need & ((pi > 31) | (pj > 31))):
                raise RuntimeError("topology rules: no parents left (generator bug)")
            pair = (one << pi.astype(np.uint32)) | (one << pj.astype(np.uint32))
            U = np.where(need, (U & ~pair) | bit, U)
        else:
            # deterministic fallback after the attempt budget: the actuator arm (0, 1)
            pi = np.where(done, pi, 0)
            pj = np.where(done, pj, 1)
        kk = np.uint32(k)
        sel = rows[need]
        adj[sel, k] |= (one << pi[need].astype(np.uint32)) | (one << pj[need].astype(np.uint32))
        np.bitwise_or.at(adj, (sel, pi[need]), one << kk)
        np.bitwise_or.at(adj, (sel, pj[need]), one << kk)
    x0 = np.zeros((m, J, 2), np.float64)
    for j in range(J):
        live = n > j
        x0[:, j, 0] = np.where(live, draw_u24(st, DRAW_POS + 2 * j), 0.0)
        x0[:, j, 1] = np.where(live, draw_u24(st, DRAW_POS + 2 * j + 1), 0.0)
    out.n[lo:hi] = n.astype(np.uint8)
    out.adj[lo:hi] = adj
    out.fixed[lo:hi] = fixed
    out.motor[lo:hi, 0] = 0
    out.motor[lo:hi, 1] = 1
    out.x0[lo:hi] = x0


def standardize_paper(b: Batch) -> Batch:
    """Paper mode positions: pivot at (0.5, 0.5), actuator arm of length 0.05 and
    horizontal at the initial position (Methodology, "Finding Valid Initial
    Positions")."""
    x0 = b.x0.copy()
    x0[:, 0] = (0.5, 0.5)
    x0[:, 1] = (0.55, 0.5)
    return Batch(b.n, b.adj, b.fixed, b.motor, x0)


# --------------------------------------------------------------------------- four-bars with coupler point

FOURBAR_EDGES = ((0, 1), (1, 3), (2, 3), (1, 4), (3, 4))


def fourbar_topology(B: int, J: int = 5) -> Batch:
    b = empty_batch(B, J)
    b.n[:] = 5
    b.fixed[:] = 0b101
    b.motor[:, 0] = 0
    b.motor[:, 1] = 1
    for i, j in FOURBAR_EDGES:
        b.adj[:, i] |= np.uint32(1 << j)
        b.adj[:, j] |= np.uint32(1 << i)
    return b


def _seg(p, q):
    return np.hypot(p[..., 0] - q[..., 0], p[..., 1] - q[..., 1])


def fourbar_batch(B: int, seed: int, crank_rocker: bool = True, grashof_margin: float = 1e-3,
                  min_height: float = 1e-2, J: int = 5, max_attempts: int = 100000,
                  first: int = 0) -> Batch:
    """Four-bars with a coupler point: ground pivots 0 and 2, crank tip 1, rocker
    tip 3, coupler joint 4 tied to joints 1 and 3.

    Positions are uniform in [0,1)^2.  With ``crank_rocker`` every candidate is
    rejection-sampled until it is a Grashof crank-rocker (the crank is the shortest
    link and s + l <= p + q - margin*l) whose coupler triangle height is at least
    ``min_height`` times the longest link.  This is input selection only; validity
    is decided by the simulation.
    """
    b = fourbar_topology(B, J)
    cand = np.arange(first, first + B, dtype=np.uint64)
    st = stream_state(seed, cand)
    pos = np.zeros((B, 5, 2))
    todo = np.arange(B)
    for a in range(max_attempts):
        if todo.size == 0:
            break
        s = st[todo]
        p = np.stack([np.stack([draw_u24(s, 1 + 10 * a + 2 * j), draw_u24(s, 2 + 10 * a + 2 * j)], -1)
                      for j in range(5)], axis=1)
        if not crank_rocker:
            pos[todo] = p
            todo = todo[:0]
            break
        crank = _seg(p[:, 0], p[:, 1])
        coupler = _seg(p[:, 1], p[:, 3])
        rocker = _seg(p[:, 2], p[:, 3])
        ground = _seg(p[:, 0], p[:, 2])
        L = np.stack([crank, coupler, rocker, ground], -1)
        s_, l_ = L.min(-1), L.max(-1)
        pq = L.sum(-1) - s_ - l_
        e14 = _seg(p[:, 1], p[:, 4])
        e34 = _seg(p[:, 3], p[:, 4])
        longest = np.maximum(l_, np.maximum(e14, e34))
        # twice the triangle area over its base gives the height of joint 4 above 1-3
        cross = np.abs((p[:, 3, 0] - p[:, 1, 0]) * (p[:, 4, 1] - p[:, 1, 1]) -
                       (p[:, 3, 1] - p[:, 1, 1]) * (p[:, 4, 0] - p[:, 1, 0]))
        height = cross / np.maximum(coupler, 1e-300)
        ok = (crank <= s_) & (s_ + l_ <= pq - grashof_margin * l_) & (height >= min_height * longest)
        acc = todo[ok]
        pos[acc] = p[ok]
        todo = todo[~ok]
    if todo.size:
        raise RuntimeError("four-bar rejection sampling did not finish")
    b.x0[:, :5] = pos
    return b


# --------------------------------------------------------------------------- named workloads

def workload(name: str, B: Optional[int] = None, seed: Optional[int] = None, first: int = 0) -> Batch:
    """Named synthetic workloads with the paper's shapes.

    fourbar        crank-rocker four-bars with a coupler point (10,000 by default)
    fourbar_u      the same topology with unconstrained uniform positions
    dyad_6_20      dyad-built candidates, n ~ U{6..20}
    dyad_skewed    n: 60% U{6..8}, 30% U{9..14}, 10% U{15..20}
    dyad_4_20      n ~ U{4..20} (serving requests)
    paper_8_20     paper-mode generation (N_g with p=1/4, standardised actuator), n ~ U{8..20}
    paper_rules_8_20  the same with the paper's topology rules (not reducible, last
                   joint linked to no fixed joint)
    dyad_rules_6_20   dyad_6_20 with the topology rules
    """
    if name == "fourbar":
        return fourbar_batch(B or 10_000, 1 if seed is None else seed, True, first=first)
    if name == "fourbar_u":
        return fourbar_batch(B or 10_000, 1 if seed is None else seed, False, first=first)
    if name == "dyad_6_20":
        return dyad_batch(B or 1_000_000, 2 if seed is None else seed, n_uniform(6, 20), 20, first=first)
    if name == "dyad_skewed":
        return dyad_batch(B or 4_000_000, 3 if seed is None else seed,
                          n_mixture(((6, 8), (9, 14), (15, 20)), (0.6, 0.3, 0.1)), 20, first=first)
    if name == "dyad_4_20":
        return dyad_batch(B or 200_000, 4 if seed is None else seed, n_uniform(4, 20), 20, first=first)
    if name == "paper_8_20":
        return standardize_paper(dyad_batch(B or 100_000, 6 if seed is None else seed, n_uniform(8, 20),
                                            20, paper_mode=True, first=first))
    if name == "paper_rules_8_20":
        return standardize_paper(dyad_batch(B or 100_000, 10 if seed is None else seed, n_uniform(8, 20),
                                            20, paper_mode=True, first=first, rules=True))
    if name == "dyad_rules_6_20":
        return dyad_batch(B or 1_000_000, 11 if seed is None else seed, n_uniform(6, 20), 20, first=first,
                          rules=True)
    raise KeyError(name)


def closed_curves(P: int, T: int, seed: int, harmonics: int = 5) -> np.ndarray:
    """P closed curves of T points each, float32 [P,T,2], sampled at equally
    spaced parameter values: random Fourier series with amplitudes falling as
    1/k^1.5 around a centre near (0.5, 0.5), so that the curves span about a unit
    box like paths in the paper's normalised frame (synthetic stand-ins for a
    bank of normalised coupler paths)."""
    rng = np.random.default_rng(seed)
    th = 2.0 * np.pi * np.arange(T) / T
    k = np.arange(1, harmonics + 1)
    amp = 0.25 / k ** 1.5
    c = rng.normal(size=(P, 4, harmonics)) * amp                    # cos x, sin x, cos y, sin y
    cos_kt, sin_kt = np.cos(np.outer(k, th)), np.sin(np.outer(k, th))  # [H, T]
    x = c[:, 0] @ cos_kt + c[:, 1] @ sin_kt
    y = c[:, 2] @ cos_kt + c[:, 3] @ sin_kt
    centre = 0.5 + 0.05 * rng.normal(size=(P, 2))
    return np.stack([x + centre[:, :1], y + centre[:, 1:]], axis=-1).astype(np.float32)


def near_copies(base: np.ndarray, n: int, sigma: float, seed: int) -> np.ndarray:
    """n noisy copies of each curve of base [P,T,2]: every point moved by
    N(0, sigma^2) per coordinate and the point order rotated by a random shift
    (the same path started elsewhere) -> float32 [P*n,T,2]."""
    rng = np.random.default_rng(seed)
    P, T = base.shape[0], base.shape[1]
    out = np.repeat(base.astype(np.float64), n, axis=0)
    shift = rng.integers(0, T, size=P * n)
    rows = (np.arange(T)[None, :] + shift[:, None]) % T
    out = np.take_along_axis(out, rows[:, :, None], axis=1)
    out += rng.normal(scale=sigma, size=out.shape)
    return out.astype(np.float32)
