"""Hand-built mechanisms for tests (edge lists -> library input layout)."""
import itertools

import numpy as np

from paper_2208_14567_amd.gen import Batch


def build(mechs, J=None):
    """mechs: list of dicts with keys n, edges, fixed (iterable), motor (pivot, tip), x0 [n,2]."""
    J = J or max(m["n"] for m in mechs)
    B = len(mechs)
    b = Batch(np.zeros(B, np.uint8), np.zeros((B, J), np.uint32), np.zeros(B, np.uint32),
              np.zeros((B, 2), np.uint8), np.zeros((B, J, 2), np.float64))
    for c, m in enumerate(mechs):
        b.n[c] = m["n"]
        for i, j in m["edges"]:
            b.adj[c, i] |= np.uint32(1 << j)
            b.adj[c, j] |= np.uint32(1 << i)
        for f in m["fixed"]:
            b.fixed[c] |= np.uint32(1 << f)
        b.motor[c] = m.get("motor", (0, 1))
        x0 = np.asarray(m.get("x0", np.zeros((m["n"], 2))), np.float64)
        b.x0[c, : len(x0)] = x0
    return b


def edges_of(b, c):
    n = int(b.n[c])
    return [(i, j) for i in range(n) for j in range(i + 1, n) if (int(b.adj[c, i]) >> j) & 1]


def permute(b, c, perm):
    """Relabel candidate c's joints: new label of old joint i is perm[i]."""
    n = int(b.n[c])
    m = {"n": n, "edges": [(perm[i], perm[j]) for i, j in edges_of(b, c)],
         "fixed": [perm[i] for i in range(n) if (int(b.fixed[c]) >> i) & 1],
         "motor": (perm[int(b.motor[c, 0])], perm[int(b.motor[c, 1])])}
    x0 = np.zeros((n, 2))
    for i in range(n):
        x0[perm[i]] = b.x0[c, i]
    m["x0"] = x0
    return m


def scale_of(b):
    s = np.zeros(b.B)
    for c in range(b.B):
        for i, j in edges_of(b, c):
            s[c] = max(s[c], np.hypot(*(b.x0[c, i] - b.x0[c, j])))
    return s


# Ways to break a candidate, each a rule of the library's input contract
# (links_solve_order / links_simulate): the last two break nothing.
MALFORM_KINDS = ["one_way_link", "self_loop", "link_beyond_n", "row_beyond_n", "fixed_beyond_n",
                 "pivot_is_tip", "pivot_free", "tip_fixed", "no_actuator_link", "nan_position",
                 "inf_position", "zero_length_link", "n_too_large", "n_too_small", "pivot_beyond_n",
                 "nan_beyond_n", "tiny_link", "untouched"]
MALFORM_BENIGN = {"nan_beyond_n", "untouched"}
MALFORM_EITHER = {"tiny_link"}   # a link within a few rounding steps of the 1e-12 limit


def malform(b, seed, frac=0.8):
    """A copy of batch b with about `frac` of its candidates broken in one of the
    MALFORM_KINDS ways.  Returns (batch, kind index per candidate)."""
    rng = np.random.default_rng(seed)
    B, J = b.adj.shape
    o = Batch(b.n.copy(), b.adj.copy(), b.fixed.copy(), b.motor.copy(), b.x0.copy())
    kinds = np.full(B, MALFORM_KINDS.index("untouched"), np.int64)
    for c in range(B):
        if rng.random() >= frac:
            continue
        k = int(rng.integers(0, len(MALFORM_KINDS) - 1))
        n = int(o.n[c])
        pv, tp = int(o.motor[c, 0]), int(o.motor[c, 1])
        name = MALFORM_KINDS[k]
        if name in ("link_beyond_n", "row_beyond_n", "fixed_beyond_n", "nan_beyond_n", "n_too_large") and n >= J:
            k = MALFORM_KINDS.index("untouched")
        elif name == "one_way_link":
            i, j = rng.choice(n, 2, replace=False)
            o.adj[c, i] ^= np.uint32(1 << int(j))
        elif name == "self_loop":
            i = int(rng.integers(0, n))
            o.adj[c, i] |= np.uint32(1 << i)
        elif name == "link_beyond_n":
            i, j = int(rng.integers(0, n)), int(rng.integers(n, J))
            o.adj[c, i] |= np.uint32(1 << j)
            o.adj[c, j] |= np.uint32(1 << i)
        elif name == "row_beyond_n":
            o.adj[c, int(rng.integers(n, J))] = np.uint32(1 << int(rng.integers(0, n)))
        elif name == "fixed_beyond_n":
            o.fixed[c] |= np.uint32(1 << int(rng.integers(n, 32)))
        elif name == "pivot_is_tip":
            o.motor[c, 1] = pv
        elif name == "pivot_free":
            o.fixed[c] &= ~np.uint32(1 << pv)
        elif name == "tip_fixed":
            o.fixed[c] |= np.uint32(1 << tp)
        elif name == "no_actuator_link":
            o.adj[c, pv] &= ~np.uint32(1 << tp)
            o.adj[c, tp] &= ~np.uint32(1 << pv)
        elif name in ("nan_position", "inf_position"):
            o.x0[c, int(rng.integers(0, n)), int(rng.integers(0, 2))] = np.nan if name == "nan_position" else -np.inf
        elif name == "zero_length_link":
            i = int(rng.integers(0, n))
            row = int(o.adj[c, i])
            nb = [j for j in range(n) if (row >> j) & 1]
            if nb:
                o.x0[c, int(rng.choice(nb))] = o.x0[c, i]
            else:
                k = MALFORM_KINDS.index("untouched")
        elif name == "n_too_large":
            o.n[c] = J + 1
        elif name == "n_too_small":
            o.n[c] = int(rng.integers(0, 3))
        elif name == "pivot_beyond_n":
            o.motor[c, 0] = int(rng.integers(n, 256))
        elif name == "nan_beyond_n":
            o.x0[c, int(rng.integers(n, J))] = np.nan
        elif name == "tiny_link":
            i = int(rng.integers(0, n))
            nb = [j for j in range(n) if (int(o.adj[c, i]) >> j) & 1]
            if nb:
                th = rng.random() * 2 * np.pi
                L = 1e-12 * (1 + int(rng.integers(-3, 4)) * 1e-4)
                o.x0[c, int(rng.choice(nb))] = o.x0[c, i] + L * np.array([np.cos(th), np.sin(th)])
            else:
                k = MALFORM_KINDS.index("untouched")
        kinds[c] = k
    return o, kinds
