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
