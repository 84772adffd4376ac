"""Bidirectional chamfer distance and path retrieval in FP64 -- TEST INFRASTRUCTURE ONLY.

Only the test suite and the benchmark's CPU-baseline leg may import this module.
It shares no code with the HIP path.

Follows "A Case Study of Mechanism Retrieval": two normalised paths are compared
as point sets with the bidirectional chamfer distance, a path counts as close to
a query when that distance is below a cut-off (0.03 in the paper), and two
search procedures are described:

  * FIRST -- go through the (shuffled) curated set in order until k candidates
    under the cut-off are found: the answer is the k lowest bank positions whose
    distance is below the cut-off;
  * BEST -- the k best matches over the whole set: the k smallest distances below
    the cut-off, equal distances ordered by bank position.

Reading of the metric (the paper names it but prints no formula): for point sets
A and B,

    CD(A, B) = mean_{a in A} min_{b in B} |a - b| + mean_{b in B} min_{a in A} |a - b|

with |.| the Euclidean norm (not its square), each direction averaged over its
own set.  A path with a non-finite coordinate has no distance (NaN), so it never
matches.  Everything here is plain numpy in float64.
"""
from __future__ import annotations

import numpy as np

CUTOFF = 0.03
FIRST, BEST = 0, 1


def chamfer(a: np.ndarray, b: np.ndarray) -> float:
    """CD of two point sets a [Ta,2] and b [Tb,2]."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if a.ndim != 2 or b.ndim != 2 or a.shape[1] != 2 or b.shape[1] != 2 or len(a) == 0 or len(b) == 0:
        raise ValueError("chamfer: point sets must be non-empty [n,2] arrays")
    if not (np.isfinite(a).all() and np.isfinite(b).all()):
        return float("nan")
    diff = a[:, None, :] - b[None, :, :]
    d = np.sqrt((diff * diff).sum(axis=-1))  # [Ta, Tb] Euclidean distances
    return float(d.min(axis=1).mean() + d.min(axis=0).mean())


def chamfer_bank(query: np.ndarray, bank: np.ndarray, block: int = 256) -> np.ndarray:
    """CD of one query [T,2] against every path of bank [P,T,2] -> [P] float64.

    Same definition as chamfer(), evaluated for a block of bank paths at a time."""
    q = np.asarray(query, np.float64)
    bk = np.asarray(bank, np.float64)
    if bk.ndim != 3 or bk.shape[2] != 2 or q.ndim != 2 or q.shape[1] != 2:
        raise ValueError("chamfer_bank: query [T,2] and bank [P,T,2] expected")
    out = np.empty(bk.shape[0], np.float64)
    for lo in range(0, bk.shape[0], block):
        b = bk[lo:lo + block]                               # [n, Tb, 2]
        diff = q[None, :, None, :] - b[:, None, :, :]       # [n, Ta, Tb, 2]
        d = np.sqrt((diff * diff).sum(axis=-1))
        out[lo:lo + block] = d.min(axis=2).mean(axis=1) + d.min(axis=1).mean(axis=1)
    finite = np.isfinite(bk).all(axis=(1, 2)) & bool(np.isfinite(q).all())
    out[~finite] = np.nan
    return out


def select(dist: np.ndarray, k: int, cutoff: float = CUTOFF, order: int = FIRST):
    """The answer of one search over precomputed distances [P].

    Returns (idx, dist): k int64 bank positions and their distances; missing
    entries (fewer than k paths under the cut-off) are -1 and NaN.  A NaN distance
    never counts as under the cut-off."""
    d = np.asarray(dist, np.float64)
    under = np.flatnonzero(d < cutoff)  # ascending positions; NaN compares false
    if order == FIRST:
        pick = under[:k]
    elif order == BEST:
        pick = under[np.lexsort((under, d[under]))][:k]  # by distance, then position
    else:
        raise ValueError("select: order must be FIRST or BEST")
    idx = np.full(k, -1, np.int64)
    out = np.full(k, np.nan)
    idx[:len(pick)] = pick
    out[:len(pick)] = d[pick]
    return idx, out


def search(queries: np.ndarray, bank: np.ndarray, k: int, cutoff: float = CUTOFF, order: int = FIRST):
    """select() for each query [Q,T,2] over bank [P,T,2] -> (idx [Q,k], dist [Q,k])."""
    qs = np.asarray(queries, np.float64)
    res = [select(chamfer_bank(q, bank), k, cutoff, order) for q in qs]
    return (np.stack([r[0] for r in res]) if res else np.zeros((0, k), np.int64),
            np.stack([r[1] for r in res]) if res else np.zeros((0, k)))
