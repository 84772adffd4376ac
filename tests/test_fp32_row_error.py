"""How far FP32 coupler rows are from FP64 ones, against the FP32 pass's tracked
error bound (CPU, no GPU).

The FP32 pass decides a candidate in FP32 while a first-order bound of every
joint's FP32 error (seeded by the rounding of x0 and of the crank table,
amplified through each placement by 2 ra rb / sqrt(K), plus the placement's own
rounding) keeps its decisions outside the bands; the coupler rows are then
recomputed in FP64.  Here the FP32 arithmetic of a placement (the kernel's
formulas: d^2, Heron's K, 1/d and sqrt(K) through reciprocal square roots, the
foot and the normal) is emulated in numpy for the valid candidates of the
headline workload's first 4,000 candidates, with every side taken from the
oracle's FP64 positions (the sides a path pass given recorded sides would use),
and compared with the oracle's FP64 positions of the output joint at every step.

Checked: the emulated FP32 error of the output joint never exceeds the tracked
bound (the bound is a bound).  Reported: how loose the bound is and how many
rows an FP32 path with this bound as its certificate could keep at the 1e-5
scale tolerance.  The emulation's reciprocal square roots are correctly rounded
(the hardware's are within a unit or so); the bound's per-placement rounding
term allows four units.
"""
import numpy as np

import oracle
from paper_2208_14567_amd import gen

U = 2.0 ** -22  # the kernel's relative rounding unit of a placement


def f32(x):
    return np.asarray(x, np.float64).astype(np.float32)


def fma32(a, b, c):
    # exact product of two FP32 values in FP64, one FP64 addition, rounded to FP32
    return f32(np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64))


def bound_up(x):
    """The kernel's storage of a bound: the upper 16 bits of its FP32 encoding, rounded up."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    return (((u + 0xFFFF) >> 16) << 16).astype(np.uint32).view(np.float32)


def longest_link(batch):
    scale = np.zeros(batch.B)
    for c in range(batch.B):
        for i in range(batch.n[c]):
            for j in range(i + 1, batch.n[c]):
                if (int(batch.adj[c, i]) >> j) & 1:
                    scale[c] = max(scale[c], float(np.hypot(*(batch.x0[c, i] - batch.x0[c, j]))))
    return scale


def emulate(batch, order, nd, ref_pos, T, scale):
    """FP32 positions of the output joint [B, T, 2] and their tracked bounds [B, T],
    sides forced to the FP64 ones."""
    B = batch.B
    x0 = batch.x0.astype(np.float64)
    piv = batch.motor[:, 0].astype(np.int64)
    tip = batch.motor[:, 1].astype(np.int64)
    rows = np.arange(B)
    P = f32(x0)                                      # [B, J, 2] FP32 positions by joint
    E = bound_up(f32(U * (np.abs(P[..., 0]).astype(np.float64) + np.abs(P[..., 1]))))  # rounding of x0
    p0 = x0[rows, piv]
    v = x0[rows, tip] - p0
    px, py, vx, vy = f32(p0[:, 0]), f32(p0[:, 1]), f32(v[:, 0]), f32(v[:, 1])
    Ut = f32(U * (np.abs(p0[:, 0]) + np.abs(p0[:, 1]) + np.abs(v[:, 0]) + np.abs(v[:, 1])))
    D = nd.astype(np.int64)
    Dmax = int(D.max())
    k_ = order[:, :Dmax, 0].astype(np.int64)
    a_ = order[:, :Dmax, 1].astype(np.int64)
    b_ = order[:, :Dmax, 2].astype(np.int64)
    # per-dyad constants rounded from FP64, as the set-up pass stores them
    def sq(i, j):
        d = x0[rows[:, None], i] - x0[rows[:, None], j]
        return d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]
    ra2 = sq(k_, a_)
    rb2 = sq(k_, b_)
    ra, rb = np.sqrt(ra2), np.sqrt(rb2)
    S, Dm, Kc = f32((ra + rb) ** 2), f32((ra - rb) ** 2), f32(0.5 * (ra2 - rb2))
    U2 = f32(U * 2.0 * scale)                        # rounding of a placement relative to the link lengths
    out = k_[rows, D - 1]
    path = np.zeros((B, T, 2), np.float32)
    bound = np.zeros((B, T), np.float32)
    for t in range(T):
        th = 2.0 * np.pi * t / T
        c, s = np.float32(np.cos(th)), np.float32(np.sin(th))
        tx = fma32(c, vx, fma32(-s, vy, px))
        ty = fma32(s, vx, fma32(c, vy, py))
        P[rows, tip, 0], P[rows, tip, 1] = tx, ty
        E[rows, tip] = bound_up(Ut)
        for j in range(Dmax):
            act = j < D
            kk, aa, bb = k_[:, j], a_[:, j], b_[:, j]
            pa, pb = P[rows, aa], P[rows, bb]
            dx = f32(pb[:, 0].astype(np.float64) - pa[:, 0])
            dy = f32(pb[:, 1].astype(np.float64) - pa[:, 1])
            d2 = fma32(dy, dy, f32(dx.astype(np.float64) * dx))
            Sj, Dmj, Kcj = S[:, j], Dm[:, j], Kc[:, j]
            K = f32(f32(Sj.astype(np.float64) - d2).astype(np.float64) * f32(d2.astype(np.float64) - Dmj))
            # (lanes past their solve order compute on padding and are discarded)
            with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
                rd = f32(1.0 / np.sqrt(d2.astype(np.float64)))
                inv = f32(rd.astype(np.float64) * rd)
                Kp = np.maximum(K, np.float32(1e-30))
                rK = f32(1.0 / np.sqrt(Kp.astype(np.float64)))
                sK = f32(Kp.astype(np.float64) * rK)
                be = f32(sK.astype(np.float64) * f32(0.5 * inv.astype(np.float64)))
                al = fma32(Kcj, inv, 0.5)
                bx, by = fma32(al, dx, pa[:, 0]), fma32(al, dy, pa[:, 1])
                ox, oy = f32(-be.astype(np.float64) * dy), f32(be.astype(np.float64) * dx)
            # the FP64 side of the joint at this step
            q = ref_pos[rows, t]
            qa, qb, qk = q[rows, aa], q[rows, bb], q[rows, kk]
            cr = (qb[:, 0] - qa[:, 0]) * (qk[:, 1] - qa[:, 1]) - (qb[:, 1] - qa[:, 1]) * (qk[:, 0] - qa[:, 0])
            sgn = np.where(cr >= 0.0, np.float32(1.0), np.float32(-1.0))
            with np.errstate(invalid="ignore", over="ignore"):
                nx, ny = fma32(sgn, ox, bx), fma32(sgn, oy, by)
                # tracked bound: parents amplified by 2 ra rb / sqrt(K), plus the placement's rounding
                Eab = f32(E[rows, aa].astype(np.float64) + E[rows, bb])
                R = fma32(np.float32(U), f32(np.abs(pa[:, 0]).astype(np.float64) + np.abs(pa[:, 1])), U2)
                A2 = f32(f32(0.5 * (Sj.astype(np.float64) - Dmj)).astype(np.float64) * rK)
                Ek = f32(A2.astype(np.float64) * f32(Eab.astype(np.float64) + R))
            P[rows[act], kk[act], 0] = nx[act]
            P[rows[act], kk[act], 1] = ny[act]
            E[rows[act], kk[act]] = bound_up(Ek)[act]
        path[:, t] = P[rows, out]
        bound[:, t] = E[rows, out]
    return path, bound, out


def test_fp32_rows_against_fp64_and_the_tracked_bound():
    T = 200
    b = gen.workload("dyad_6_20", 4000, seed=2)
    ref = oracle.simulate(b, T=T, pos_all=True, margins=True, nthreads=4)
    keep = (ref["status"] == 0) & ~oracle.in_band(ref["margins"])
    idx = np.nonzero(keep)[0]
    assert len(idx) > 300
    sub = b.take(idx)
    order, nd, _, st = oracle.solve_order(sub)
    assert np.all(st == 0)
    pos = ref["pos_all"][idx]
    scale = longest_link(sub)
    path32, bound, out = emulate(sub, order, nd, pos, T, scale)
    rows = np.arange(sub.B)
    exact = pos[rows, :, out]                                   # [B, T, 2]
    err = np.hypot(path32[..., 0] - exact[..., 0], path32[..., 1] - exact[..., 1])
    e_row = err.max(axis=1) / scale
    b_row = bound.max(axis=1) / scale
    # the tracked bound bounds the FP32 error at every step
    assert np.all(err <= bound * (1 + 1e-6) + 1e-30), float(np.max(err / np.maximum(bound, 1e-38)))
    ratio = bound.max(axis=1) / np.maximum(err.max(axis=1), 1e-30)
    print(f"\n[fp32 rows] {sub.B} valid rows: max error / scale median {np.median(e_row):.2e}, "
          f"99th pct {np.percentile(e_row, 99):.2e}, max {e_row.max():.2e}; rows within 1e-6: "
          f"{(e_row <= 1e-6).mean():.3f}, within 1e-5: {(e_row <= 1e-5).mean():.3f}; tracked bound / scale "
          f"median {np.median(b_row):.2e}, rows certified at 0.5e-5: {(b_row <= 0.5e-5).mean():.3f}; "
          f"bound / error median {np.median(ratio):.1f}")
