"""Pins of the oracle's path normalisation (Methodology, "Dataset Curation & Processing")."""
import math

import numpy as np

import oracle

T = 200


def _ellipse(A, B, T=T, ph=0.0):
    t = 2 * np.pi * np.arange(T) / T + ph
    return np.stack([A * np.cos(t), B * np.sin(t)], -1)


def _sim(p, s, ang, shift):
    c, sn = math.cos(ang), math.sin(ang)
    return s * p @ np.array([[c, -sn], [sn, c]]).T + np.asarray(shift)


def test_pca_ellipse_canonical(oracle_lib):
    e = _ellipse(3.0, 1.0)
    # a lopsided ellipse: drop the left half's sign ambiguity with an offset bump
    e[:40, 0] += 0.3
    p = _sim(e, 0.2, 1.1, (5, -2))
    out, xf = oracle.normalize_paths(p[None], oracle.NORM_PCA)
    q = out[0]
    assert np.allclose(q.mean(0), 0, atol=1e-12)
    assert abs(np.sqrt((q ** 2).sum(1).mean()) - 1) < 1e-12
    C = np.cov(q.T, bias=True)
    assert abs(C[0, 1]) < 1e-12 and C[0, 0] > C[1, 1]
    assert (q[:, 0] ** 3).sum() > 0 and int(xf[0, 4]) == 0
    # similarity invariance
    out2, _ = oracle.normalize_paths(_sim(p, 7.0, -0.4, (1, 1))[None], oracle.NORM_PCA)
    assert np.allclose(out2, out, atol=1e-10)
    # idempotence
    out3, _ = oracle.normalize_paths(out, oracle.NORM_PCA)
    assert np.allclose(out3, out, atol=1e-10)
    # xform reproduces the output
    cx, cy, s, phi, _ = xf[0]
    R = np.array([[math.cos(phi), math.sin(phi)], [-math.sin(phi), math.cos(phi)]])
    assert np.allclose(((p - [cx, cy]) / s) @ R.T, q, atol=1e-12)


def test_pca_plain_ellipse_semi_axes(oracle_lib):
    out, xf = oracle.normalize_paths(_sim(_ellipse(2.0, 1.0), 1.0, 0.3, (0, 0))[None], oracle.NORM_PCA)
    rms = math.sqrt((4.0 + 1.0) / 2)
    q = out[0]
    assert abs(np.abs(q[:, 0]).max() - 2.0 / rms) < 1e-9 and abs(np.abs(q[:, 1]).max() - 1.0 / rms) < 1e-3
    assert int(xf[0, 4]) & oracle.NF_SIGN_TIE  # symmetric: the third moment vanishes


def test_circle_is_isotropic_and_constant_path(oracle_lib):
    out, xf = oracle.normalize_paths(np.stack([_ellipse(1.0, 1.0), np.ones((T, 2))]), oracle.NORM_PCA)
    assert int(xf[0, 4]) & oracle.NF_ISOTROPIC and xf[0, 3] in (0.0, math.pi)
    assert np.allclose(np.hypot(*out[0].T), 1.0)
    assert int(xf[1, 4]) == oracle.NF_CONSTANT and np.all(out[1] == 0)


def test_diameter_segment_and_box(oracle_lib):
    t = np.linspace(0, 1, T)
    seg = np.stack([2 + 3 * t, 1 - 4 * t], -1)      # length 5
    out, xf = oracle.normalize_paths(seg[None], oracle.NORM_DIAMETER)
    q = out[0]
    assert np.allclose(q[0], [0.0, 0.5]) and np.allclose(q[-1], [1.0, 0.5]) and abs(xf[0, 2] - 5) < 1e-12
    e = _sim(_ellipse(2.0, 0.5, ph=0.01), 0.3, 0.9, (4, 4))
    out, xf = oracle.normalize_paths(e[None], oracle.NORM_DIAMETER)
    q = out[0]
    # longest chord becomes the unit x extent, bounding box centred at (0.5, 0.5)
    assert abs(q[:, 0].max() - q[:, 0].min() - 1) < 1e-12
    assert abs((q[:, 0].max() + q[:, 0].min()) / 2 - 0.5) < 1e-12 and abs((q[:, 1].max() + q[:, 1].min()) / 2 - 0.5) < 1e-12
    assert abs((q[:, 1].max() - q[:, 1].min()) - 0.25) < 1e-3
    out2, _ = oracle.normalize_paths(_sim(e, 3.0, 2.0, (-1, 0))[None], oracle.NORM_DIAMETER)
    assert np.allclose(out2, out, atol=1e-10) or (int(xf[0, 4]) & oracle.NF_DIAM_TIE)
