"""Pins of the oracle's refined vertex fit (the more precise vertex
reconstruction that Section VII names as the next step after the rough
estimate of Section IV-C).

The refined vertex of an e+e+e- triple minimises the weighted squared
distances to the three helices, jointly over the vertex and one turning
angle per track; the weights are eq. track-error's variances at the tracks'
points of closest approach to the rough estimate.

* noiseless decays: the helices meet at the true vertex, so the minimum is
  zero there -- this fixes the helix (turning direction, z slope, circle);
* a third track displaced from the common vertex by 50 um: near the vertex
  the helices are straight lines to within 1e-5 mm, and the minimiser of
  weighted squared distances to three lines has a closed form (a 3x3 linear
  system), with the weights computed here through the pinned closest-
  approach and variance functions -- this fixes the weights;
* scipy's trust-region least squares on the same residuals from the same
  start reaches the same minimum -- this fixes the solver;
* rotation about the beam axis and translation along it move the vertex
  with the hits;
* on decays with multiple scattering and pixel quantisation the refined
  vertex is closer to the truth than the rough estimate (what the refinement
  is for).
"""
import numpy as np
import pytest
from scipy.optimize import least_squares

from oracle import oracle
from paper_2206_11535_amd import synth
from paper_2206_11535_amd.params import default_params
from helpers import helix_hits

P = default_params()


def decays(n, seed, ms=False, quant=False, shift=0.0):
    """Signal decays (e+, e+, e- hits [n, 3, 4, 3]), their vertices, the
    production points and momenta; with shift > 0 the e- starts shift mm
    from the vertex, perpendicular to its momentum."""
    rng = np.random.default_rng(seed)
    mom = synth.sample_signal(rng, n)          # particles (e+, e-, e+)
    v = synth.sample_target(rng, n)
    H, V, A, M = [], [], [], []
    for k in range(n):
        start = np.repeat(v[k][None], 3, 0)
        if shift:
            t = mom[k, 1] / np.linalg.norm(mom[k, 1])
            u = np.cross(t, rng.normal(size=3))
            start[1] += shift * u / np.linalg.norm(u)
        h = helix_hits(start, mom[k], [1, -1, 1], ms=ms, quant=quant, accept=False, rng=rng)
        if np.all(np.isfinite(h)):
            order = [0, 2, 1]                  # e+, e+, e-
            H.append(h[order]); V.append(v[k]); A.append(start[order]); M.append(mom[k][order])
    return np.array(H), np.array(V), np.array(A), np.array(M)


def start_point(h, rough_xy):
    """Closest-approach turning angles and variances of the three tracks at
    the rough transverse vertex, through the pinned track functions."""
    g, ok = oracle.track_geom(h.reshape(-1, 4, 3), P)
    assert ok.all()
    c = np.stack([g["cx"], g["cy"]], 1)
    d = np.repeat(rough_xy[None], 3, 0) - c
    q = c + g["rt"][:, None] * d / np.linalg.norm(d, axis=1, keepdims=True)
    tp, ok = oracle.track_point(h.reshape(-1, 4, 3), q, P)
    assert ok.all()
    return tp[:, 0], tp[:, 2]


def test_noiseless_decays_exact():
    H, V, _, _ = decays(60, 21)
    assert len(H) > 20
    out, st = oracle.refine4(H, P)
    assert (st == 1).all()
    assert np.max(np.abs(out[:, :3] - V)) < 1e-9
    assert np.max(out[:, 3]) < 1e-18


def test_displaced_track_matches_weighted_lines():
    H, V, A, M = decays(40, 22, shift=0.05)
    out, st = oracle.refine4(H, P)
    assert (st == 1).sum() > 15
    n_checked = 0
    spread = []
    for i in np.nonzero(st == 1)[0]:
        _, s2 = start_point(H[i], out[i, 10:12])
        w = 1.0 / s2
        S = np.zeros((3, 3))
        b = np.zeros(3)
        for k in range(3):
            t = M[i, k] / np.linalg.norm(M[i, k])
            Q = np.eye(3) - np.outer(t, t)
            S += w[k] * Q
            b += w[k] * Q @ A[i, k]
        v_lines = np.linalg.solve(S, b)
        assert np.linalg.norm(out[i, :3] - v_lines) < 2e-4, (i, out[i, :3], v_lines)
        # the weights matter here: equal weights move the vertex by much more
        S1 = sum(np.eye(3) - np.outer(m, m) / (m @ m) for m in M[i])
        b1 = sum((np.eye(3) - np.outer(m, m) / (m @ m)) @ a for m, a in zip(M[i], A[i]))
        spread.append(np.linalg.norm(np.linalg.solve(S1, b1) - v_lines))
        n_checked += 1
    assert n_checked > 15
    assert np.median(spread) > 5e-3


def test_independent_solver_same_minimum():
    H, V, _, _ = decays(40, 23, ms=True, quant=True)
    out, st = oracle.refine4(H, P)
    idx = np.nonzero(st == 1)[0]
    assert len(idx) > 20
    for i in idx[:25]:
        phi, s2 = start_point(H[i], out[i, 10:12])
        x0 = np.concatenate([out[i, 10:13], phi])

        def fun(x):
            return oracle.refine_residual(H[i][None], x[None], s2[None], P)[0]

        r = least_squares(fun, x0, method="trf", jac="3-point", xtol=1e-15, ftol=1e-15, gtol=1e-15,
                          max_nfev=5000)
        assert np.max(np.abs(r.x[:3] - out[i, :3])) < 1e-7, (i, r.x, out[i, :7])
        assert np.max(np.abs(r.x[3:] - out[i, 4:7])) < 1e-8
        assert abs(2 * r.cost - out[i, 3]) <= 1e-9 * max(out[i, 3], 1.0)


def test_rotation_and_translation():
    H, V, _, _ = decays(30, 24, ms=True, quant=True)
    out, st = oracle.refine4(H, P)
    a = 0.7
    R = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
    Hr = H @ R.T
    Hz = H + np.array([0.0, 0.0, 3.25])
    outr, str_ = oracle.refine4(Hr, P)
    outz, stz = oracle.refine4(Hz, P)
    ok = (st == 1) & (str_ == 1) & (stz == 1)
    assert ok.sum() > 15
    assert np.max(np.abs(outr[ok, :3] - out[ok, :3] @ R.T)) < 1e-7
    assert np.max(np.abs(outz[ok, :3] - out[ok, :3] - [0, 0, 3.25])) < 1e-7
    assert np.max(np.abs(outr[ok, 3] - out[ok, 3]) / (1 + out[ok, 3])) < 1e-7


def test_refined_vertex_closer_to_truth():
    H, V, _, _ = decays(400, 25, ms=True, quant=True)
    out, st = oracle.refine4(H, P)
    ok = st == 1
    assert ok.sum() > 150
    assert (st[~ok] == 0).all()                 # only triples whose rough estimate fails are left out
    e_ref = np.linalg.norm(out[ok, :3] - V[ok], axis=1)
    e_rough = np.linalg.norm(out[ok, 10:13] - V[ok], axis=1)
    assert np.median(e_ref) < 0.8 * np.median(e_rough)
    # the rough estimate with its closest-approach points is the start, and
    # its chi2 is the objective there: the minimum is never above it
    assert (out[ok, 3] <= out[ok, 13] * (1 + 1e-12) + 1e-15).all()


@pytest.mark.parametrize("kind", ["no_rough_vertex", "bad_track"])
def test_refine_status(kind):
    H, V, _, _ = decays(10, 26)
    h = H[:1].copy()
    if kind == "no_rough_vertex":
        h[0, 2, :, :2] = -h[0, 2, :, :2]        # e- track turned by pi: the circles no longer meet at the target
        want = 0
    else:
        h[0, 0, 1] = h[0, 0, 0]                  # two equal hits: the triplet fit fails
        want = -2
    out, st = oracle.refine4(h, P)
    assert st[0] == want
    assert np.isnan(out[0, :4]).all()
