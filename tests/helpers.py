"""Test helpers: noiseless helices and hand-built frames.

Everything here is built from the generator (paper_2206_11535_amd.synth), never
from the oracle or the HIP path."""
from __future__ import annotations

import numpy as np

from paper_2206_11535_amd import synth


def helix_hits(vertex, mom, charge, ms=False, quant=False, accept=False, rng=None, ms_layers=(0, 1, 2, 3)):
    """Hits of one or more particles on the four layers: returns an array
    [n_particles, 4, 3] (NaN where a layer is not reached)."""
    vertex = np.atleast_2d(np.asarray(vertex, float))
    mom = np.atleast_2d(np.asarray(mom, float))
    charge = np.atleast_1d(np.asarray(charge, float))
    rng = rng if rng is not None else np.random.default_rng(0)
    pid, lay, x, y, z = synth.propagate(rng, vertex, mom, charge, ms=ms, quant=quant, accept=accept,
                                        ms_layers=ms_layers)
    out = np.full((len(charge), 4, 3), np.nan)
    out[pid, lay, 0] = x
    out[pid, lay, 1] = y
    out[pid, lay, 2] = z
    return out


def momentum(p, theta, phi):
    return np.array([p * np.sin(theta) * np.cos(phi), p * np.sin(theta) * np.sin(phi), p * np.cos(theta)])


class Frames:
    """Minimal frame container built from per-frame lists of per-layer hits."""

    def __init__(self, frames):
        xs, ys, zs, lay, lo = [], [], [], [], [0]
        for fr in frames:
            for l in range(4):
                pts = np.asarray(fr[l], float).reshape(-1, 3)
                xs.append(pts[:, 0]); ys.append(pts[:, 1]); zs.append(pts[:, 2])
                lay.append(np.full(len(pts), l))
                lo.append(lo[-1] + len(pts))
        self.x = np.concatenate(xs).astype(np.float32)
        self.y = np.concatenate(ys).astype(np.float32)
        self.z = np.concatenate(zs).astype(np.float32)
        self.layer = np.concatenate(lay).astype(np.uint16)
        self.sensor = synth.sensor_of(self.layer.astype(np.int64), self.x, self.y, self.z).astype(np.uint16)
        self.layer_offsets = np.asarray(lo, np.int32)

    @property
    def n_frames(self):
        return (len(self.layer_offsets) - 1) // 4

    @property
    def n_hits(self):
        return len(self.x)


def frame_from_particles(hits):
    """hits [n, 4, 3] -> one frame (list per layer), skipping NaN layers."""
    fr = [[], [], [], []]
    for p in hits:
        for l in range(4):
            if np.all(np.isfinite(p[l])):
                fr[l].append(p[l])
    return fr


C_LIGHT = 0.299792458


def true_circle(vertex, mom, charge):
    """Transverse circle of a helix from the generator's conventions
    (synth.propagate): centre on the right of the motion for positive
    charge, radius p_t / (0.2998 B).  Returns (centre [2], radius)."""
    pt = np.hypot(mom[0], mom[1])
    rho = pt / (C_LIGHT * synth.B_TESLA)
    ux, uy = mom[0] / pt, mom[1] / pt
    return np.array([vertex[0] + charge * rho * uy, vertex[1] - charge * rho * ux]), rho


def point_behind(centre, rho, charge, h0, alpha):
    """Point of the circle reached from h0 by travelling backwards through
    the turning angle alpha (forward motion turns the position angle by
    -charge per radian, as the generator propagates)."""
    psi = np.arctan2(h0[1] - centre[1], h0[0] - centre[0]) + charge * alpha
    return centre + rho * np.array([np.cos(psi), np.sin(psi)])


def angle_behind(centre, charge, h0, q):
    """Inverse of point_behind: the backward turning angle in [0, 2 pi)
    from h0 to the circle point q."""
    a = np.arctan2(q[1] - centre[1], q[0] - centre[0]) - np.arctan2(h0[1] - centre[1], h0[0] - centre[0])
    return np.mod(charge * a, 2 * np.pi)


def circle_intersections(ca, ra, cb, rb, n=20001):
    """Intersections of two circles by bracketing the sign changes of
    |a(t) - cb| - rb along circle a and refining each with Brent's method
    (a route independent of the closed-form intersection)."""
    from scipy import optimize
    t = np.linspace(-np.pi, np.pi, n)
    g = lambda u: np.hypot(ca[0] + ra * np.cos(u) - cb[0], ca[1] + ra * np.sin(u) - cb[1]) - rb
    gv = g(t)
    out = []
    for i in np.nonzero(np.sign(gv[:-1]) * np.sign(gv[1:]) < 0)[0]:
        r = optimize.brentq(g, t[i], t[i + 1], xtol=1e-15, rtol=1e-15)
        out.append(ca + ra * np.array([np.cos(r), np.sin(r)]))
    return out


def merge_pairs(fs):
    """Host construction of the overlapping frame pairs (the plain
    definition the GPU's k_pairs must reproduce): merged frame g holds, per
    layer, the hits of frame g and then those of frame g + 1.  Returns
    (x, y, z, layer_offsets, orig) with orig[i] the input index of merged
    hit i."""
    lo = np.asarray(fs.layer_offsets, np.int64)
    F = (len(lo) - 1) // 4
    idx, off = [], [0]
    for g in range(F - 1):
        for l in range(4):
            a = np.arange(lo[4 * g + l], lo[4 * g + l + 1])
            b = np.arange(lo[4 * g + 4 + l], lo[4 * g + 5 + l])
            idx.append(a)
            idx.append(b)
            off.append(off[-1] + len(a) + len(b))
    orig = np.concatenate(idx) if idx else np.zeros(0, np.int64)
    return (fs.x[orig], fs.y[orig], fs.z[orig], np.asarray(off, np.int32), orig)
