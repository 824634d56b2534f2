"""Test helpers: noiseless helices and hand-built frames.

Everything here is built from the generator (paper_2206_11535_amd.synth), never
from the oracle or the HIP path."""
from __future__ import annotations

import numpy as np

from paper_2206_11535_amd import synth


def helix_hits(vertex, mom, charge, ms=False, quant=False, accept=False, rng=None):
    """Hits of one or more particles on the four layers: returns an array
    [n_particles, 4, 3] (NaN where a layer is not reached)."""
    vertex = np.atleast_2d(np.asarray(vertex, float))
    mom = np.atleast_2d(np.asarray(mom, float))
    charge = np.atleast_1d(np.asarray(charge, float))
    rng = rng if rng is not None else np.random.default_rng(0)
    pid, lay, x, y, z = synth.propagate(rng, vertex, mom, charge, ms=ms, quant=quant, accept=accept)
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
