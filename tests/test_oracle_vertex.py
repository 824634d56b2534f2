"""Pins of the oracle's vertex stage (Section IV-C) and frame flags (Section
V-B, Algs. 1-4).

* noiseless signal decays: the three track circles meet at the true vertex;
  the estimate recovers it, chi2 ~ 0, sum E = m_mu, sum p = 0 -- this fixes
  the circle centres' side, the backward turning angle, the z back-projection
  and the momentum directions;
* generated signal decays with scattering: recovery near the truth;
* hand-built frames for every flag and for the caps (count > cap).
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle
from paper_2206_11535_amd import synth
from paper_2206_11535_amd.params import default_params
from helpers import Frames, frame_from_particles, helix_hits

P = default_params()
M_MU = 105.6583755


def signal_hits(n, seed, ms=False, quant=False):
    rng = np.random.default_rng(seed)
    mom = synth.sample_signal(rng, n)
    v = synth.sample_target(rng, n)
    out = []
    for k in range(n):
        h = helix_hits(np.repeat(v[k][None], 3, 0), mom[k], [1, -1, 1], ms=ms, quant=quant,
                       accept=False, rng=rng)
        if np.all(np.isfinite(h)):
            out.append((h, v[k], mom[k]))
    return out


def test_noiseless_signal_vertex_recovered():
    dec = signal_hits(60, 11)
    assert len(dec) > 10
    for h, v, mom in dec:
        hv = h[[0, 2, 1]]                   # e+, e+, e-
        o = oracle.vertex4(hv[None], P)[0]
        assert o[0] == 1 and o[9] == 1
        assert np.max(np.abs(o[1:4] - v)) < 1e-7
        assert o[4] < 1e-12
        assert abs(o[5] - M_MU) < 1e-9
        assert o[8] < 1e-8                  # |sum p|
        assert o[7] < 1e-7                  # on the target surface


def test_noiseless_signal_vertex_invariant_under_mirror():
    """Mirror y -> -y swaps the charge of every track: the vertex mirrors,
    with e- as the odd one out it is no longer an e+e+e- triple (fails to
    meet the kinematics only through sign conventions if they are wrong)."""
    h, v, mom = signal_hits(20, 12)[0]
    m = h.copy()
    m[..., 1] *= -1
    t, ok = oracle.track4(m.reshape(-1, 4, 3), P)
    assert ok.all() and list(np.sign(t[:, 0])) == [-1, 1, -1]


def test_signal_with_scattering_near_truth():
    dec = signal_hits(300, 13, ms=True, quant=True)
    hv = np.array([h[[0, 2, 1]] for h, _, _ in dec])
    tv = np.array([v for _, v, _ in dec])
    o = oracle.vertex4(hv, P)
    found = o[:, 0] == 1
    assert found.mean() > 0.7
    d = np.linalg.norm(o[found, 1:4] - tv[found], axis=1)
    assert np.median(d) < 1.0


def test_cone_distance_and_nonintersecting():
    # two e+ on the same circle side far from the e-: built from noiseless
    # tracks of different decays -> circles do not meet near the target
    a = signal_hits(10, 14)
    b = signal_hits(10, 15)
    hv = np.array([[a[0][0][0], a[0][0][2], b[0][0][1]]])
    o = oracle.vertex4(hv, P)
    assert o[0, 0] == 0


def frame_with(hits_list):
    return Frames([frame_from_particles(np.concatenate(hits_list, 0))])


@pytest.fixture(scope="module")
def signal_frame():
    h, v, mom = signal_hits(40, 16)[0]
    return frame_with([h]), v


def test_frame_vertex_flag(signal_frame):
    fs, v = signal_frame
    r = oracle.run(fs, P)
    assert r.flags[0] == oracle.VERTEX | oracle.KEEP
    assert r.counts[0].tolist() == [3, 3, 1]
    assert np.max(np.abs(r.vertex[0, :3] - v)) < 1e-3       # float32 hits


@pytest.mark.parametrize("cap,field,flag", [("max_triplets", 0, oracle.TRIPLET_OVF),
                                            ("max_tracks", 1, oracle.TRACK_OVF),
                                            ("max_combos", 2, oracle.COMBO_OVF)])
def test_caps_mark_for_storage(signal_frame, cap, field, flag):
    fs, _ = signal_frame
    n = [3, 3, 1][field]
    r = oracle.run(fs, default_params(**{cap: n - 1}))
    assert r.flags[0] == flag | oracle.KEEP
    assert r.counts[0, field] == n
    assert np.all(r.counts[0, field + 1:] == 0)
    r = oracle.run(fs, default_params(**{cap: n}))      # count == cap is no overflow
    assert r.flags[0] == oracle.VERTEX | oracle.KEEP


def test_hits_overflow(signal_frame):
    fs, _ = signal_frame
    r = oracle.run(fs, default_params(max_layer_hits=2))
    assert r.flags[0] == oracle.HITS_OVF | oracle.KEEP


def test_empty_and_degenerate_frames():
    fs = Frames([[[], [], [], []], [[(25.0, 0, 0)], [], [(73.0, 0, 0)], []],
                 [[(25.0, 0, 0)], [(31.0, 0, 0)], [(73.0, 0, 0)], [(85.0, 0, 0)]]])
    r = oracle.run(fs, P)
    assert np.all(r.flags == 0) and np.all(r.counts == 0)
    assert np.all(np.isnan(r.vertex))


def test_michel_only_frames_rarely_kept():
    fs = synth.generate(dataclasses.replace(synth.CONFIGS[2], signal_frac=0.0), n_frames=2000, salt=3)
    r = oracle.run(fs, P, lists=False)
    assert np.mean(r.flags & oracle.KEEP > 0) < 0.02
