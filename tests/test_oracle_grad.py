"""Pins of the oracle's alignment gradient: the forward-mode dual gradient of
L(theta) = sum_t chi2_t(A(h; theta)) (Section IV-B objective, summed) against
central finite differences of the value path, and against the invariances of
L under a global rigid motion (rotation about z, translation): the summed
gradient components along such a motion vanish."""
import numpy as np
import pytest

from oracle import oracle
from paper_2206_11535_amd import synth
from paper_2206_11535_amd.params import default_params

P = default_params()


@pytest.fixture(scope="module")
def setup():
    fs = synth.generate(5, n_frames=400)
    r = oracle.run(fs, P)
    tr = r.tracks[(r.tracks[:, 6] == 1) & (r.tracks[:, 7] == 0)]
    trip = np.concatenate([tr[:, [1, 2, 3]], tr[:, [2, 3, 4]]])
    return fs, trip


def test_dual_vs_central_differences(setup):
    fs, trip = setup
    S = synth.N_SENSORS
    theta = np.zeros((S, 4))
    L, g = oracle.align_loss_grad(fs, trip, theta, P)
    assert L > 0 and np.linalg.norm(g) > 0
    used = np.unique(fs.sensor[trip.ravel()])
    rng = np.random.default_rng(0)
    for s in rng.choice(used, 12, replace=False):
        for j in range(4):
            step = 1e-3 if j < 3 else 1e-3 / synth.R_LAYER[np.searchsorted(synth.SENSOR_BASE, s, "right") - 1]
            tp, tm = theta.copy(), theta.copy()
            tp[s, j] += step
            tm[s, j] -= step
            Lp, _ = oracle.align_loss_grad(fs, trip, tp, P, grad=False)
            Lm, _ = oracle.align_loss_grad(fs, trip, tm, P, grad=False)
            fd = (Lp - Lm) / (2 * step)
            assert abs(fd - g[s, j]) <= 1e-5 * max(abs(g[s, j]), 1e-3 * np.abs(g).max())


def test_global_motion_invariance(setup):
    fs, trip = setup
    S = synth.N_SENSORS
    _, g = oracle.align_loss_grad(fs, trip, np.zeros((S, 4)), P)
    scale = np.abs(g).sum(axis=0)
    # translations: sum of d/dt over sensors = derivative along a global shift
    for j in range(3):
        assert abs(g[:, j].sum()) < 1e-9 * scale[j]
    # rotation about z through the origin: d/dalpha per sensor is already the
    # derivative of the rotation of its hits about the origin
    assert abs(g[:, 3].sum()) < 1e-9 * scale[3]


def test_true_alignment_lowers_loss(setup):
    fs, trip = setup
    L0, _ = oracle.align_loss_grad(fs, trip, np.zeros((synth.N_SENSORS, 4)), P, grad=False)
    L1, _ = oracle.align_loss_grad(fs, trip, fs.align, P, grad=False)
    assert L1 < L0
