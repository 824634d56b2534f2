"""The seeded generator: layout, geometry and physics distributions."""
import numpy as np
import pytest
from scipy import stats

from paper_2206_11535_amd import synth


@pytest.fixture(scope="module")
def cfg2():
    return synth.generate(2, n_frames=3000)


def test_layout_sorted_and_offsets(cfg2):
    fs = cfg2
    lo = fs.layer_offsets
    assert lo.dtype == np.int32 and len(lo) == 4 * fs.n_frames + 1
    assert lo[0] == 0 and lo[-1] == fs.n_hits and np.all(np.diff(lo) >= 0)
    seg = np.repeat(np.arange(4 * fs.n_frames), np.diff(lo))
    assert np.array_equal(seg % 4, fs.layer.astype(np.int64))
    for a in (fs.x, fs.y, fs.z):
        assert a.dtype == np.float32
    assert fs.layer.dtype == np.uint16 and fs.sensor.dtype == np.uint16
    assert fs.sensor.max() < synth.N_SENSORS


def test_hits_on_cylinders_within_acceptance(cfg2):
    fs = cfg2
    r = np.hypot(fs.x.astype(np.float64), fs.y)
    R = synth.R_LAYER[fs.layer]
    assert np.max(np.abs(r - R)) < 1e-4
    assert np.all(np.abs(fs.z) <= synth.Z_HALF[fs.layer] + 1e-6)
    # pixel centres in z: (k + 1/2) * 80 um
    k = fs.z.astype(np.float64) / synth.PIXEL - 0.5
    assert np.max(np.abs(k - np.round(k))) < 1e-3


def test_noise_count_and_rate(cfg2):
    fs = cfg2
    assert np.all(np.bincount(np.repeat(np.arange(4 * fs.n_frames), np.diff(fs.layer_offsets))[fs.pid < 0],
                              minlength=4 * fs.n_frames) == 5)
    lam = fs.particles["lam"]
    assert np.allclose(lam, 6.4)


def test_michel_spectrum():
    rng = np.random.default_rng(1)
    p = synth.sample_michel(rng, 200000)
    assert p.min() >= synth.P_MICHEL_MIN and p.max() <= synth.P_MICHEL_MAX
    a = synth.P_MICHEL_MIN / synth.P_MICHEL_MAX

    def cdf(pp):
        x = pp / synth.P_MICHEL_MAX
        F = lambda u: u ** 3 - u ** 4 / 2    # integral of x^2 (3 - 2x) / 3 ... up to a constant
        return (F(x) - F(a)) / (F(1.0) - F(a))
    assert stats.kstest(p, cdf).pvalue > 1e-3


def test_target_surface():
    rng = np.random.default_rng(2)
    v = synth.sample_target(rng, 100000)
    r = np.hypot(v[:, 0], v[:, 1])
    assert np.allclose(r, synth.TARGET_R * (1 - np.abs(v[:, 2]) / synth.TARGET_HALF))
    # |z| density proportional to r(|z|): mean |z| = L/3
    assert abs(np.mean(np.abs(v[:, 2])) - synth.TARGET_HALF / 3) < 0.3


def test_signal_kinematics():
    rng = np.random.default_rng(3)
    mom = synth.sample_signal(rng, 5000)
    assert np.max(np.abs(mom.sum(axis=1))) < 1e-9
    E = np.sqrt(np.sum(mom ** 2, axis=2) + synth.M_E ** 2).sum(axis=1)
    assert np.max(np.abs(E - synth.M_MU)) < 1e-9


def test_helix_radius_and_sign():
    """Noiseless propagation: hits lie on the transverse circle of radius
    p_t / (c B), positive charges turn clockwise."""
    from helpers import helix_hits, momentum
    p, th, ph = 30.0, 1.2, 0.4
    for q in (1, -1):
        h = helix_hits([[0.0, 0.0, 0.0]], [momentum(p, th, ph)], [q])[0]
        rho = p * np.sin(th) / (synth.C_LIGHT * synth.B_TESLA)
        # centre on the right of the initial direction for q > 0
        u = np.array([np.cos(ph), np.sin(ph)])
        c = q * rho * np.array([u[1], -u[0]])
        d = np.hypot(h[:, 0] - c[0], h[:, 1] - c[1])
        assert np.allclose(d, rho, rtol=1e-12)
        ang = np.arctan2(h[:, 1] - c[1], h[:, 0] - c[0])
        step = np.diff(np.unwrap(ang))
        assert np.all(q * step < 0)           # clockwise for q = +1


def test_deterministic():
    a = synth.generate(1, n_frames=200)
    b = synth.generate(1, n_frames=200)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.layer_offsets, b.layer_offsets)
    c = synth.generate(1, n_frames=200, salt=7)
    assert not np.array_equal(a.x[:50], c.x[:50])


def test_misalignment_applied():
    fs = synth.generate(5, n_frames=300)
    assert fs.align is not None and fs.align.shape == (synth.N_SENSORS, 4)
    assert abs(np.std(fs.align[:, :3]) - 0.05) < 0.005
    # re-aligning with the true parameters puts hits back on the cylinders
    s = fs.sensor.astype(np.int64)
    t, a = fs.align[s, :3], fs.align[s, 3]
    x = np.cos(a) * fs.x - np.sin(a) * fs.y + t[:, 0]
    y = np.sin(a) * fs.x + np.cos(a) * fs.y + t[:, 1]
    R = synth.R_LAYER[fs.layer]
    assert np.max(np.abs(np.hypot(x, y) - R)) < 1e-3
    assert np.max(np.abs(np.hypot(fs.x, fs.y) - R)) > 1e-2
