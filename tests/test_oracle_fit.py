"""Pins of the oracle's triplet fit (Section IV-B, eq. objective-function and
the linearisation around the transverse circle), the layer-3 extension and the
two-triplet track (eq. objective-function-global, weighted mean curvature).

* noiseless helices: R* = R_true exactly, chi2 = 0, correct charge sign,
  exact layer-3 prediction;
* an exact nonlinear minimiser of the same chi2 model (root-finding per arc,
  bounded minimisation) agrees to second order in the kink: halving the kink
  quarters the difference, which fails for any first-order mistake in the
  expansion coefficients or in the minimisation algebra;
* pulls on multiple-scattering-only samples follow N(0, 1) and chi2 ~ chi2(1);
* symmetries: rotation, z translation, mirror (charge flip).
"""
import numpy as np
import pytest
from scipy import optimize

from oracle import oracle
from paper_2206_11535_amd import synth
from paper_2206_11535_amd.params import default_params
from helpers import helix_hits, momentum

P = default_params()
KC = 0.299792458


def noiseless(p, theta, phi, q, vertex=(2.0, -3.0, 5.0)):
    return helix_hits([vertex], [momentum(p, theta, phi)], [q])[0]


@pytest.mark.parametrize("p,theta,phi,q", [(30.0, 1.2, 0.4, 1), (45.0, 2.0, -1.0, -1),
                                             (15.0, 1.57079, 2.5, 1), (52.0, 0.9, -2.9, -1)])
def test_noiseless_helix_exact(p, theta, phi, q):
    h = noiseless(p, theta, phi, q)
    f, ok = oracle.fit(h[None, :3], P)
    assert ok[0]
    R_true = p / (KC * P["b_tesla"])
    assert abs(f["r_star"][0] - R_true) < 1e-9 * R_true
    assert f["chi2"][0] < 1e-16
    assert np.sign(f["kappa"][0]) == q
    assert abs(f["theta1"][0] - theta) < 1e-10 and abs(f["theta2"][0] - theta) < 1e-10
    assert abs(abs(f["rtc"][0]) - p * np.sin(theta) / KC) < 1e-9 * R_true
    # second triplet of the same helix and the combined track
    f2, ok2 = oracle.fit(h[None, 1:4], P)
    assert ok2[0] and abs(f2["r_star"][0] - R_true) < 1e-9 * R_true
    t, tok = oracle.track4(h[None], P)
    assert tok[0] and abs(t[0, 0] - q / R_true) < 1e-12 and t[0, 1] < 1e-16


@pytest.mark.parametrize("p,theta,phi,q", [(30.0, 1.2, 0.4, 1), (45.0, 2.0, -1.0, -1), (22.0, 1.0, 3.0, 1)])
def test_noiseless_layer3_prediction(p, theta, phi, q):
    h = noiseless(p, theta, phi, q)
    pr, ok = oracle.predict_l3(h[None, :3], P)
    assert ok[0]
    assert np.max(np.abs(pr[0] - h[3])) < 1e-9


def exact_fit(h, sigma, sn2):
    """Exact minimum of chi2(R) = (sin^2(theta) Phi_MS(R)^2 + Theta_MS(R)^2) / sigma^2
    where, for each arc, Phi_k(R) solves R^2 = d^2/(4 sin^2(Phi/2)) + z^2/Phi^2
    exactly (no expansion); Phi_MS = -(1/2) sum_k (Phi_k(R) - Phi_k(circle)),
    Theta_MS = theta_2(R) - theta_1(R) with cos(theta_k) = z_k / (R Phi_k)."""
    d = [np.hypot(*(h[1, :2] - h[0, :2])), np.hypot(*(h[2, :2] - h[1, :2]))]
    z = [h[1, 2] - h[0, 2], h[2, 2] - h[1, 2]]
    # circle solution: transverse circumradius of the three points
    a, b, c = d[0], d[1], np.hypot(*(h[2, :2] - h[0, :2]))
    s = (a + b + c) / 2
    rho = a * b * c / (4 * np.sqrt(s * (s - a) * (s - b) * (s - c)))
    phic = [2 * np.arcsin(dk / (2 * rho)) for dk in d]

    def arc(k, R):
        g = lambda ph: d[k] ** 2 / (4 * np.sin(ph / 2) ** 2) + z[k] ** 2 / ph ** 2 - R * R
        ph = optimize.brentq(g, 1e-9, np.pi, xtol=1e-15, rtol=1e-15, maxiter=500)
        return ph, np.arccos(z[k] / (R * ph))

    def chi2(R):
        (p1, t1), (p2, t2) = arc(0, R), arc(1, R)
        phims = -0.5 * ((p1 - phic[0]) + (p2 - phic[1]))
        return (sn2 * phims ** 2 + (t2 - t1) ** 2) / sigma ** 2

    Rc = [np.hypot(rho, z[k] / phic[k]) for k in range(2)]
    lo = max(max(np.hypot(d[k] / 2, z[k] / np.pi) for k in range(2)) * 1.0001, 0.7 * min(Rc))
    res = optimize.minimize_scalar(chi2, bounds=(lo, 1.4 * max(Rc)), method="bounded",
                                   options={"xatol": 1e-11 * max(Rc)})
    return res.x, res.fun


def test_linearisation_is_second_order():
    """Kinked triplets: |R*_lin - R*_exact| scales with the square of the kink."""
    base = noiseless(30.0, 1.25, 0.3, 1)[:3]
    errs = []
    for eps in (0.1, 0.05, 0.025):
        h = base.copy()
        # move the middle hit along z and along the layer (kinks in both planes)
        h[1, 2] += eps
        phi1 = np.arctan2(h[1, 1], h[1, 0]) + eps / 31.0
        h[1, 0], h[1, 1] = 31.0 * np.cos(phi1), 31.0 * np.sin(phi1)
        f, ok = oracle.fit(h[None], P)
        assert ok[0]
        sn2 = np.sin(0.5 * (f["theta1"][0] + f["theta2"][0])) ** 2
        Rx, cx = exact_fit(h, f["sigma_ms"][0], sn2)
        errs.append((abs(f["r_star"][0] - Rx) / Rx, f["chi2"][0], cx))
    e = [x[0] for x in errs]
    assert e[0] < 1e-6
    # ratios tend to 4 (a first-order mistake gives 2); the cubic term still
    # shows at the largest kink
    assert 3.5 < e[0] / e[1] < 6.5 and 3.5 < e[1] / e[2] < 5.5
    # chi2 agrees to relative order kink
    rel = [abs(x[1] - x[2]) / x[2] for x in errs]
    assert rel[0] < 1e-5 and 1.6 < rel[0] / rel[1] < 2.6 and 1.6 < rel[1] / rel[2] < 2.6


def test_pulls_ms_only():
    """Multiple scattering only (no pixel quantisation): pulls of R* are
    N(0,1)-like and chi2_min averages to one degree of freedom."""
    rng = np.random.default_rng(5)
    n = 6000
    v = synth.sample_target(rng, n)
    p = rng.uniform(20, 50, n)
    th = np.arccos(rng.uniform(-0.6, 0.6, n))
    ph = rng.uniform(-np.pi, np.pi, n)
    mom = np.stack([p * np.sin(th) * np.cos(ph), p * np.sin(th) * np.sin(ph), p * np.cos(th)], 1)
    q = np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    h = helix_hits(v, mom, q, ms=True, quant=False, accept=False, rng=rng)
    good = np.all(np.isfinite(h[:, :3, 0]), axis=1)
    f, ok = oracle.fit(h[good, :3], P)
    Rt = p[good] / KC
    pull = (f["r_star"][ok] - Rt[ok]) / np.sqrt(f["sigma2_r"][ok])
    assert abs(np.median(pull)) < 0.1
    assert 0.8 < np.std(np.clip(pull, -6, 6)) < 1.25
    assert 0.8 < np.mean(f["chi2"][ok]) < 1.3
    assert np.all(np.sign(f["kappa"][ok]) == q[good][ok])


def test_fit_symmetries():
    rng = np.random.default_rng(6)
    hs = []
    for _ in range(50):
        hh = helix_hits(synth.sample_target(rng, 1), [momentum(rng.uniform(20, 50), rng.uniform(0.9, 2.2),
                                                               rng.uniform(-3, 3))], [1], ms=True, rng=rng)[0]
        if np.all(np.isfinite(hh[:3])):
            hs.append(hh[:3])
    h = np.array(hs)
    f, _ = oracle.fit(h, P)
    a = -1.1
    r = h.copy()
    r[..., 0] = np.cos(a) * h[..., 0] - np.sin(a) * h[..., 1]
    r[..., 1] = np.sin(a) * h[..., 0] + np.cos(a) * h[..., 1]
    r[..., 2] += 7.5
    fr, _ = oracle.fit(r, P)
    for k in ("kappa", "chi2", "r_star", "sigma2_kappa"):
        assert np.allclose(fr[k], f[k], rtol=1e-8, atol=1e-12)
    m = h.copy()
    m[..., 1] *= -1
    fm, _ = oracle.fit(m, P)
    assert np.allclose(fm["kappa"], -f["kappa"], rtol=1e-10)
    assert np.allclose(fm["chi2"], f["chi2"], rtol=1e-8, atol=1e-12)
