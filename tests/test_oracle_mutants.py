"""Mutation check of the oracle's pins: every plausible mistake listed below
is planted in a copy of oracle/mu3e_oracle.cpp (on the CPU, never in the
product), the copy is compiled, and the oracle pin tests are run against it
through MU3E_ORACLE_LIB.  Each mutant must make at least one pin fail; the
unmutated copy, built the same way, must pass them all.

The mistakes are the kind a reader of the paper could make: a sign, a
swapped operand, a dropped term, a wrong weight, 3D instead of transverse,
the wrong trigonometric function, an off-by-one in a cap.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mu3e_oracle.cpp")
PIN_FILES = ["test_oracle_cuts.py", "test_oracle_fit.py", "test_oracle_track.py", "test_oracle_vertex.py",
             "test_oracle_vertex_model.py", "test_oracle_grad.py", "test_oracle_refine.py"]

# name -> [(original text, planted text), ...]; every original occurs once.
MUTANTS = {
    # Selection Cuts (Section IV-A)
    "dlambda_sign": [("q.dlambda = tl12 - tl01;", "q.dlambda = tl01 - tl12;")],
    "dlambda_slope_radii": [("double tl01 = (h1[2] - h0[2]) / (R1 - R0);",
                             "double tl01 = (h1[2] - h0[2]) / (R2 - R0);")],
    "rtc_chord_3d": [("double d01 = std::hypot(h0[0] - h1[0], h0[1] - h1[1]);",
                      "double d01 = std::sqrt((h0[0] - h1[0]) * (h0[0] - h1[0]) + (h0[1] - h1[1]) * "
                      "(h0[1] - h1[1]) + (h0[2] - h1[2]) * (h0[2] - h1[2]));")],
    "rtc_factor_two": [(": d01 * d12 * d20 / (2.0 * cross);", ": d01 * d12 * d20 / cross;")],
    "cap_at_equal": [("if (lo_cnt > P.max_triplets)", "if (lo_cnt >= P.max_triplets)")],
    # Single triplet fit (Section IV-B)
    "fit_sin_is_cos": [("T sn = sin(thbar);", "T sn = cos(thbar);")],
    "fit_chi2_without_sin2": [("o.chi2 = s2 * num * num / (den * sms * sms);",
                               "o.chi2 = num * num / (den * sms * sms);")],
    "fit_highland_log_sign": [("T sms = 13.6 / p * sqrt(X) * (1.0 + 0.038 * log(X));",
                               "T sms = 13.6 / p * sqrt(X) * (1.0 - 0.038 * log(X));")],
    "fit_sigma_r_without_ms": [("o.sigma2_r = sms * sms / den;", "o.sigma2_r = 1.0 / den;")],
    "l3_slope_of_arc1": [("out[2] = h2[2] + best * (h2[2] - h1[2]) / f.phi2;",
                          "out[2] = h2[2] + best * (h2[2] - h1[2]) / f.phi1;")],
    "l3_backwards": [("double dphi = (f.sgn > 0) ? psi_2 - psi_p : psi_p - psi_2;",
                      "double dphi = (f.sgn > 0) ? psi_p - psi_2 : psi_2 - psi_p;")],
    # Two-triplet track (Section IV-B, Triplets Fit)
    "kbar_inverse_weights": [("double w1 = 1 / f1.sigma2_kappa, w2 = 1 / f2.sigma2_kappa;",
                              "double w1 = f1.sigma2_kappa, w2 = f2.sigma2_kappa;")],
    "kbar_equal_weights": [("double w1 = 1 / f1.sigma2_kappa, w2 = 1 / f2.sigma2_kappa;",
                            "double w1 = 1, w2 = 1;")],
    "chi2g_without_curvature_terms": [
        ("chi2 = f1.chi2 + (rbar - f1.r_star)", "chi2 = f1.chi2 + 0.0 * (rbar - f1.r_star)"),
        ("+ f2.chi2 + (rbar - f2.r_star)", "+ f2.chi2 + 0.0 * (rbar - f2.r_star)")],
    "chi2g_sigma_not_squared": [
        ("* (rbar - f1.r_star) / f1.sigma2_r", "* (rbar - f1.r_star) / std::sqrt(f1.sigma2_r)"),
        ("* (rbar - f2.r_star) / f2.sigma2_r;", "* (rbar - f2.r_star) / std::sqrt(f2.sigma2_r);")],
    # Vertex stage (Section IV-C)
    "circle_radius_3d": [("double rt = t.rbar * std::sin(t.theta1);", "double rt = t.rbar;")],
    "circle_wrong_side": [("double sg = t.charge > 0 ? 1.0 : -1.0;", "double sg = t.charge > 0 ? -1.0 : 1.0;")],
    "energy_without_mass": [("t.E = std::sqrt(t.p * t.p + kMe * kMe);", "t.E = t.p;")],
    "sms0_without_path_factor": [("t.sms0 = highland(t.p, P.xx0 / std::sin(t.theta1));",
                                  "t.sms0 = highland(t.p, P.xx0);")],
    "back_angle_forward": [("double d = (t.charge > 0) ? ps_q - ps_0 : ps_0 - ps_q;",
                            "double d = (t.charge > 0) ? ps_0 - ps_q : ps_q - ps_0;")],
    "path_with_3d_radius": [("double s = t.rt * back_angle(t, qx, qy);",
                             "double s = t.rbar * back_angle(t, qx, qy);")],
    "pixel_sigma_unsquared": [("return t.sms0 * t.sms0 * s * s + P.sigma_pix * P.sigma_pix;",
                               "return t.sms0 * t.sms0 * s * s + P.sigma_pix;")],
    "path_not_squared": [("return t.sms0 * t.sms0 * s * s + P.sigma_pix * P.sigma_pix;",
                          "return t.sms0 * t.sms0 * s + P.sigma_pix * P.sigma_pix;")],
    "cone_apex": [("bz = s * 50.0;", "bz = s * 40.0;")],
    "target_without_tolerance": [("if (rq <= lim)", "if (rq <= P.r_target)")],
    "intersection_sigma_one_track": [
        ("double s2 = 0.5 * (point_sigma2(*T[pr[k][0]], qx, qy, P) + point_sigma2(*T[pr[k][1]], qx, qy, P));",
         "double s2 = point_sigma2(*T[pr[k][0]], qx, qy, P);")],
    "mu_t_unweighted": [("sw += 1 / s2; mx += qx / s2; my += qy / s2;", "sw += 1; mx += qx; my += qy;")],
    "mu_t_inverse_weights": [("sw += 1 / s2; mx += qx / s2; my += qy / s2;",
                              "sw += s2; mx += qx * s2; my += qy * s2;")],
    "pca_is_the_mean": [("cax[k] = t.cx + t.rt * vx / vn;", "cax[k] = mx;"),
                        ("cay[k] = t.cy + t.rt * vy / vn;", "cay[k] = my;")],
    "z_with_sin": [("zz[k] = t.h0[2] - dphi * t.rbar * std::cos(t.theta1);",
                    "zz[k] = t.h0[2] - dphi * t.rbar * std::sin(t.theta1);")],
    "mu_z_unweighted": [("wz += 1 / sg2[k]; mz += zz[k] / sg2[k];", "wz += 1; mz += zz[k];")],
    "chi2v_sigma_not_squared": [("chi2 += (dx * dx + dy * dy + dz * dz) / sg2[k];",
                                 "chi2 += (dx * dx + dy * dy + dz * dz) / std::sqrt(sg2[k]);")],
    "chi2v_without_z": [("chi2 += (dx * dx + dy * dy + dz * dz) / sg2[k];",
                         "chi2 += (dx * dx + dy * dy) / sg2[k];")],
    "psum_pz_with_sin": [("sz += t.p * std::cos(t.theta1);", "sz += t.p * std::sin(t.theta1);")],
    "energy_sum_two_tracks": [("double sE = A.E + B.E + C.E;", "double sE = A.E + B.E;")],
    # Refined vertex (the finer vertex fit that Section VII names as future work)
    "refine_helix_forward": [("double ps = ps0 + (t.charge > 0 ? phi : -phi);",
                              "double ps = ps0 + (t.charge > 0 ? -phi : phi);")],
    "refine_z_slope_sin": [("p[2] = t.h0[2] - phi * t.rbar * std::cos(t.theta1);",
                            "p[2] = t.h0[2] - phi * t.rbar * std::sin(t.theta1);")],
    "refine_weights_unsquared": [("double sk = std::sqrt(s2[k]);", "double sk = s2[k];")],
    "refine_weights_equal": [("double sk = std::sqrt(s2[k]);", "double sk = 1.0;")],
    "refine_sigma_at_layer0_hit": [("o.s2[k] = point_sigma2(t, cax, cay, P);",
                                    "o.s2[k] = point_sigma2(t, t.h0[0], t.h0[1], P);")],
    "refine_stops_early": [("if (dv < 1e-10 && dp < 1e-12) { tiny = true; break; }",
                            "if (dv < 1e-2 && dp < 1e-3) { tiny = true; break; }")],
}


def _build(src_text, path):
    with open(path + ".cpp", "w") as f:
        f.write(src_text)
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", path,
                           path + ".cpp"], stderr=subprocess.DEVNULL)


def _pins(lib_path):
    env = dict(os.environ, MU3E_ORACLE_LIB=lib_path, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *[os.path.join(ROOT, "tests", f) for f in PIN_FILES]],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


def _mutate(src, edits):
    for old, new in edits:
        assert src.count(old) == 1, f"mutation anchor not unique or missing: {old!r}"
        src = src.replace(old, new)
    return src


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    d = tmp_path_factory.mktemp("oracle_mutants")
    src = open(SRC).read()
    jobs = {"unmutated": src}
    for name, edits in MUTANTS.items():
        jobs[name] = _mutate(src, edits)

    def run(item):
        name, text = item
        path = str(d / f"{name}.so")
        _build(text, path)
        return name, _pins(path)

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        return dict(ex.map(run, jobs.items()))


def test_unmutated_copy_passes(outcomes):
    rc, out = outcomes["unmutated"]
    assert rc == 0, out


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(outcomes, name):
    rc, out = outcomes[name]
    # 1: some test failed (a collection or usage error would be 2-4)
    assert rc == 1, f"mutant {name} not caught by the pins (pytest exit {rc}):\n{out}"
