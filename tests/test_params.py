"""The frozen default parameters equal the calibration procedure's output
(tests/golden/calibrate_params.py, which uses only the generator and the
oracle), and the stored calibration record matches both."""
import json
import os

import numpy as np

from paper_2206_11535_amd.params import DEFAULT, lifted_caps, INT32_MAX

HERE = os.path.dirname(os.path.abspath(__file__))


def test_defaults_equal_calibration():
    import importlib.util
    spec = importlib.util.spec_from_file_location("cal", os.path.join(HERE, "golden", "calibrate_params.py"))
    cal = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(cal)
    res = cal.calibrate()
    with open(os.path.join(HERE, "golden", "params_calibrated.json")) as f:
        stored = json.load(f)
    for k in ("dlambda", "cosphi01", "cosphi12", "rtc_abs"):
        assert tuple(res["cuts"][k]) == tuple(DEFAULT[k]) == tuple(stored["cuts"][k])
    for k in ("de_max", "chi2_vertex_max", "d_target_max", "p_sum_max"):
        assert res["vertex"][k] == DEFAULT[k] == stored["vertex"][k]
    # the calibration kept at least 98.5 % of true triplets per cut edge
    # (Section IV-A requirement) by construction: 0.1 % per tail, 4 cuts
    assert res["cuts"]["n_true"] > 100000


def test_paper_fixed_values():
    assert DEFAULT["r_layer"] == (25.0, 31.0, 73.0, 85.0)
    assert DEFAULT["chi2_track_max"] == 32.0
    assert DEFAULT["max_triplets"] == 768
    assert DEFAULT["r_target"] == 19.0
    assert DEFAULT["b_tesla"] == 1.0
    p = lifted_caps()
    assert p["max_triplets"] == p["max_tracks"] == p["max_combos"] == INT32_MAX
