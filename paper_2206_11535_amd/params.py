"""Selection parameters: geometry, cut windows, thresholds and caps.

The paper fixes the layer radii (Section IV), the 1 T field (Section III-B),
the 19 mm target radius (Section IV-C), the track chi2 cut of 32 (Section
IV-B) and the 768-triplet cap (Section VI-B).  It leaves the cut windows
("a set range", Section IV-A), the vertex thresholds (Section IV-C, Signal
Estimation) and the track / combination caps unstated.  Those values were
calibrated on truth of the synthetic generator and then frozen here:

* cut windows: the [0.1 %, 99.9 %] quantiles of the cut quantities of true
  layer-0/1/2 triplets, rounded outward to 4 significant figures; the cos(Phi)
  windows are one-sided (true triplets reach cos = 1);
* energy window, vertex chi2, target distance and momentum sum: the 99th
  percentiles on reconstructed signal decays;
* max_tracks and max_combos: 256 each (placeholders of this reading);
* max_layer_hits: 1023, the most hits per layer the kernels take (larger
  layers are tiled through LDS up to it); the paper keeps a whole frame in
  shared memory and has no such limit.

`tests/golden/calibrate_params.py` recomputes the calibrated numbers and a
test checks that they equal the values below.
"""
from __future__ import annotations

import copy
import math

DEFAULT = dict(
    r_layer=(25.0, 31.0, 73.0, 85.0),
    z_half=(62.0, 62.0, 175.0, 175.0),
    b_tesla=1.0,
    x_over_x0=0.001,
    sigma_pixel=0.08 / math.sqrt(12.0),
    # calibrated windows (pass iff lo <= q <= hi)
    dlambda=(-0.6612, 0.6515),
    cosphi01=(0.9619, 2.0),
    cosphi12=(0.3048, 2.0),
    rtc_abs=(32.28, 190.6),
    chi2_track_max=32.0,
    max_triplets=768,
    max_tracks=256,
    max_combos=256,
    # capacity of this implementation (frame-local hit indices are packed in
    # 10 bits), not a rule of the method: a frame above it is kept unprocessed
    max_layer_hits=1023,
    # calibrated vertex thresholds
    de_max=5.64,
    r_target=19.0,
    target_tol=2.0,
    chi2_vertex_max=206.0,
    d_target_max=3.31,
    p_sum_max=5.69,
    # relative half-width of the band around a cut edge inside which a
    # decision counts as ambiguous for parity (oracle only)
    amb=1e-5,
)

INT32_MAX = 2 ** 31 - 1


def default_params(**overrides) -> dict:
    p = copy.deepcopy(DEFAULT)
    for k, v in overrides.items():
        if k not in p:
            raise KeyError(k)
        p[k] = v
    return p


def lifted_caps(p: dict | None = None) -> dict:
    """Caps removed (pile-up stress run): every frame is processed fully."""
    p = default_params() if p is None else copy.deepcopy(p)
    p.update(max_triplets=INT32_MAX, max_tracks=INT32_MAX, max_combos=INT32_MAX)
    return p
