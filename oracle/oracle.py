"""Python access to the FP64 oracle (mu3e_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark.  The product library never imports it.

Parameters are passed as a plain dict with the field names of PARAM_FIELDS;
float fields are rounded to float32 first, so the oracle sees exactly the
values the float32 GPU parameter block carries.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mu3e_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

# Flag bits (same meaning as the product's frame flags; defined here again on
# purpose: the oracle shares nothing with the product).
KEEP, TRIPLET_OVF, TRACK_OVF, COMBO_OVF, VERTEX, HITS_OVF = 1, 2, 4, 8, 16, 32

PARAM_FIELDS = (
    [("r_layer", 4), ("z_half", 4), ("b_tesla", 1), ("x_over_x0", 1), ("sigma_pixel", 1),
     ("dlambda", 2), ("cosphi01", 2), ("cosphi12", 2), ("rtc_abs", 2),
     ("chi2_track_max", 1),
     ("max_triplets", 1), ("max_tracks", 1), ("max_combos", 1), ("max_layer_hits", 1),
     ("de_max", 1), ("r_target", 1), ("target_tol", 1), ("chi2_vertex_max", 1),
     ("d_target_max", 1), ("p_sum_max", 1), ("amb", 1)])
INT_FIELDS = {"max_triplets", "max_tracks", "max_combos", "max_layer_hits"}


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _bind(path: str):
    """Load an oracle shared library and declare its entry points."""
    L = ctypes.CDLL(path)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.oc_run.restype = P
    L.oc_run.argtypes = [P, P, P, P, I, P, I, I]
    L.oc_seconds.restype = D
    L.oc_seconds.argtypes = [P]
    L.oc_threads_used.restype = I
    L.oc_threads_used.argtypes = [I]
    L.oc_sizes.argtypes = [P, P, P, P]
    L.oc_frames.argtypes = [P, P, P, P, P, P, P]
    L.oc_lists.argtypes = [P, P, P, P, P, P]
    L.oc_free.argtypes = [P]
    L.oc_cut_quantities.argtypes = [P, I, P, P, P]
    L.oc_fit.argtypes = [P, I, P, P, P]
    L.oc_predict_l3.argtypes = [P, I, P, P, P]
    L.oc_track4.argtypes = [P, I, P, P, P]
    L.oc_vertex4.argtypes = [P, I, P, P]
    L.oc_track_geom.argtypes = [P, I, P, P, P]
    L.oc_track_point.argtypes = [P, P, I, P, P, P]
    L.oc_cone_distance.argtypes = [P, I, P, P]
    L.oc_refine4.argtypes = [P, I, P, P, P]
    L.oc_refine_residual.argtypes = [P, P, P, I, P, P]
    L.oc_align_loss_grad.restype = D
    L.oc_align_loss_grad.argtypes = [P, P, P, P, P, I, P, I, P, P, I, P]
    L.oc_param_count.restype = I
    return L


def lib():
    """The oracle library: the in-tree build, or the build named by the
    environment variable MU3E_ORACLE_LIB (the mutation tests point it at
    copies of the source with a planted mistake)."""
    global _lib
    if _lib is None:
        alt = os.environ.get("MU3E_ORACLE_LIB")
        if alt:
            _lib = _bind(alt)
        else:
            build()
            _lib = _bind(LIB)
    return _lib


class use_library:
    """Context manager: route every call of this module to another build of
    the oracle source (the mutation tests compile copies with a planted
    mistake and check that the pins reject them)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = _bind(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def pack_params(p: dict) -> np.ndarray:
    vals = []
    for name, n in PARAM_FIELDS:
        v = p[name]
        v = list(v) if n > 1 else [v]
        assert len(v) == n, name
        for x in v:
            vals.append(float(int(x)) if name in INT_FIELDS else float(np.float32(x)))
    arr = np.asarray(vals, np.float64)
    assert len(arr) == lib().oc_param_count()
    return arr


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class OracleResult:
    flags: np.ndarray        # uint32 [F]
    amb: np.ndarray          # uint32 [F] flag bits whose value is ambiguous
    counts: np.ndarray       # int32 [F, 3] sure counts: triplets, tracks, energy-passing triples
    namb: np.ndarray         # int32 [F, 3] ambiguous candidates per stage
    vertex: np.ndarray       # float64 [F, 4] x, y, z, chi2 (NaN if none)
    stats: np.ndarray        # int64 [6]
    seconds: float
    trips: np.ndarray = None     # int32 [n, 6] frame, h0, h1, h2, pass, amb
    trip_rtc: np.ndarray = None  # float64 [n]
    tracks: np.ndarray = None    # int32 [n, 8] frame, h0..h3, charge, pass, amb
    track_f: np.ndarray = None   # float64 [n, 2] kbar, chi2
    triples: np.ndarray = None   # int32 [n, 12] frame, 3x(h0,h1,h2), pass, amb


def run(fs, params: dict, lists: bool = True, threads: int = 0) -> OracleResult:
    """Run the full selection over a FrameSet (or an object with x, y, z,
    layer_offsets)."""
    L = lib()
    x = np.ascontiguousarray(fs.x, np.float32)
    y = np.ascontiguousarray(fs.y, np.float32)
    z = np.ascontiguousarray(fs.z, np.float32)
    lo = np.ascontiguousarray(fs.layer_offsets, np.int32)
    F = (len(lo) - 1) // 4
    pp = pack_params(params)
    h = L.oc_run(_ptr(x), _ptr(y), _ptr(z), _ptr(lo), F, _ptr(pp), int(lists), int(threads))
    try:
        flags = np.zeros(F, np.uint32)
        amb = np.zeros(F, np.uint32)
        counts = np.zeros((F, 3), np.int32)
        namb = np.zeros((F, 3), np.int32)
        vtx = np.zeros((F, 4), np.float64)
        stats = np.zeros(6, np.int64)
        L.oc_frames(h, _ptr(flags), _ptr(amb), _ptr(counts), _ptr(namb), _ptr(vtx), _ptr(stats))
        res = OracleResult(flags, amb, counts, namb, vtx, stats, L.oc_seconds(h))
        if lists:
            a, b, c = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_longlong()
            L.oc_sizes(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
            res.trips = np.zeros((a.value, 6), np.int32)
            res.trip_rtc = np.zeros(a.value, np.float64)
            res.tracks = np.zeros((b.value, 8), np.int32)
            res.track_f = np.zeros((b.value, 2), np.float64)
            res.triples = np.zeros((c.value, 12), np.int32)
            L.oc_lists(h, _ptr(res.trips), _ptr(res.trip_rtc), _ptr(res.tracks),
                       _ptr(res.track_f), _ptr(res.triples))
        return res
    finally:
        L.oc_free(h)


def threads_used(threads: int = 0) -> int:
    return lib().oc_threads_used(int(threads))


def cut_quantities(h: np.ndarray, params: dict):
    """h [n, 3, 3] (hit, xyz) -> (q [n, 4] dlambda, cosphi01, cosphi12, rtc; dec [n])."""
    h = np.ascontiguousarray(h, np.float64).reshape(-1, 9)
    n = len(h)
    out = np.zeros((n, 4))
    dec = np.zeros(n, np.int32)
    lib().oc_cut_quantities(_ptr(h), n, _ptr(pack_params(params)), _ptr(out), _ptr(dec))
    return out, dec


FIT_FIELDS = ("kappa", "sigma2_kappa", "chi2", "r_star", "sigma2_r", "rtc", "theta1",
              "theta2", "phi1", "phi2", "rbar_c", "sigma_ms", "cx", "cy")


def fit(h: np.ndarray, params: dict):
    """Single triplet fit; h [n, 3, 3] -> (dict of [n] arrays, ok [n])."""
    h = np.ascontiguousarray(h, np.float64).reshape(-1, 9)
    n = len(h)
    out = np.zeros((n, 14))
    ok = np.zeros(n, np.int32)
    lib().oc_fit(_ptr(h), n, _ptr(pack_params(params)), _ptr(out), _ptr(ok))
    return {k: out[:, i] for i, k in enumerate(FIT_FIELDS)}, ok.astype(bool)


def predict_l3(h: np.ndarray, params: dict):
    h = np.ascontiguousarray(h, np.float64).reshape(-1, 9)
    n = len(h)
    out = np.zeros((n, 3))
    ok = np.zeros(n, np.int32)
    lib().oc_predict_l3(_ptr(h), n, _ptr(pack_params(params)), _ptr(out), _ptr(ok))
    return out, ok.astype(bool)


def track4(h: np.ndarray, params: dict):
    """Track from four hits; h [n, 4, 3] -> (out [n, 4] kbar, chi2, theta1, rbar; ok [n])."""
    h = np.ascontiguousarray(h, np.float64).reshape(-1, 12)
    n = len(h)
    out = np.full((n, 4), np.nan)
    ok = np.zeros(n, np.int32)
    lib().oc_track4(_ptr(h), n, _ptr(pack_params(params)), _ptr(out), _ptr(ok))
    return out, ok.astype(bool)


def vertex4(h: np.ndarray, params: dict):
    """Vertex of e+ e+ e- track triples; h [n, 3, 4, 3] -> out [n, 10]
    (pass, x, y, z, chi2, sumE, amb, dtarget, psum, reached)."""
    h = np.ascontiguousarray(h, np.float64).reshape(-1, 36)
    n = len(h)
    out = np.zeros((n, 10))
    lib().oc_vertex4(_ptr(h), n, _ptr(pack_params(params)), _ptr(out))
    return out


TRACK_FIELDS = ("kbar", "rbar", "rt", "cx", "cy", "sms0", "E", "p", "theta1")


def track_geom(h: np.ndarray, params: dict):
    """Vertex-stage quantities of tracks given by four hits; h [n, 4, 3] ->
    (dict of [n] arrays with TRACK_FIELDS, ok [n])."""
    h = np.ascontiguousarray(h, np.float64).reshape(-1, 12)
    n = len(h)
    out = np.zeros((n, 9))
    ok = np.zeros(n, np.int32)
    lib().oc_track_geom(_ptr(h), n, _ptr(pack_params(params)), _ptr(out), _ptr(ok))
    return {k: out[:, i] for i, k in enumerate(TRACK_FIELDS)}, ok.astype(bool)


def track_point(h: np.ndarray, q: np.ndarray, params: dict):
    """Backward turning angle from the layer-0 hit to the transverse point q,
    the path length and the position variance there (eq. track-error);
    h [n, 4, 3], q [n, 2] -> (out [n, 3], ok [n])."""
    h = np.ascontiguousarray(h, np.float64).reshape(-1, 12)
    q = np.ascontiguousarray(q, np.float64).reshape(-1, 2)
    n = len(h)
    out = np.zeros((n, 3))
    ok = np.zeros(n, np.int32)
    lib().oc_track_point(_ptr(h), _ptr(q), n, _ptr(pack_params(params)), _ptr(out), _ptr(ok))
    return out, ok.astype(bool)


def cone_distance(rz: np.ndarray, params: dict):
    """Distance of (rho, z) points [n, 2] to the double-cone target surface."""
    rz = np.ascontiguousarray(rz, np.float64).reshape(-1, 2)
    out = np.zeros(len(rz))
    lib().oc_cone_distance(_ptr(rz), len(rz), _ptr(pack_params(params)), _ptr(out))
    return out


REFINE_FIELDS = ("x", "y", "z", "J", "phi0", "phi1", "phi2", "s2_0", "s2_1", "s2_2",
                 "rough_x", "rough_y", "rough_z", "rough_chi2", "iters", "rough_amb")


def refine4(h: np.ndarray, params: dict):
    """Refined vertex of e+ e+ e- track triples given by four hits each (the
    minimiser of the weighted squared distances to the three helices,
    started from the rough estimate); h [n, 3, 4, 3] -> (out [n, 16] with
    REFINE_FIELDS, status [n]: 1 converged, 0 rough estimate does not pass,
    -1 no convergence, -2 a track fit fails)."""
    h = np.ascontiguousarray(h, np.float64).reshape(-1, 36)
    n = len(h)
    out = np.zeros((n, 16))
    st = np.zeros(n, np.int32)
    lib().oc_refine4(_ptr(h), n, _ptr(pack_params(params)), _ptr(out), _ptr(st))
    return out, st


def refine_residual(h: np.ndarray, x: np.ndarray, s2: np.ndarray, params: dict):
    """Weighted residuals [n, 9] of the refined-vertex objective at x [n, 6]
    = (vertex, three turning angles) with fixed variances s2 [n, 3]."""
    h = np.ascontiguousarray(h, np.float64).reshape(-1, 36)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 6)
    s2 = np.ascontiguousarray(s2, np.float64).reshape(-1, 3)
    n = len(h)
    r = np.zeros((n, 9))
    lib().oc_refine_residual(_ptr(h), _ptr(x), _ptr(s2), n, _ptr(pack_params(params)), _ptr(r))
    return r


def align_loss_grad(fs, trip: np.ndarray, theta: np.ndarray, params: dict, grad: bool = True, weight=None):
    """L(theta) = sum over triplets of (weight *) the fit chi2 after per-sensor
    alignment, and dL/dtheta [S, 4] (exact, forward-mode duals)."""
    x = np.ascontiguousarray(fs.x, np.float32)
    y = np.ascontiguousarray(fs.y, np.float32)
    z = np.ascontiguousarray(fs.z, np.float32)
    s = np.ascontiguousarray(fs.sensor, np.uint16)
    t = np.ascontiguousarray(trip, np.int32).reshape(-1, 3)
    th = np.ascontiguousarray(theta, np.float64)
    S = th.shape[0]
    g = np.zeros((S, 4))
    w = None if weight is None else np.ascontiguousarray(weight, np.float64)
    Lv = lib().oc_align_loss_grad(_ptr(x), _ptr(y), _ptr(z), _ptr(s), _ptr(t), len(t), _ptr(th), S,
                                  _ptr(pack_params(params)), _ptr(g), int(grad), None if w is None else _ptr(w))
    return Lv, g
