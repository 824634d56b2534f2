"""Sanitizer builds on the CPU: the oracle with AddressSanitizer and
UndefinedBehaviorSanitizer runs a set of workloads and every helper entry
point and must give the plain build's results; the HIP library with its
host code instrumented the same way (device code untouched) runs every
argument check of the C ABI.  Any sanitizer report aborts the child
process, which fails the test.  Nothing here needs a GPU."""
import glob
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:detect_odr_violation=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}

ORACLE_CHILD = r"""
import sys, os
sys.path.insert(0, sys.argv[1])
import numpy as np
from oracle import oracle
from paper_2206_11535_amd import synth
from paper_2206_11535_amd.params import default_params, lifted_caps
import json
out = {}
p = default_params()
def fsum(a):   # finite sum and the count of non-finite entries
    a = np.asarray(a, dtype=np.float64)
    return [float(np.sum(np.where(np.isfinite(a), a, 0.0))), int(np.sum(~np.isfinite(a)))]
cases = [("cfg1", synth.generate(1, n_frames=150), p), ("cfg2", synth.generate(2, n_frames=120), p),
         ("cfg4 lifted", synth.generate(4, n_frames=6), lifted_caps()),
         ("caps 0", synth.generate(1, n_frames=60), default_params(max_triplets=0, max_tracks=0, max_combos=0)),
         ("layer capacity 8", synth.generate(2, n_frames=40), default_params(max_layer_hits=8))]
for name, fs, q in cases:
    r = oracle.run(fs, q)
    out[name] = [int(r.flags.sum()), int(r.counts.sum()), int(r.amb.sum()), len(r.trips), len(r.tracks),
                 len(r.triples), *fsum(r.vertex)]
fs = synth.generate(2, n_frames=200)
tt, _, tab = synth.true_triplets(fs)
h = np.stack([np.stack([fs.x[tt[:, k]], fs.y[tt[:, k]], fs.z[tt[:, k]]], 1) for k in range(3)], 1)
f, ok = oracle.fit(h, p)
out["fit"] = [*fsum(f["chi2"]), int(ok.sum())]
q, dec = oracle.cut_quantities(h, p)
out["cuts"] = [*fsum(q), int(dec.sum())]
pr, ok = oracle.predict_l3(h, p)
out["l3"] = [*fsum(pr), int(ok.sum())]
t4 = tab[np.all(tab >= 0, axis=1)]
h4 = np.stack([np.stack([fs.x[t4[:, k]], fs.y[t4[:, k]], fs.z[t4[:, k]]], 1) for k in range(4)], 1)
o4, ok = oracle.track4(h4, p)
out["track4"] = [*fsum(o4), int(ok.sum())]
g, ok = oracle.track_geom(h4, p)
out["geom"] = [*fsum(g["E"]), int(ok.sum())]
tp, ok = oracle.track_point(h4, h4[:, 0, :2] * 0.5, p)
out["point"] = [*fsum(tp), int(ok.sum())]
out["cone"] = float(oracle.cone_distance(np.array([[10.0, 5.0], [0.0, 60.0], [25.0, -3.0]]), p).sum())
n3 = len(h4) // 3 * 3
v = oracle.vertex4(h4[:n3].reshape(-1, 3, 4, 3), p)
out["vertex4"] = fsum(v)
fa = synth.generate(5, n_frames=100)
r = oracle.run(fa, p)
k = r.tracks[(r.tracks[:, 6] == 1) & (r.tracks[:, 7] == 0)]
trip = np.concatenate([k[:, [1, 2, 3]], k[:, [2, 3, 4]]]).astype(np.int32)
L, G = oracle.align_loss_grad(fa, trip, np.zeros((synth.N_SENSORS, 4)), p)
out["align"] = [float(L), float(np.abs(G).sum())]
print(json.dumps(out))
"""


def _run_child(code, env_extra, args):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([sys.executable, "-c", code, *args], capture_output=True, text=True, timeout=600, env=env,
                       cwd=ROOT)
    assert r.returncode == 0, f"child failed ({r.returncode}):\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    return r.stdout.strip().splitlines()[-1]


def test_oracle_under_asan_ubsan(tmp_path):
    src = os.path.join(ROOT, "oracle", "mu3e_oracle.cpp")
    so = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", "-fPIC",
                           "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", so, src])
    asan = subprocess.check_output(["g++", "-print-file-name=libasan.so"], text=True).strip()
    ubsan = subprocess.check_output(["g++", "-print-file-name=libubsan.so"], text=True).strip()
    plain = _run_child(ORACLE_CHILD, {}, [ROOT])
    san = _run_child(ORACLE_CHILD, {**SAN_ENV, "LD_PRELOAD": f"{asan}:{ubsan}", "MU3E_ORACLE_LIB": so,
                                    "OMP_NUM_THREADS": "2"}, [ROOT])
    a, b = json.loads(plain), json.loads(san)
    assert a.keys() == b.keys()
    # counts equal; sums equal up to the order of a threaded reduction
    for k in a:
        for x, y in zip(np.atleast_1d(a[k]), np.atleast_1d(b[k])):
            assert x == y if float(x).is_integer() else abs(x - y) <= 1e-12 * max(abs(x), 1.0), (k, x, y)


ABI_CHILD = r"""
import ctypes, sys
sys.path.insert(0, sys.argv[1])
from paper_2206_11535_amd.lib import Hits, Params, Tracks, Tuning, Debug, make_params, declare
from paper_2206_11535_amd.params import default_params
L = declare(ctypes.CDLL(sys.argv[2]))   # the binding's declarations, without torch
p = make_params(default_params())
h = Hits(16, 32, 48, None, None, 64, 5, 10)
hn = Hits(16, 32, 48, None, 112, 64, 5, -1)
hf = Hits(16, 32, 48, None, None, 64, -1, 10)
checks = []
for s in (0, -1, -2, -3, -4, 7):
    checks.append(L.mu3e_status_string(s) is not None)
for F, tc, kc in ((0, 0, 0), (1000, 64000, 16000), (100000, 1 << 22, 1 << 17), (-1, 10, 10), (10, (1 << 30) + 1, 10)):
    L.mu3e_select_workspace_size(F, tc, kc)
    for n in range(0, 6):
        L.mu3e_plan_workspace_size(F, tc, kc, n)
for n in (-5, 0, 100, 1 << 20):
    L.mu3e_vertex_workspace_size(n)
for n in (-1, 0, 8, 2048, 4096):
    L.mu3e_align_workspace_size(n)
checks.append(L.mu3e_select_frames(None, ctypes.byref(p), 1, 1, 1, 1, 1 << 30, 10, 10, None, None) == -1)
checks.append(L.mu3e_select_frames(ctypes.byref(h), ctypes.byref(p), 1, 1, 1, 1, 16, 10, 10, None, None) == -3)
checks.append(L.mu3e_select_frames(ctypes.byref(hf), ctypes.byref(p), 1, 1, 1, 1, 1 << 30, 10, 10, None, None) == -1)
checks.append(L.mu3e_select_frames(ctypes.byref(hn), ctypes.byref(p), 1, 1, 1, 1, 1 << 30, 10, 10, None, None) == -1)
for bad in (dict(dlambda=(0.5, -0.5)), dict(max_tracks=-1), dict(r_layer=(25.0, 24.0, 73.0, 85.0)),
            dict(b_tesla=0.0), dict(rtc_abs=(-1.0, 5.0))):
    q = make_params(default_params(**bad))
    checks.append(L.mu3e_select_frames(ctypes.byref(h), ctypes.byref(q), 1, 1, 1, 1, 1 << 30, 10, 10, None,
                                       None) == -1)
q = make_params(default_params(max_layer_hits=1024))
checks.append(L.mu3e_select_frames(ctypes.byref(h), ctypes.byref(q), 1, 1, 1, 1, 1 << 30, 10, 10, None, None) == -4)
checks.append(L.mu3e_select_frames_static(ctypes.byref(h), ctypes.byref(p), 1, 1, 1, 1 << 30, 1 << 20, None,
                                          None) == -3)
checks.append(L.mu3e_fit_triplets(ctypes.byref(hn), 1, 5, ctypes.byref(p), 1, None) == -1)
checks.append(L.mu3e_fit_triplets_backward(ctypes.byref(h), None, 5, ctypes.byref(p), 1, 1, None) == -1)
checks.append(L.mu3e_vertex(ctypes.byref(h), None, ctypes.byref(p), 1, 1, 1, 1, 1 << 20, None) == -1)
tr = Tracks(80, 96, 4, 1000)
checks.append(L.mu3e_vertex(ctypes.byref(h), ctypes.byref(tr), ctypes.byref(p), 1, 1, 1, 1, 8, None) == -3)
checks.append(L.mu3e_align_chi2(ctypes.byref(hn), 1, 5, 1, 8, ctypes.byref(p), 1, None) == -1)
checks.append(L.mu3e_vertex_refine(ctypes.byref(h), ctypes.byref(tr), 1, 5, None, ctypes.byref(p), 1, 1, 1, 8,
                                   None) == -3)
checks.append(L.mu3e_vertex_refine(ctypes.byref(hn), ctypes.byref(tr), 1, 5, None, ctypes.byref(p), 1, 1, 1,
                                   1 << 20, None) == -1)
t = Tuning(8, 4, 0, 101, 64, 1)
plan = ctypes.c_void_p()
checks.append(L.mu3e_plan_create(ctypes.byref(plan), ctypes.byref(h), ctypes.byref(p), 1, 1, 1, 1, 1 << 30, 10, 10,
                                 ctypes.byref(t)) == -1)
t = Tuning(8, 4, 0, 0, 96, 1)
checks.append(L.mu3e_plan_create(ctypes.byref(plan), ctypes.byref(h), ctypes.byref(p), 1, 1, 1, 1, 1 << 30, 10, 10,
                                 ctypes.byref(t)) == -1)
t = Tuning(8, 4, 0, 0, 64, 9)
checks.append(L.mu3e_plan_create(ctypes.byref(plan), ctypes.byref(h), ctypes.byref(p), 1, 1, 1, 1, 1 << 30, 10, 10,
                                 ctypes.byref(t)) == -1)
checks.append(L.mu3e_plan_run(None, None) == -1 and L.mu3e_plan_run_timed(None, None, None) == -1)
checks.append(L.mu3e_plan_part_info(None, 0, None, None, None) == -1)
L.mu3e_plan_destroy(None)
checks.append(L.mu3e_chunk_unpack(ctypes.c_void_p(4098), 1024, 10, 100, 16, 32, 48, 64, 80, None) == -1)
checks.append(L.mu3e_chunk_unpack(None, 1024, 10, 100, 16, 32, 48, 64, 80, None) == -1)
print("ok" if all(checks) else f"failed {[i for i, c in enumerate(checks) if not c]}")
"""


def test_abi_host_checks_under_asan_ubsan(tmp_path):
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("no clang AddressSanitizer runtime in this ROCm")
    from paper_2206_11535_amd import build
    so = str(tmp_path / "libmu3e_san.so")
    flags = [f for f in build.FLAGS if f != "-Wall"]
    subprocess.check_call(["hipcc", *flags, "-g", "-Xarch_host", "-fsanitize=address",
                           "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(build.PKG, "csrc"),
                           "-o", so, build.SRC], stderr=subprocess.DEVNULL)
    out = _run_child(ABI_CHILD, {**SAN_ENV, "LD_PRELOAD": rt[-1]}, [ROOT, so])
    assert out == "ok"
