"""Throughput of the online event selection on one MI355X.

One step = the whole selection (Selection Cuts -> Track Reconstruction ->
Vertex Fit) over one batch of synthetic frames already resident in HBM.
Workload: the nominal rate, 100,000 frames of 64 ns at 1e8 mu/s
(Poisson(6.4) Michel decays per frame, 5 noise hits per layer, signal in 1 %
of frames).  Both forms run on it: the plain per-frame kernels and the
batched persistent form (one hipGraph launch, autotuned shape).  `value` is
the batched form with `--inflight` batches in flight, as a continuous stream
of batches is processed: each of that many distinct batches (different
seeds, same workload) has its own plan and stream, and step k runs batch
k mod n, so one batch's latency-bound stages overlap another's cuts.  The
same form with one batch in flight is reported alongside.  Optional legs:
the mixed-rate 1,000,000-frame batch (both forms, one batch in flight,
identical outputs required) and the alignment gradient.  Prints one JSON
line.
"""
from __future__ import annotations

import argparse
import ctypes
import gc
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

STAGES = ("cuts", "tracks", "vertex_prep", "vertex")

# Algorithmic float32 operations of the track stage per selected triplet
# (first fit, layer-3 crossing, second fit, weighted combination), plus 8 per
# layer-3 hit scanned (3D squared distance).  Counted from the formulas of the
# circumcircle, the linearised triplet fit and the circle intersection.
FLOPS_PER_TRIPLET = 430
FLOPS_PER_L3_HIT = 8
# Selection Cuts: cos Phi of a pair (2 mul, 1 add, 1 scale) = 4, plus the
# slope tan(lambda) of an (h1, h2) pair (sub, mul) = 2; per joined
# combination the (h0, h1) slope and the difference = 3; per Delta-lambda
# survivor the signed circumradius test (3 chord differences, cross product,
# 3 squared chords, their product, 4 cross^2, two scaled bounds) = 24.
FLOPS_PAIR01, FLOPS_PAIR12, FLOPS_JOIN, FLOPS_RTC = 4, 6, 3, 24

# HBM bytes per launch of the roofline kernel on this workload, from
# rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by a copy probe, keyed by
# "<hash of the kernel sources>|<kernel>" of the build it was measured on
# (null once the source changes).
TRAFFIC = {
    # profiles/nominal_hbm_traffic.md: 88.70 MB read + 23.21 MB written per launch
    "cf79a04bb751ce55|k_batched": 111892060,
}

PEAK_FP32 = 157.3   # TFLOP/s, MI355X float32 vector (published)


def source_hash() -> str:
    """Hash of the kernel sources and the build flags (build.py)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2206_11535_amd", "csrc")
    names = sorted(n for n in os.listdir(csrc) if n.endswith((".hip", ".hpp")))
    for p in [os.path.join(csrc, n) for n in names] + [os.path.join(ROOT, "paper_2206_11535_amd", "build.py")]:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


class Hip:
    """hipEvent_* of the process's HIP runtime (the one torch loaded)."""

    def __init__(self):
        self.L = ctypes.CDLL("libamdhip64.so.7")
        self.L.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.L.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        self.L.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.L.hipEventSynchronize.argtypes = [ctypes.c_void_p]

    @staticmethod
    def _ok(status, what):
        if status != 0:
            raise RuntimeError(f"{what} failed with HIP error {status}")

    def events(self, n):
        arr = (ctypes.c_void_p * n)()
        for i in range(n):
            e = ctypes.c_void_p()
            self._ok(self.L.hipEventCreate(ctypes.byref(e)), "hipEventCreate")
            arr[i] = e
        return arr

    def record(self, e, stream):
        self._ok(self.L.hipEventRecord(e, ctypes.c_void_p(stream.cuda_stream)), "hipEventRecord")

    def elapsed(self, a, b) -> float:
        ms = ctypes.c_float()
        self._ok(self.L.hipEventSynchronize(b), "hipEventSynchronize")
        self._ok(self.L.hipEventElapsedTime(ctypes.byref(ms), a, b), "hipEventElapsedTime")
        return ms.value


def cpu_baseline(fs, params, min_seconds=10.0):
    from oracle import oracle
    threads = oracle.threads_used(0)
    done, secs, reps = 0, 0.0, 0
    while secs < min_seconds and reps < 60:
        r = oracle.run(fs, params, lists=False)
        secs += r.seconds
        done += fs.n_frames
        reps += 1
    return {"value": done / secs, "unit": "frames/s", "cores": threads, "kind": "oracle",
            "sample": f"the {fs.n_frames}-frame nominal workload x {reps} passes ({secs:.1f} s of the FP64 C++ "
                      f"oracle, OpenMP over frames)"}


def time_steps(sel, dh, stream, hip, steps, warmup, staged=False):
    """Mean ms per step over `steps` timed steps (HIP events on the launch
    stream, bracketed by device synchronisation); per-stage means if the
    selector records stage events."""
    import torch
    for _ in range(warmup):
        sel.run(dh, stream)
    torch.cuda.synchronize()
    c = sel.counters()
    if c[2] != 0:
        raise RuntimeError(f"candidate lists overflowed the workspace: {c}")
    ev = [hip.events(5) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        if staged:
            sel.run(dh, stream, events=ev[k])
        else:
            hip.record(ev[k][0], stream)
            sel.run(dh, stream)
            hip.record(ev[k][4], stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [hip.elapsed(ev[k][0], ev[k][4]) for k in range(steps)]
    stage = None
    if staged:
        stage = np.mean([[hip.elapsed(ev[k][s], ev[k][s + 1]) for s in range(4)] for k in range(steps)], axis=0)
    return float(np.mean(step_ms)), stage, wall


def time_inflight(plans, streams, hip, steps, warmup):
    """Wall-clock ms per step with step k on plans[k % n] / streams[k % n]
    (bracketed by device synchronisation), and the mean latency of one batch
    (HIP events around its graph launch on its stream)."""
    import torch
    n = len(plans)
    for k in range(warmup * n):
        plans[k % n].run(None, streams[k % n])
    torch.cuda.synchronize()
    for pl in plans:
        c = pl.counters()
        if c[2] != 0:
            raise RuntimeError(f"candidate lists overflowed the workspace: {c}")
    ev = [hip.events(2) for _ in range(steps)]
    torch.cuda.synchronize()
    gc.disable()   # no collector pause while the host feeds the streams
    t0 = time.perf_counter()
    for k in range(steps):
        st = streams[k % n]
        hip.record(ev[k][0], st)
        plans[k % n].run(None, st)
        hip.record(ev[k][1], st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gc.enable()
    lat = float(np.mean([hip.elapsed(e[0], e[1]) for e in ev]))
    return wall / steps * 1e3, lat, wall


def fitted_triplets(sel, fs):
    from paper_2206_11535_amd import lib
    flags, counts, _ = sel.result()
    ovf = (flags & (lib.TRIPLET_OVF | lib.HITS_OVF)) != 0
    n3 = np.diff(fs.layer_offsets)[3::4]
    fitted = int(counts[~ovf, 0].sum())
    flops = float(np.sum(counts[~ovf, 0].astype(np.float64) * (FLOPS_PER_TRIPLET + FLOPS_PER_L3_HIT * n3[~ovf])))
    return fitted, flops, flags


def _pairs(fs, la, lb):
    """Global hit indices of every (layer la, layer lb) pair of each frame."""
    lo = fs.layer_offsets.astype(np.int64)
    oa, ob = lo[la:-1:4], lo[lb:-1:4]
    na, nb = lo[la + 1::4] - oa, lo[lb + 1::4] - ob
    npair = na * nb
    start = np.concatenate([[0], np.cumsum(npair)[:-1]])
    pf = np.repeat(np.arange(len(na)), npair)
    k = np.arange(int(npair.sum()), dtype=np.int64) - start[pf]
    return oa[pf] + k // nb[pf], ob[pf] + k % nb[pf]


def cut_work(fs, p):
    """Counts of the units the Selection Cuts work on, from the hits on the
    host in float32 (the same windows): pairs per layer pair, joined
    combinations and Delta-lambda survivors.  Work accounting only."""
    x, y, z = fs.x, fs.y, fs.z
    R = np.asarray(p["r_layer"], np.float32)
    i0, i1 = _pairs(fs, 0, 1)
    j1, j2 = _pairs(fs, 1, 2)
    c01 = (x[i0] * x[i1] + y[i0] * y[i1]) * np.float32(1.0 / (R[0] * R[1]))
    c12 = (x[j1] * x[j2] + y[j1] * y[j2]) * np.float32(1.0 / (R[1] * R[2]))
    a = (c01 >= p["cosphi01"][0]) & (c01 <= p["cosphi01"][1])
    b = (c12 >= p["cosphi12"][0]) & (c12 <= p["cosphi12"][1])
    i0, i1, j1, j2 = i0[a], i1[a], j1[b], j2[b]
    t01 = (z[i1] - z[i0]) * np.float32(1.0 / (R[1] - R[0]))
    t12 = (z[j2] - z[j1]) * np.float32(1.0 / (R[2] - R[1]))
    # join on the shared layer-1 hit
    o01, o12 = np.argsort(i1, kind="stable"), np.argsort(j1, kind="stable")
    i1s, t01s = i1[o01], t01[o01]
    j1s, t12s = j1[o12], t12[o12]
    n = fs.n_hits
    n01 = np.bincount(i1s, minlength=n)
    n12 = np.bincount(j1s, minlength=n)
    s12 = np.concatenate([[0], np.cumsum(n12)[:-1]])
    rep = n12[i1s]
    joins = int(rep.sum())
    left = np.repeat(np.arange(len(i1s)), rep)
    st = np.concatenate([[0], np.cumsum(rep)[:-1]])
    right = s12[i1s[left]] + (np.arange(joins) - st[left])
    dl = t12s[right] - t01s[left]
    dl_pass = int(np.count_nonzero((dl >= p["dlambda"][0]) & (dl <= p["dlambda"][1])))
    del n01
    return {"pairs01": int(a.size), "pairs12": int(b.size), "joins": joins, "dlambda_pass": dl_pass}


def cut_flops(w) -> float:
    return float(FLOPS_PAIR01 * w["pairs01"] + FLOPS_PAIR12 * w["pairs12"] + FLOPS_JOIN * w["joins"] +
                 FLOPS_RTC * w["dlambda_pass"])


def same_outputs(a, b) -> bool:
    fa, ca, va = a.result()
    fb, cb, vb = b.result()
    return bool(np.array_equal(fa, fb) and np.array_equal(ca, cb) and
                np.array_equal(np.nan_to_num(va), np.nan_to_num(vb)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--frames", type=int, default=None, help="prefix of the workload (debug)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mixed", action="store_true", help="also the mixed-rate 1,000,000-frame batch")
    ap.add_argument("--align", action="store_true", help="also the alignment gradient (misaligned frames)")
    ap.add_argument("--inflight", type=int, default=3,
                    help="distinct batches in flight on their own streams for `value` (1: one at a time)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (scale for the HBM traffic counters)")
    a = ap.parse_args()
    if a.inflight < 1:
        ap.error("--inflight must be at least 1")
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {a.gpus} requested): frames are independent, so more GPUs "
              f"would each take a contiguous range of frames; that split is not built here", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2206_11535_amd import autotune, lib, synth
    from paper_2206_11535_amd.params import default_params

    fs = synth.generate(synth.CONFIGS[2], n_frames=a.frames)
    p = default_params()
    F = fs.n_frames
    dev = torch.device("cuda:0")
    dh = lib.to_device(fs, dev)
    hip = Hip()
    stream = torch.cuda.current_stream(dev)
    # ---- plain form (per-stage events)
    plain = lib.Selector(F, p, device=dev)
    ms_plain, stage_ms, _ = time_steps(plain, dh, stream, hip, a.steps, a.warmup, staged=True)
    fitted, flops, flags = fitted_triplets(plain, fs)
    # ---- batched form (autotuned shape, cached)
    (w, c, u, st), _, _ = autotune.tune(dh, p)
    batched = lib.BatchedSelector(dh, p, device=dev, waves_per_cu=w, frames_per_claim=c, fuse_fits=u,
                                  steal_percent=st)
    ms_one, _, wall_one = time_steps(batched, dh, stream, hip, a.steps, a.warmup)
    identical = same_outputs(plain, batched)
    # ---- the batched form with `inflight` distinct batches in flight
    latency = ms_one
    ms_batched, wall = ms_one, wall_one
    inflight_equal = True
    if a.inflight > 1:
        plans, streams = [batched], [torch.cuda.Stream(dev)]
        refs = []
        for i in range(1, a.inflight):
            fi = synth.generate(synth.CONFIGS[2], n_frames=a.frames, salt=i)
            di = lib.to_device(fi, dev)
            plans.append(lib.BatchedSelector(di, p, device=dev, waves_per_cu=w, frames_per_claim=c, fuse_fits=u,
                                             steal_percent=st))
            streams.append(torch.cuda.Stream(dev))
            refs.append(lib.select_frames(di, p))
        ms_batched, latency, wall = time_inflight(plans, streams, hip, a.steps, a.warmup)
        torch.cuda.synchronize()
        inflight_equal = same_outputs(plain, batched) and all(same_outputs(r, q) for r, q in zip(refs, plans[1:]))
        Fb = [q.hits.n_frames for q in plans]
        if len(set(Fb)) != 1:
            raise RuntimeError(f"batches of different sizes in flight: {Fb}")
        del refs
    # kernel durations: the same sequence launched eagerly with events around
    # the persistent kernel and the fit kernel, on the launch stream
    ev = [hip.events(4) for _ in range(a.steps)]
    for k in range(a.steps):
        batched.run(None, stream, events=ev[k])
    torch.cuda.synchronize()
    ms_kbatched = float(np.mean([hip.elapsed(e[0], e[1]) for e in ev]))
    ms_ktracks = float(np.mean([hip.elapsed(e[1], e[2]) for e in ev]))
    identical = identical and same_outputs(plain, batched)
    work = cut_work(fs, p)
    fused = bool(batched.effective[2])
    # algorithmic flops of each kernel (the fused persistent kernel also fits;
    # the few fits it leaves to k_tracks are counted with it)
    kernels = {"k_batched": (ms_kbatched, cut_flops(work) + (flops if fused else 0.0)),
               "k_tracks": (ms_ktracks, 0.0 if fused else flops)}
    dom = max(kernels, key=lambda k: kernels[k][0])
    if a.copy_probe:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)   # an elementwise kernel: 256 MiB read, 256 MiB written
        torch.cuda.synchronize()
    # roofline of the dominant kernel of the batched step (algorithmic flops
    # / its measured time)
    dom_ms, dom_flops = kernels[dom]
    achieved = dom_flops / (dom_ms / 1e3) / 1e12
    tracks_achieved = flops / (stage_ms[1] / 1e3) / 1e12
    sh = source_hash()
    out = {
        "metric": "frames/s at 1e8 mu/s-equivalent load (batched persistent form; plain form alongside)",
        "value": F / (ms_batched / 1e3), "unit": "frames/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_batched, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"nominal rate, {F} frames of 64 ns, Poisson(6.4) Michel decays + 5 noise "
                               f"hits/layer, signal in 1% of frames", "frames": F, "form": "batched",
                   "batches_in_flight": a.inflight,
                   "waves_per_cu": batched.effective[0], "frames_per_claim": batched.effective[1],
                   "fused_fits": fused, "steal_percent": batched.effective[3]},
        "fitted_triplets_per_s": fitted / (ms_batched / 1e3),
        "batch_latency_ms": latency,
        "one_in_flight": {"value": F / (ms_one / 1e3), "ms_per_step": ms_one},
        "inflight_equals_plain": inflight_equal,
        "plain": {"value": F / (ms_plain / 1e3), "ms_per_step": ms_plain,
                  "fitted_triplets_per_s": fitted / (ms_plain / 1e3),
                  "stage_ms": {s: float(v) for s, v in zip(STAGES, stage_ms)},
                  "k_tracks_tflops": tracks_achieved},
        "batched_equals_plain": identical,
        "kept_fraction": float(np.mean(flags & lib.KEEP)),
        "roofline": {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": PEAK_FP32,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32, "traffic": TRAFFIC.get(f"{sh}|{dom}"),
                     "kernel_ms": dom_ms, "flops_per_launch": dom_flops,
                     "kernels_ms": {k: v[0] for k, v in kernels.items()}, "work": work,
                     "fitted_triplets": fitted, "source": sh},
        "wall_s_timed": wall,
        "paper_context": "1.4e6 frames/s on a GTX 1080Ti at 1e8 mu/s (Geant4 frames, not this workload)",
    }
    if a.mixed:
        fm = synth.generate(synth.CONFIGS[3])
        dm = lib.to_device(fm, dev)
        sp = lib.Selector(fm.n_frames, p, device=dev)
        msp, _, _ = time_steps(sp, dm, stream, hip, max(3, a.steps // 4), 1)
        (wm, cm, um, sm), _, _ = autotune.tune(dm, p)
        sb = lib.BatchedSelector(dm, p, device=dev, waves_per_cu=wm, frames_per_claim=cm, fuse_fits=um,
                                 steal_percent=sm)
        msb, _, _ = time_steps(sb, dm, stream, hip, max(3, a.steps // 4), 1)
        out["mixed"] = {"workload": f"{fm.n_frames} frames, lambda per frame from {{2, 6.4, 12, 20}}",
                        "plain_frames_per_s": fm.n_frames / (msp / 1e3),
                        "batched_frames_per_s": fm.n_frames / (msb / 1e3),
                        "batched_equals_plain": same_outputs(sp, sb),
                        "waves_per_cu": sb.effective[0], "frames_per_claim": sb.effective[1],
                        "fused_fits": bool(sb.effective[2]), "steal_percent": sb.effective[3]}
        del sp, sb, dm
    if a.align:
        fa = synth.generate(synth.CONFIGS[5])
        da = lib.to_device(fa, dev)
        sa = lib.Selector(fa.n_frames, p, device=dev)
        sa.run(da, stream)
        torch.cuda.synchronize()
        _, tracks, _, _ = sa.lists(fa.layer_offsets)
        trip = np.ascontiguousarray(np.concatenate([tracks[:, [1, 2, 3]], tracks[:, [2, 3, 4]]]), dtype=np.int32)
        tt = torch.from_numpy(trip).to(dev)
        theta = torch.zeros((synth.N_SENSORS, 4), dtype=torch.float32, device=dev)
        gch = torch.ones(len(trip), dtype=torch.float32, device=dev)
        for _ in range(2):
            lib.align_backward(da, tt, theta, p, gch)
        torch.cuda.synchronize()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        for _ in range(a.steps):
            lib.align_chi2(da, tt, theta, p)
        e1.record()
        for _ in range(a.steps):
            lib.align_backward(da, tt, theta, p, gch)
        e2.record()
        e2.synchronize()
        out["align"] = {"workload": f"{fa.n_frames} misaligned frames, {len(trip)} frozen triplets, "
                                    f"{synth.N_SENSORS} sensors x 4 parameters",
                        "forward_ms": e0.elapsed_time(e1) / a.steps, "backward_ms": e1.elapsed_time(e2) / a.steps}
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(fs, p)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
