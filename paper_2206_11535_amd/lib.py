"""Python binding of the C ABI (include/mu3e.h): argument marshalling only.

Device memory and streams come from PyTorch (ROCm); every step of the
selection runs in the HIP kernels of libmu3e.so.  There is no fallback: if the
library is missing, importing the compute entry points raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, replace

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmu3e.so")

KEEP, TRIPLET_OVF, TRACK_OVF, COMBO_OVF, VERTEX, HITS_OVF, LIST_FULL = 1, 2, 4, 8, 16, 32, 64
MAX_LAYER_HITS = 128
STATUS = {0: "ok", -1: "invalid argument", -2: "HIP runtime error", -3: "workspace too small",
          -4: "unsupported parameter"}


class Mu3eError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS.get(status, status)} ({status})")
        self.status = status


class Window(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_float), ("hi", ctypes.c_float)]


class Params(ctypes.Structure):
    _fields_ = [("r_layer", ctypes.c_float * 4), ("z_half", ctypes.c_float * 4),
                ("b_tesla", ctypes.c_float), ("x_over_x0", ctypes.c_float), ("sigma_pixel", ctypes.c_float),
                ("dlambda", Window), ("cosphi01", Window), ("cosphi12", Window), ("rtc_abs", Window),
                ("chi2_track_max", ctypes.c_float),
                ("max_triplets", ctypes.c_int32), ("max_tracks", ctypes.c_int32),
                ("max_combos", ctypes.c_int32), ("max_layer_hits", ctypes.c_int32),
                ("de_max", ctypes.c_float), ("r_target", ctypes.c_float), ("target_tol", ctypes.c_float),
                ("chi2_vertex_max", ctypes.c_float), ("d_target_max", ctypes.c_float),
                ("p_sum_max", ctypes.c_float)]


class Hits(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("layer", ctypes.c_void_p), ("sensor", ctypes.c_void_p),
                ("layer_offsets", ctypes.c_void_p), ("n_frames", ctypes.c_int32),
                ("n_hits", ctypes.c_int32)]


class Tracks(ctypes.Structure):
    _fields_ = [("hit", ctypes.c_void_p), ("frame_offsets", ctypes.c_void_p),
                ("n_frames", ctypes.c_int32), ("n_tracks", ctypes.c_int32)]


class Debug(ctypes.Structure):
    _fields_ = [("counters", ctypes.c_void_p), ("triplets", ctypes.c_void_p), ("tracks", ctypes.c_void_p),
                ("triplet_capacity", ctypes.c_int32), ("track_capacity", ctypes.c_int32),
                ("chunks", ctypes.c_void_p), ("max_chunks", ctypes.c_int32), ("chunk_size", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("waves_per_cu", ctypes.c_int32), ("frames_per_claim", ctypes.c_int32),
                ("fuse_fits", ctypes.c_int32), ("steal_percent", ctypes.c_int32), ("tile_hits", ctypes.c_int32),
                ("sub_batches", ctypes.c_int32)]


def make_params(p: dict) -> Params:
    s = Params()
    for i in range(4):
        s.r_layer[i] = p["r_layer"][i]
        s.z_half[i] = p["z_half"][i]
    s.b_tesla, s.x_over_x0, s.sigma_pixel = p["b_tesla"], p["x_over_x0"], p["sigma_pixel"]
    for name in ("dlambda", "cosphi01", "cosphi12", "rtc_abs"):
        w = getattr(s, name)
        w.lo, w.hi = p[name]
    s.chi2_track_max = p["chi2_track_max"]
    s.max_triplets, s.max_tracks = int(p["max_triplets"]), int(p["max_tracks"])
    s.max_combos, s.max_layer_hits = int(p["max_combos"]), int(p["max_layer_hits"])
    for name in ("de_max", "r_target", "target_tol", "chi2_vertex_max", "d_target_max", "p_sum_max"):
        setattr(s, name, p[name])
    return s


_lib = None


def load(path: str = LIB_PATH):
    """Load libmu3e.so (after torch, so that the process has one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2206_11535_amd.build.build()")
    import torch  # noqa: F401  -- load torch's HIP runtime first
    _lib = declare(ctypes.CDLL(path))
    return _lib


def declare(L):
    """Declares the argument and result types of the C ABI on a loaded
    library handle (no GPU call)."""
    P, I, Z = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    L.mu3e_status_string.restype = ctypes.c_char_p
    L.mu3e_status_string.argtypes = [ctypes.c_int]
    L.mu3e_select_workspace_size.restype = Z
    L.mu3e_select_workspace_size.argtypes = [I, I, I]
    L.mu3e_select_frames.restype = ctypes.c_int
    L.mu3e_select_frames.argtypes = [ctypes.POINTER(Hits), ctypes.POINTER(Params), P, P, P, P, Z, I, I,
                                     ctypes.POINTER(Debug), P]
    L.mu3e_select_frames_timed.restype = ctypes.c_int
    L.mu3e_select_frames_timed.argtypes = [ctypes.POINTER(Hits), ctypes.POINTER(Params), P, P, P, P, Z, I, I,
                                           ctypes.POINTER(Debug), P, P]
    L.mu3e_select_frames_static.restype = ctypes.c_int
    L.mu3e_select_frames_static.argtypes = [ctypes.POINTER(Hits), ctypes.POINTER(Params), P, P, P, I, I,
                                            ctypes.POINTER(Debug), P]
    L.mu3e_chunk_unpack.restype = ctypes.c_int
    L.mu3e_chunk_unpack.argtypes = [P, ctypes.c_int64, I, I, P, P, P, P, P, P]
    L.mu3e_pair_frames.restype = ctypes.c_int
    L.mu3e_pair_frames.argtypes = [ctypes.POINTER(Hits), P, P, P, P, ctypes.c_int64, P]
    L.mu3e_fit_triplets.restype = ctypes.c_int
    L.mu3e_fit_triplets.argtypes = [ctypes.POINTER(Hits), P, I, ctypes.POINTER(Params), P, P]
    L.mu3e_fit_triplets_backward.restype = ctypes.c_int
    L.mu3e_fit_triplets_backward.argtypes = [ctypes.POINTER(Hits), P, I, ctypes.POINTER(Params), P, P, P]
    L.mu3e_vertex_workspace_size.restype = Z
    L.mu3e_vertex_workspace_size.argtypes = [I]
    L.mu3e_vertex.restype = ctypes.c_int
    L.mu3e_vertex.argtypes = [ctypes.POINTER(Hits), ctypes.POINTER(Tracks), ctypes.POINTER(Params), P, P, P, P, Z, P]
    L.mu3e_vertex_debug.restype = ctypes.c_int
    L.mu3e_vertex_debug.argtypes = [ctypes.POINTER(Hits), ctypes.POINTER(Tracks), ctypes.POINTER(Params), P, P, P,
                                    P, Z, P, I, P, P]
    L.mu3e_vertex_refine.restype = ctypes.c_int
    L.mu3e_vertex_refine.argtypes = [ctypes.POINTER(Hits), ctypes.POINTER(Tracks), P, I, P, ctypes.POINTER(Params),
                                     P, P, P, Z, P]
    L.mu3e_plan_create.restype = ctypes.c_int
    L.mu3e_plan_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Hits), ctypes.POINTER(Params),
                                   P, P, P, P, Z, I, I, ctypes.POINTER(Tuning)]
    L.mu3e_plan_run.restype = ctypes.c_int
    L.mu3e_plan_run.argtypes = [P, P]
    L.mu3e_plan_run_timed.restype = ctypes.c_int
    L.mu3e_plan_run_timed.argtypes = [P, P, P]
    L.mu3e_plan_info.restype = ctypes.c_int
    L.mu3e_plan_info.argtypes = [P, ctypes.POINTER(Debug), ctypes.POINTER(Tuning)]
    L.mu3e_plan_workspace_size.restype = Z
    L.mu3e_plan_workspace_size.argtypes = [I, I, I, I]
    L.mu3e_plan_part_info.restype = ctypes.c_int
    L.mu3e_plan_part_info.argtypes = [P, I, ctypes.POINTER(Debug), ctypes.POINTER(I), ctypes.POINTER(I)]
    L.mu3e_plan_destroy.restype = None
    L.mu3e_plan_destroy.argtypes = [P]
    L.mu3e_align_chi2.restype = ctypes.c_int
    L.mu3e_align_chi2.argtypes = [ctypes.POINTER(Hits), P, I, P, I, ctypes.POINTER(Params), P, P]
    L.mu3e_align_workspace_size.restype = Z
    L.mu3e_align_workspace_size.argtypes = [I]
    L.mu3e_align_backward.restype = ctypes.c_int
    L.mu3e_align_backward.argtypes = [ctypes.POINTER(Hits), P, I, P, I, ctypes.POINTER(Params), P, P, P, Z, P]
    return L


def _check(st: int, what: str):
    if st != 0:
        raise Mu3eError(st, what)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype, shape_tail=(), name="tensor"):
    """A GPU tensor argument as the C ABI reads it: row-major contiguous,
    of the given dtype and trailing shape (a contiguous copy is made when
    needed; a wrong dtype, shape or a host tensor raises)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: expected a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name}: expected shape [n, {', '.join(map(str, shape_tail))}], got {tuple(t.shape)}")
    return t.contiguous()


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


@dataclass
class DeviceHits:
    """Hits resident on the GPU (torch tensors) plus the ABI struct."""
    x: object
    y: object
    z: object
    layer: object
    sensor: object
    layer_offsets: object
    n_frames: int
    n_hits: int

    def struct(self) -> Hits:
        return Hits(self.x.data_ptr(), self.y.data_ptr(), self.z.data_ptr(),
                    self.layer.data_ptr() if self.layer is not None else None,
                    self.sensor.data_ptr() if self.sensor is not None else None,
                    self.layer_offsets.data_ptr(), self.n_frames, self.n_hits)


def to_device(fs, device="cuda") -> DeviceHits:
    import torch
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).astype(dt, copy=False)).to(device)
    layer = t(fs.layer.astype(np.int16), np.int16) if getattr(fs, "layer", None) is not None else None
    sensor = t(fs.sensor.astype(np.int16), np.int16) if getattr(fs, "sensor", None) is not None else None
    return DeviceHits(t(fs.x, np.float32), t(fs.y, np.float32), t(fs.z, np.float32), layer, sensor,
                      t(fs.layer_offsets, np.int32), int(fs.n_frames), int(len(fs.x)))


class Selector:
    """Preallocated outputs and workspace for repeated mu3e_select_frames calls."""

    def __init__(self, n_frames: int, params: dict, triplet_capacity: int | None = None,
                 track_capacity: int | None = None, device="cuda"):
        import torch
        L = load()
        self.n_frames = n_frames
        self.params = make_params(params)
        self.tcap = int(triplet_capacity if triplet_capacity is not None else 128 * n_frames + 65536)
        self.kcap = int(track_capacity if track_capacity is not None else 16 * n_frames + 4096)
        nb = self._workspace_bytes()
        if nb == 0 and n_frames > 0:
            raise Mu3eError(-1, "workspace size")
        self.ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=device)
        self.flags = torch.empty(max(n_frames, 1), dtype=torch.int32, device=device)
        self.counts = torch.empty((max(n_frames, 1), 3), dtype=torch.int32, device=device)
        self.vertex = torch.empty((max(n_frames, 1), 4), dtype=torch.float32, device=device)
        self.dbg = Debug()

    def _workspace_bytes(self) -> int:
        return load().mu3e_select_workspace_size(self.n_frames, self.tcap, self.kcap)

    def run(self, hits: DeviceHits, stream=None, events=None):
        """events: optional ctypes array of 5 hipEvent_t recorded between the
        stage kernels."""
        L = load()
        if hits.n_frames != self.n_frames:
            raise ValueError(f"hits hold {hits.n_frames} frames; the selector's outputs are sized for "
                             f"{self.n_frames}")
        hs = hits.struct()
        if events is None:
            st = L.mu3e_select_frames(ctypes.byref(hs), ctypes.byref(self.params), _ptr(self.flags),
                                      _ptr(self.counts), _ptr(self.vertex), _ptr(self.ws), self.ws.numel(),
                                      self.tcap, self.kcap, ctypes.byref(self.dbg), _stream(stream))
        else:
            st = L.mu3e_select_frames_timed(ctypes.byref(hs), ctypes.byref(self.params), _ptr(self.flags),
                                            _ptr(self.counts), _ptr(self.vertex), _ptr(self.ws),
                                            self.ws.numel(), self.tcap, self.kcap, ctypes.byref(self.dbg),
                                            _stream(stream), ctypes.cast(events, ctypes.c_void_p))
        _check(st, "mu3e_select_frames")

    def _parts(self):
        """(debug view, first frame) of each independent part of the
        workspace: one for the plain form."""
        return [(self.dbg, 0)]

    def _counters_of(self, d):
        import torch
        n = 11
        base = d.counters - self.ws.data_ptr()
        return self.ws[base:base + 4 * n].view(torch.int32).cpu().numpy()

    def counters(self):
        """Device counters (synchronises): [0] triplets selected, [2] status
        bits, [7] triplet entries handed out in chunks, ...; over the parts
        of a batched plan: [0] summed, [2] or-ed, the rest those of part 0."""
        cs = [self._counters_of(d) for d, _ in self._parts()]
        c = cs[0].copy()
        c[0] = sum(int(x[0]) for x in cs)
        c[2] = np.bitwise_or.reduce([int(x[2]) for x in cs])
        return c

    def lists(self, hits_offsets: np.ndarray):
        """Host copies of the selected triplets and the accepted tracks
        (global hit indices); triplets of frames flagged TRIPLET_OVF are left
        out.  Returns (triplets [n, 4]: frame, h0, h1, h2; tracks [m, 5]:
        frame, h0..h3; kf [m, 2]: kappa_bar, chi2; counters)."""
        import torch
        ws = self.ws
        trips_l, res_l = [], []
        for d, first in self._parts():
            c = self._counters_of(d)
            nch = min(int(c[7]), d.triplet_capacity) // d.chunk_size if d.chunk_size > 0 else 0
            cb = d.chunks - ws.data_ptr()
            ch = ws[cb:cb + 16 * nch].view(torch.int32).cpu().numpy().reshape(-1, 4)
            tb = d.triplets - ws.data_ptr()
            allt = ws[tb:tb + 8 * d.triplet_capacity].view(torch.int32).cpu().numpy().reshape(-1, 2)
            rb = d.tracks - ws.data_ptr()
            allr = ws[rb:rb + 16 * d.triplet_capacity].view(torch.int32).cpu().numpy().reshape(-1, 4)
            idx = np.concatenate([np.arange(a, a + n) for a, n in ch[:, :2]]) if nch else np.zeros(0, np.int64)
            t = allt[idx].copy()
            t[:, 0] += first
            trips_l.append(t)
            res_l.append(allr[idx])
        trips, res = np.concatenate(trips_l), np.concatenate(res_l)
        flags = self.flags[:self.n_frames].cpu().numpy().view(np.uint32)
        keep = (flags[trips[:, 0]] & TRIPLET_OVF) == 0 if len(trips) else np.zeros(0, bool)
        trips, res = trips[keep], res[keep]
        lo = np.asarray(hits_offsets)
        f = trips[:, 0].astype(np.int64)
        pk = trips[:, 1].astype(np.int64)
        g = np.stack([lo[4 * f] + (pk & 0x3ff), lo[4 * f + 1] + ((pk >> 10) & 0x3ff),
                      lo[4 * f + 2] + (pk >> 20)], 1)
        triplets = np.concatenate([f[:, None], g], 1)
        acc = res[:, 0] == 1
        tracks = np.concatenate([triplets[acc], (lo[4 * f[acc] + 3] + res[acc, 1])[:, None]], 1)
        kf = res[acc, 2:4].copy().view(np.float32)
        return triplets, tracks, kf, self.counters()

    def result(self):
        F = self.n_frames
        return (self.flags[:F].cpu().numpy().view(np.uint32), self.counts[:F].cpu().numpy(),
                self.vertex[:F].cpu().numpy())


class BatchedSelector(Selector):
    """The batched persistent form (mu3e_plan_*): per sub-batch two hipGraph
    launches (cuts; fits and vertex stage).  Same outputs as Selector; the
    plan binds `hits`."""

    def __init__(self, hits: DeviceHits, params: dict, triplet_capacity: int | None = None,
                 track_capacity: int | None = None, device="cuda", waves_per_cu: int = 0,
                 frames_per_claim: int = 0, fuse_fits: int = 0, steal_percent: int = 0, tile_hits: int = 0,
                 sub_batches: int = 0):
        self.sub_batches = int(sub_batches)
        super().__init__(hits.n_frames, params, triplet_capacity, track_capacity, device)
        L = load()
        self.hits = hits
        self._hs = hits.struct()
        self.tuning = Tuning(int(waves_per_cu), int(frames_per_claim), int(fuse_fits), int(steal_percent),
                             int(tile_hits), self.sub_batches)
        plan = ctypes.c_void_p()
        _check(L.mu3e_plan_create(ctypes.byref(plan), ctypes.byref(self._hs), ctypes.byref(self.params),
                                  _ptr(self.flags), _ptr(self.counts), _ptr(self.vertex), _ptr(self.ws),
                                  self.ws.numel(), self.tcap, self.kcap, ctypes.byref(self.tuning)),
               "mu3e_plan_create")
        self.plan = plan
        eff = Tuning()
        _check(L.mu3e_plan_info(self.plan, ctypes.byref(self.dbg), ctypes.byref(eff)), "mu3e_plan_info")
        self.effective = (eff.waves_per_cu, eff.frames_per_claim, eff.fuse_fits, eff.steal_percent, eff.tile_hits,
                          eff.sub_batches)
        self.parts = []
        for j in range(eff.sub_batches):
            d, first, n = Debug(), ctypes.c_int32(), ctypes.c_int32()
            _check(L.mu3e_plan_part_info(self.plan, j, ctypes.byref(d), ctypes.byref(first), ctypes.byref(n)),
                   "mu3e_plan_part_info")
            self.parts.append((d, first.value, n.value))

    def _workspace_bytes(self) -> int:
        return load().mu3e_plan_workspace_size(self.n_frames, self.tcap, self.kcap, self.sub_batches)

    def _parts(self):
        return [(d, first) for d, first, _ in self.parts]

    def tuning_dict(self) -> dict:
        """The shape in effect (after the occupancy and frame-count caps)."""
        keys = ("waves_per_cu", "frames_per_claim", "fuse_fits", "steal_percent", "tile_hits", "sub_batches")
        return dict(zip(keys, (int(v) for v in self.effective)))

    def run(self, hits: DeviceHits = None, stream=None, events=None):
        """events: optional ctypes array of 4 hipEvent_t per sub-batch; then
        the plan's kernels are launched directly (no graph, the sub-batches
        one after another) with the events around each sub-batch's
        persistent kernel and fit kernel (mu3e_plan_run_timed)."""
        if hits is not None and hits is not self.hits:
            raise ValueError("a plan is bound to the hits it was created with")
        if events is None:
            _check(load().mu3e_plan_run(self.plan, _stream(stream)), "mu3e_plan_run")
        else:
            if len(events) < 4 * len(self.parts):
                raise ValueError(f"{len(events)} events for {len(self.parts)} sub-batches (4 each)")
            _check(load().mu3e_plan_run_timed(self.plan, _stream(stream), ctypes.cast(events, ctypes.c_void_p)),
                   "mu3e_plan_run_timed")

    def __del__(self):
        plan = getattr(self, "plan", None)
        if plan is not None and _lib is not None:
            _lib.mu3e_plan_destroy(plan)
            self.plan = None


def pair_frames(hits: DeviceHits, stream=None) -> DeviceHits:
    """The overlapping frame pairs of a batch (mu3e_pair_frames): merged
    frame g holds, per layer, frame g's hits and then frame g + 1's.  The
    returned hits are sized for 2 * n_hits; their n_hits is that capacity
    (the offsets hold the real count)."""
    import torch
    if hits.n_frames < 2:
        raise ValueError("frame pairs need at least two frames")
    cap = 2 * hits.n_hits
    dev = hits.x.device
    x = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    lo = torch.empty(4 * (hits.n_frames - 1) + 1, dtype=torch.int32, device=dev)
    hs = hits.struct()
    _check(load().mu3e_pair_frames(ctypes.byref(hs), _ptr(x), _ptr(y), _ptr(z), _ptr(lo), cap, _stream(stream)),
           "mu3e_pair_frames")
    return DeviceHits(x, y, z, None, None, lo, hits.n_frames - 1, cap)


# ------------------------------------------------------------ chunk ingest
def chunk_capacity(chunk_bytes: int, max_frames: int) -> int:
    """Most hit records a chunk of chunk_bytes holds with max_frames frames."""
    return max(0, (int(chunk_bytes) // 4 * 4 - 4 - 4 * (4 * int(max_frames) + 1)) // 12)


def pack_chunk(fs, f0: int, f1: int, out: np.ndarray) -> int:
    """Writes frames [f0, f1) of a host FrameSet into the chunk buffer `out`
    (uint8, as the readout would: records {x, y, z} float32 from the front,
    the layer offsets and the frame count at the tail; see mu3e.h).  Returns
    the number of hits written; raises if the frames do not fit."""
    lo = np.asarray(fs.layer_offsets)
    h0, h1 = int(lo[4 * f0]), int(lo[4 * f1])
    F, n = f1 - f0, h1 - h0
    nb = len(out) // 4 * 4
    tail = 4 + 4 * (4 * F + 1)
    if 12 * n + tail > nb:
        raise ValueError(f"{F} frames with {n} hits need {12 * n + tail} bytes; the chunk has {nb}")
    rec = out[:12 * n].view(np.float32).reshape(n, 3)
    rec[:, 0] = fs.x[h0:h1]
    rec[:, 1] = fs.y[h0:h1]
    rec[:, 2] = fs.z[h0:h1]
    t = out[nb - tail:nb].view(np.int32)
    t[:-1] = lo[4 * f0:4 * f1 + 1] - h0
    t[-1] = F
    return n


class ChunkStream:
    """Chunk ingest with overlapped copies (Sections V-A, V-B): n_buffers
    slots, each with a pinned host chunk, a device chunk, SoA hit buffers
    and a selection bound to them (the batched plan, or the plain form), and
    its own stream.  submit() fills the next slot's pinned chunk through
    `fill(view)` (the readout writing into host memory), then queues on the
    slot's stream: the copy to the GPU (of the records and the tail only,
    as the tail in host memory gives them), mu3e_chunk_unpack, the selection
    and the copy of the frame flags back; so one chunk's copies overlap
    another chunk's selection.  A slot is reused once its previous chunk is
    done.  Four slots keep the copy engine busy (with three the loop ran at
    half the rate, waiting on slots)."""

    def __init__(self, params: dict, chunk_bytes: int, max_frames: int, n_buffers: int = 4, form: str = "batched",
                 triplet_capacity: int | None = None, track_capacity: int | None = None, tuning: dict | None = None,
                 device="cuda"):
        import torch
        L = load()
        self.chunk_bytes = int(chunk_bytes) // 16 * 16
        self.max_frames = int(max_frames)
        self.max_hits = chunk_capacity(self.chunk_bytes, self.max_frames)
        if self.max_hits <= 0:
            raise ValueError("chunk too small for its frame table")
        self.params = params
        self.slots = []
        for _ in range(int(n_buffers)):
            host = torch.empty(self.chunk_bytes, dtype=torch.uint8, pin_memory=True)
            dchunk = torch.empty(self.chunk_bytes, dtype=torch.uint8, device=device)
            x = torch.zeros(self.max_hits, dtype=torch.float32, device=device)
            y = torch.zeros_like(x)
            z = torch.zeros_like(x)
            lo = torch.zeros(4 * self.max_frames + 1, dtype=torch.int32, device=device)
            info = torch.zeros(2, dtype=torch.int32, device=device)
            hits = DeviceHits(x, y, z, None, None, lo, self.max_frames, self.max_hits)
            if form == "batched":
                sel = BatchedSelector(hits, params, triplet_capacity, track_capacity, device=device, **(tuning or {}))
            elif form == "plain":
                sel = Selector(self.max_frames, params, triplet_capacity, track_capacity, device=device)
            else:
                raise ValueError(f"form {form!r}: 'batched' or 'plain'")
            out_flags = torch.empty(self.max_frames, dtype=torch.int32, pin_memory=True)
            out_info = torch.empty(2, dtype=torch.int32, pin_memory=True)
            self.slots.append(dict(host=host, dchunk=dchunk, hits=hits, info=info, sel=sel, stream=torch.cuda.Stream(device),
                                   event=None, out_flags=out_flags, out_info=out_info))
        self.next = 0
        self.L = L

    def submit(self, fill) -> int:
        """fill(host_view: np.ndarray uint8) writes a chunk into the next
        slot's pinned buffer; returns the slot index (for result())."""
        import torch
        k = self.next
        self.next = (k + 1) % len(self.slots)
        sl = self.slots[k]
        if sl["event"] is not None:
            sl["event"].synchronize()   # the slot's previous chunk is done
        buf = sl["host"].numpy()
        fill(buf)
        front, tail = self._used(buf)
        st = sl["stream"]
        with torch.cuda.stream(st):
            if front is None:   # an inconsistent tail: the whole buffer, for mu3e_chunk_unpack to reject
                sl["dchunk"].copy_(sl["host"], non_blocking=True)
            else:               # only the records and the tail (the space between is never read)
                nb = self.chunk_bytes
                if front > 0:
                    sl["dchunk"][:front].copy_(sl["host"][:front], non_blocking=True)
                sl["dchunk"][nb - tail:].copy_(sl["host"][nb - tail:], non_blocking=True)
            h = sl["hits"]
            _check(self.L.mu3e_chunk_unpack(_ptr(sl["dchunk"]), self.chunk_bytes, self.max_frames, self.max_hits,
                                            _ptr(h.x), _ptr(h.y), _ptr(h.z), _ptr(h.layer_offsets), _ptr(sl["info"]),
                                            _stream(st)), "mu3e_chunk_unpack")
            if isinstance(sl["sel"], BatchedSelector):
                sl["sel"].run(None, st)
            else:
                sl["sel"].run(h, st)
            sl["out_flags"].copy_(sl["sel"].flags[:self.max_frames], non_blocking=True)
            sl["out_info"].copy_(sl["info"], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        sl["event"] = ev
        return k

    def _used(self, buf):
        """(front, tail) bytes a filled chunk uses, read from its tail in host
        memory: the records of offsets[4F] hits and the tail of 4F + 2 int32;
        (None, None) if the tail does not describe a chunk of this buffer."""
        nb = self.chunk_bytes
        F = int(buf[nb - 4:nb].view(np.int32)[0])
        if not 0 <= F <= self.max_frames:
            return None, None
        tail = 4 * (4 * F + 2)
        n = int(buf[nb - 8:nb - 4].view(np.int32)[0])
        if n < 0 or 12 * n + tail > nb:
            return None, None
        return 12 * n, tail

    def result(self, k: int):
        """(frames, flags[frames]) of the chunk last submitted to slot k
        (waits for it); frames = -1 for a malformed chunk."""
        sl = self.slots[k]
        sl["event"].synchronize()
        F = int(sl["out_info"][0])
        return F, sl["out_flags"].numpy()[:max(F, 0)].view(np.uint32).copy()

    def synchronize(self):
        for sl in self.slots:
            if sl["event"] is not None:
                sl["event"].synchronize()


def select_frames(hits: DeviceHits, params: dict, stream=None, **kw):
    s = Selector(hits.n_frames, params, **kw)
    s.run(hits, stream)
    return s


def select_frames_static(hits: DeviceHits, params: dict, triplet_capacity: int, track_capacity: int,
                         flags=None, counts=None, vertex=None, stream=None):
    """mu3e_select_frames_static: the selection with the library's static
    per-GPU workspace (the call itself allocates nothing; outputs are
    allocated here unless given).  Returns (flags, counts, vertex) tensors."""
    import torch
    F = hits.n_frames
    dev = hits.x.device
    flags = torch.empty(max(F, 1), dtype=torch.int32, device=dev) if flags is None else flags
    counts = torch.empty((max(F, 1), 3), dtype=torch.int32, device=dev) if counts is None else counts
    vertex = torch.empty((max(F, 1), 4), dtype=torch.float32, device=dev) if vertex is None else vertex
    if flags.numel() < F or counts.numel() < 3 * F or vertex.numel() < 4 * F:
        raise ValueError("output tensors too small for the frames")
    hs = hits.struct()
    dbg = Debug()
    _check(load().mu3e_select_frames_static(ctypes.byref(hs), ctypes.byref(make_params(params)), _ptr(flags),
                                            _ptr(counts), _ptr(vertex), int(triplet_capacity),
                                            int(track_capacity), ctypes.byref(dbg), _stream(stream)),
           "mu3e_select_frames_static")
    return flags, counts, vertex


def fit_triplets(hits: DeviceHits, trip, params: dict, stream=None):
    """trip: int32 cuda tensor [n, 3] of global hit indices -> float32 [n, 8]."""
    import torch
    L = load()
    trip = _dev(trip, torch.int32, (3,), "trip")
    n = int(trip.shape[0])
    out = torch.empty((max(n, 1), 8), dtype=torch.float32, device=trip.device)
    hs = hits.struct()
    pp = make_params(params)
    _check(L.mu3e_fit_triplets(ctypes.byref(hs), _ptr(trip), n, ctypes.byref(pp), _ptr(out), _stream(stream)),
           "mu3e_fit_triplets")
    return out[:n]


def fit_triplets_backward(hits: DeviceHits, trip, params: dict, grad_chi2, grad_xyz=None, stream=None):
    """d(sum_t grad_chi2[t] chi2_t) / d(hit x, y, z), float32 [n_hits, 3]
    (added to grad_xyz when given, else to a new zero tensor)."""
    import torch
    L = load()
    trip = _dev(trip, torch.int32, (3,), "trip")
    grad_chi2 = _dev(grad_chi2, torch.float32, (), "grad_chi2")
    n = int(trip.shape[0])
    if int(grad_chi2.shape[0]) != n:
        raise ValueError("grad_chi2: one entry per triplet expected")
    if grad_xyz is None:
        grad_xyz = torch.zeros((max(hits.n_hits, 1), 3), dtype=torch.float32, device=trip.device)
    elif (not isinstance(grad_xyz, torch.Tensor) or grad_xyz.dtype != torch.float32 or not grad_xyz.is_cuda
          or tuple(grad_xyz.shape) != (hits.n_hits, 3) or not grad_xyz.is_contiguous()):
        raise ValueError("grad_xyz: a contiguous float32 GPU tensor [n_hits, 3] expected")
    hs = hits.struct()
    pp = make_params(params)
    _check(L.mu3e_fit_triplets_backward(ctypes.byref(hs), _ptr(trip), n, ctypes.byref(pp), _ptr(grad_chi2),
                                        _ptr(grad_xyz), _stream(stream)), "mu3e_fit_triplets_backward")
    return grad_xyz[:hits.n_hits]


def vertex(hits: DeviceHits, track_hits, frame_offsets, params: dict, stream=None, triple_capacity: int = 0):
    """track_hits int32 [n, 4], frame_offsets int32 [F+1] (cuda tensors) ->
    (flags [F], combos [F], vertex [F, 4]); with triple_capacity > 0 also
    the energy-passing triples (mu3e_vertex_debug): int32 [m, 4] rows
    {frame, e+ track, e+ track, e- track} and the true count m' >= m."""
    import torch
    L = load()
    track_hits = _dev(track_hits, torch.int32, (4,), "track_hits")
    frame_offsets = _dev(frame_offsets, torch.int32, (), "frame_offsets")
    F = int(frame_offsets.shape[0]) - 1
    n = int(track_hits.shape[0])
    dev = frame_offsets.device
    flags = torch.empty(max(F, 1), dtype=torch.int32, device=dev)
    combos = torch.empty(max(F, 1), dtype=torch.int32, device=dev)
    vtx = torch.empty((max(F, 1), 4), dtype=torch.float32, device=dev)
    nb = L.mu3e_vertex_workspace_size(n)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
    hs = hits.struct()
    tr = Tracks(track_hits.data_ptr() if n else None, frame_offsets.data_ptr(), F, n)
    pp = make_params(params)
    if triple_capacity <= 0:
        _check(L.mu3e_vertex(ctypes.byref(hs), ctypes.byref(tr), ctypes.byref(pp), _ptr(flags), _ptr(combos),
                             _ptr(vtx), _ptr(ws), ws.numel(), _stream(stream)), "mu3e_vertex")
        return flags[:F], combos[:F], vtx[:F]
    rows = torch.empty((int(triple_capacity), 4), dtype=torch.int32, device=dev)
    nrow = torch.zeros(1, dtype=torch.int32, device=dev)
    _check(L.mu3e_vertex_debug(ctypes.byref(hs), ctypes.byref(tr), ctypes.byref(pp), _ptr(flags), _ptr(combos),
                               _ptr(vtx), _ptr(ws), ws.numel(), _ptr(rows), int(triple_capacity), _ptr(nrow),
                               _stream(stream)), "mu3e_vertex_debug")
    m = int(nrow.item())
    return flags[:F], combos[:F], vtx[:F], rows[:min(m, int(triple_capacity))], m


REFINE_FIELDS = ("x", "y", "z", "J", "rough_x", "rough_y", "rough_z", "rough_chi2")


def vertex_refine(hits: DeviceHits, track_hits, rows, params: dict, n_valid=None, stream=None):
    """Refined vertex of listed e+e+e- track triples (mu3e_vertex_refine):
    track_hits int32 [n_tracks, 4], rows int32 [n, 4] {frame, a, b, c} (the
    rows vertex(..., triple_capacity) returns), optional n_valid (an int32
    cuda tensor [1] bounding the rows read) -> (out float64 [n, 8] with
    REFINE_FIELDS, status int32 [n]: steps used, 0 no rough vertex, -1 no
    convergence, -2 invalid track)."""
    import torch
    L = load()
    track_hits = _dev(track_hits, torch.int32, (4,), "track_hits")
    rows = _dev(rows, torch.int32, (4,), "rows")
    if n_valid is not None:
        n_valid = _dev(n_valid, torch.int32, (), "n_valid")
    n, nt = int(rows.shape[0]), int(track_hits.shape[0])
    dev = rows.device
    out = torch.full((max(n, 1), 8), float("nan"), dtype=torch.float64, device=dev)
    status = torch.full((max(n, 1),), -3, dtype=torch.int32, device=dev)
    ws = torch.empty(max(L.mu3e_vertex_workspace_size(nt), 256), dtype=torch.uint8, device=dev)
    hs = hits.struct()
    tr = Tracks(track_hits.data_ptr() if nt else None, None, 0, nt)
    pp = make_params(params)
    _check(L.mu3e_vertex_refine(ctypes.byref(hs), ctypes.byref(tr), _ptr(rows) if n else None, n,
                                _ptr(n_valid) if n_valid is not None else None, ctypes.byref(pp), _ptr(out),
                                _ptr(status), _ptr(ws), ws.numel(), _stream(stream)), "mu3e_vertex_refine")
    return out[:n], status[:n]


def align_chi2(hits: DeviceHits, trip, theta, params: dict, stream=None):
    """Triplet-fit chi2 [n] after per-sensor alignment theta [S, 4] (float32
    cuda tensors; trip int32 [n, 3])."""
    import torch
    L = load()
    trip = _dev(trip, torch.int32, (3,), "trip")
    theta = _dev(theta, torch.float32, (4,), "theta")
    n = int(trip.shape[0])
    out = torch.empty(max(n, 1), dtype=torch.float32, device=theta.device)
    hs = hits.struct()
    pp = make_params(params)
    _check(L.mu3e_align_chi2(ctypes.byref(hs), _ptr(trip), n, _ptr(theta), int(theta.shape[0]), ctypes.byref(pp),
                             _ptr(out), _stream(stream)), "mu3e_align_chi2")
    return out[:n]


def align_backward(hits: DeviceHits, trip, theta, params: dict, grad_chi2, stream=None):
    """d(sum_t grad_chi2[t] chi2_t) / d theta, float32 [S, 4]."""
    import torch
    L = load()
    trip = _dev(trip, torch.int32, (3,), "trip")
    theta = _dev(theta, torch.float32, (4,), "theta")
    grad_chi2 = _dev(grad_chi2, torch.float32, (), "grad_chi2")
    n = int(trip.shape[0])
    if int(grad_chi2.shape[0]) != n:
        raise ValueError("grad_chi2: one entry per triplet expected")
    S = int(theta.shape[0])
    nb = L.mu3e_align_workspace_size(S)
    if nb == 0:
        raise Mu3eError(-4, "mu3e_align_workspace_size")
    ws = torch.empty(nb, dtype=torch.uint8, device=theta.device)
    g = torch.empty((S, 4), dtype=torch.float32, device=theta.device)
    hs = hits.struct()
    pp = make_params(params)
    _check(L.mu3e_align_backward(ctypes.byref(hs), _ptr(trip), n, _ptr(theta), S, ctypes.byref(pp),
                                 _ptr(grad_chi2), _ptr(g), _ptr(ws), ws.numel(), _stream(stream)),
           "mu3e_align_backward")
    return g


def _autograd():
    import torch

    class AlignChi2(torch.autograd.Function):
        """chi2[n] of frozen triplets as a function of the per-sensor
        alignment theta [S, 4] = (tx, ty, tz, alpha); backward is the
        hand-written adjoint of the fit (mu3e_align_backward)."""

        @staticmethod
        def forward(ctx, theta, hits, trip, params):
            theta = theta.detach().contiguous().float()
            ctx.hits, ctx.trip, ctx.params = hits, trip, params
            ctx.save_for_backward(theta)
            return align_chi2(hits, trip, theta, params)

        @staticmethod
        def backward(ctx, grad_chi2):
            (theta,) = ctx.saved_tensors
            g = align_backward(ctx.hits, ctx.trip, theta, ctx.params, grad_chi2.contiguous().float())
            return g, None, None, None

    return AlignChi2


_align_fn = None


def align_chi2_autograd(theta, hits: DeviceHits, trip, params: dict):
    """Differentiable chi2[n] (torch.autograd.Function around the C ABI)."""
    global _align_fn
    if _align_fn is None:
        _align_fn = _autograd()
    return _align_fn.apply(theta, hits, trip, params)


def _fit_autograd():
    import torch

    class FitChi2(torch.autograd.Function):
        """chi2_min[n] of explicit triplets as a function of the hit
        coordinates x, y, z [n_hits] (float32 GPU tensors); forward is
        mu3e_fit_triplets, backward the hand-written adjoint
        (mu3e_fit_triplets_backward).  Degenerate triplets give NaN and no
        gradient."""

        @staticmethod
        def forward(ctx, x, y, z, hits, trip, params):
            h = replace(hits, x=x.detach().contiguous().float(), y=y.detach().contiguous().float(),
                        z=z.detach().contiguous().float())
            ctx.h, ctx.trip, ctx.params = h, trip, params
            return fit_triplets(h, trip, params)[:, 2].contiguous()

        @staticmethod
        def backward(ctx, grad_chi2):
            g = fit_triplets_backward(ctx.h, ctx.trip, ctx.params, grad_chi2.contiguous().float())
            return g[:, 0].contiguous(), g[:, 1].contiguous(), g[:, 2].contiguous(), None, None, None

    return FitChi2


_fit_fn = None


def fit_chi2_autograd(x, y, z, hits: DeviceHits, trip, params: dict):
    """Differentiable chi2_min[n] of the triplets trip [n, 3] with respect to
    the hit coordinates x, y, z [n_hits] (torch.autograd.Function around the
    C ABI; the other fields of `hits` are taken as they are)."""
    import torch
    for name, t in (("x", x), ("y", y), ("z", z)):
        if (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32
                or tuple(t.shape) != (hits.n_hits,)):
            raise ValueError(f"{name}: a float32 GPU tensor [n_hits] = [{hits.n_hits}] expected")
    global _fit_fn
    if _fit_fn is None:
        _fit_fn = _fit_autograd()
    return _fit_fn.apply(x, y, z, hits, trip, params)
