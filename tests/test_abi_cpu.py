"""The C-ABI library without a GPU: it loads, exports every function that
include/mu3e.h declares, and rejects bad arguments on the host before any
launch (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mu3e.h")


@pytest.fixture(scope="module")
def L():
    from paper_2206_11535_amd import lib
    if not os.path.exists(lib.LIB_PATH):
        from paper_2206_11535_amd import build
        build.build()
    return lib.load()


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mu3e_[a-z_0-9]+)\s*\(", txt)))


def test_exports_every_declared_symbol(L):
    names = declared()
    assert {"mu3e_select_frames", "mu3e_fit_triplets", "mu3e_vertex"} <= set(names)
    for n in names:
        assert hasattr(L, n), n


def test_status_strings(L):
    assert L.mu3e_status_string(0) == b"ok"
    assert b"invalid" in L.mu3e_status_string(-1)
    assert L.mu3e_status_string(-3) == b"workspace too small"


def test_workspace_sizes(L):
    assert L.mu3e_select_workspace_size(-1, 10, 10) == 0
    a = L.mu3e_select_workspace_size(1000, 64000, 16000)
    b = L.mu3e_select_workspace_size(2000, 64000, 16000)
    assert 0 < a < b and a % 256 == 0
    assert L.mu3e_vertex_workspace_size(-5) == 0
    assert L.mu3e_vertex_workspace_size(100) > L.mu3e_vertex_workspace_size(10)


def _hits(lib, F):
    # dummy non-null device-pointer stand-ins: never dereferenced, every call
    # below fails validation before any launch
    return lib.Hits(16, 32, 48, None, None, 64, F, 10)


def test_host_validation(L):
    from paper_2206_11535_amd import lib
    from paper_2206_11535_amd.params import default_params
    p = lib.make_params(default_params())
    dbg = lib.Debug()
    h = _hits(lib, 5)
    # null hits
    assert L.mu3e_select_frames(None, ctypes.byref(p), 1, 1, 1, 1, 1 << 30, 10, 10, None, None) == -1
    # workspace too small
    assert L.mu3e_select_frames(ctypes.byref(h), ctypes.byref(p), 1, 1, 1, 1, 16, 10, 10, None, None) == -3
    # unsupported layer capacity
    q = lib.make_params(default_params(max_layer_hits=1024))
    assert L.mu3e_select_frames(ctypes.byref(h), ctypes.byref(q), 1, 1, 1, 1, 1 << 30, 10, 10, None, None) == -4
    # inverted window, negative cap, bad radii
    for bad in (dict(dlambda=(0.5, -0.5)), dict(max_tracks=-1), dict(r_layer=(25.0, 24.0, 73.0, 85.0))):
        q = lib.make_params(default_params(**bad))
        assert L.mu3e_select_frames(ctypes.byref(h), ctypes.byref(q), 1, 1, 1, 1, 1 << 30, 10, 10,
                                    ctypes.byref(dbg), None) == -1
    # negative capacities / frames
    assert L.mu3e_select_frames(ctypes.byref(h), ctypes.byref(p), 1, 1, 1, 1, 1 << 30, -1, 10, None, None) == -1
    h2 = _hits(lib, -1)
    assert L.mu3e_select_frames(ctypes.byref(h2), ctypes.byref(p), 1, 1, 1, 1, 1 << 30, 10, 10, None, None) == -1
    # fit: negative n, null triplets
    assert L.mu3e_fit_triplets(ctypes.byref(h), None, -1, ctypes.byref(p), None, None) == -1
    assert L.mu3e_fit_triplets(ctypes.byref(h), None, 5, ctypes.byref(p), 1, None) == -1
    assert L.mu3e_fit_triplets_backward(ctypes.byref(h), None, -1, ctypes.byref(p), None, None, None) == -1
    assert L.mu3e_fit_triplets_backward(ctypes.byref(h), None, 5, ctypes.byref(p), 1, 1, None) == -1
    assert L.mu3e_fit_triplets_backward(None, None, 0, ctypes.byref(p), None, None, None) == -1
    # vertex: null tracks, too small workspace
    assert L.mu3e_vertex(ctypes.byref(h), None, ctypes.byref(p), 1, 1, 1, 1, 1 << 20, None) == -1
    tr = lib.Tracks(80, 96, 4, 1000)
    assert L.mu3e_vertex(ctypes.byref(h), ctypes.byref(tr), ctypes.byref(p), 1, 1, 1, 1, 8, None) == -3
    # refined vertex: null rows or outputs, negative count, too small workspace
    tr = lib.Tracks(80, 96, 4, 1000)
    assert L.mu3e_vertex_refine(ctypes.byref(h), ctypes.byref(tr), None, 5, None, ctypes.byref(p), 1, 1, 1,
                                1 << 20, None) == -1
    assert L.mu3e_vertex_refine(ctypes.byref(h), ctypes.byref(tr), 1, -1, None, ctypes.byref(p), 1, 1, 1,
                                1 << 20, None) == -1
    assert L.mu3e_vertex_refine(ctypes.byref(h), ctypes.byref(tr), 1, 5, None, ctypes.byref(p), None, 1, 1,
                                1 << 20, None) == -1
    assert L.mu3e_vertex_refine(ctypes.byref(h), None, 1, 5, None, ctypes.byref(p), 1, 1, 1, 1 << 20, None) == -1
    assert L.mu3e_vertex_refine(ctypes.byref(h), ctypes.byref(tr), 1, 5, None, ctypes.byref(p), 1, 1, 1, 8,
                                None) == -3
    assert L.mu3e_vertex_refine(ctypes.byref(h), ctypes.byref(tr), None, 0, None, ctypes.byref(p), None, None,
                                None, 0, None) == 0
    # triplet capacity beyond 2^30
    assert L.mu3e_select_workspace_size(10, (1 << 30) + 1, 10) == 0
    assert L.mu3e_select_frames(ctypes.byref(h), ctypes.byref(p), 1, 1, 1, 1, 1 << 30, (1 << 30) + 1, 10, None,
                                None) == -1
    # the static-workspace entry: a request beyond the library's array, and
    # negative sizes, are refused before any device call
    assert L.mu3e_select_frames_static(ctypes.byref(h), ctypes.byref(p), 1, 1, 1, 1 << 30, 1 << 20, None,
                                       None) == -3
    assert L.mu3e_select_frames_static(ctypes.byref(h), ctypes.byref(p), 1, 1, 1, -1, 10, None, None) == -1
    assert L.mu3e_select_frames_static(ctypes.byref(h2), ctypes.byref(p), 1, 1, 1, 10, 10, None, None) == -1
    assert L.mu3e_select_frames_static(None, ctypes.byref(p), 1, 1, 1, 10, 10, None, None) == -1
    # plan: null out pointer, invalid steal share (checked before any device call)
    t = lib.Tuning(8, 4, 0, 101)
    assert L.mu3e_plan_create(None, ctypes.byref(h), ctypes.byref(p), 1, 1, 1, 1, 1 << 30, 10, 10,
                              ctypes.byref(t)) == -1
    plan = ctypes.c_void_p()
    assert L.mu3e_plan_create(ctypes.byref(plan), ctypes.byref(h), ctypes.byref(p), 1, 1, 1, 1, 1 << 30, 10, 10,
                              ctypes.byref(t)) == -1
    assert plan.value is None
    # timed plan run without a plan or events
    assert L.mu3e_plan_run_timed(None, None, None) == -1
    # a negative hit count is refused by every entry point that reads hits,
    # before any launch (with n_hits < 0 an index check (unsigned)g < n_hits
    # in the kernels would otherwise accept negative indices)
    hn = lib.Hits(16, 32, 48, None, 112, 64, 5, -1)
    sens = L.mu3e_align_workspace_size(8)
    assert L.mu3e_select_frames(ctypes.byref(hn), ctypes.byref(p), 1, 1, 1, 1, 1 << 30, 10, 10, None, None) == -1
    assert L.mu3e_fit_triplets(ctypes.byref(hn), 1, 5, ctypes.byref(p), 1, None) == -1
    assert L.mu3e_fit_triplets_backward(ctypes.byref(hn), 1, 5, ctypes.byref(p), 1, 1, None) == -1
    assert L.mu3e_vertex(ctypes.byref(hn), ctypes.byref(lib.Tracks(80, 96, 4, 10)), ctypes.byref(p), 1, 1, 1, 1,
                         1 << 20, None) == -1
    assert L.mu3e_align_chi2(ctypes.byref(hn), 1, 5, 1, 8, ctypes.byref(p), 1, None) == -1
    assert L.mu3e_vertex_refine(ctypes.byref(hn), ctypes.byref(lib.Tracks(80, 96, 4, 10)), 1, 5, None,
                                ctypes.byref(p), 1, 1, 1, 1 << 20, None) == -1
    assert L.mu3e_align_backward(ctypes.byref(hn), 1, 5, 1, 8, ctypes.byref(p), 1, 1, 1, sens, None) == -1
    assert L.mu3e_plan_create(ctypes.byref(plan), ctypes.byref(hn), ctypes.byref(p), 1, 1, 1, 1, 1 << 30, 10, 10,
                              None) == -1


def test_binding_fails_loudly_without_library():
    """The binding has no CPU fallback: with the shared library missing,
    loading it raises instead of computing anything elsewhere."""
    import subprocess
    import sys
    code = ("from paper_2206_11535_amd import lib\n"
            "try:\n"
            "    lib.load('/nonexistent/libmu3e.so')\n"
            "except ImportError as e:\n"
            "    print('raised', e)\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert out.returncode == 0 and out.stdout.startswith("raised"), out.stdout + out.stderr


def test_selector_rejects_other_frame_count(L):
    """The binding refuses hits with more (or fewer) frames than a
    selector's outputs are sized for, before any call into the library
    (host tensors: nothing reaches a GPU)."""
    import torch  # noqa: F401
    from paper_2206_11535_amd import lib, synth
    from paper_2206_11535_amd.params import default_params
    fs = synth.generate(2, n_frames=20)
    hits = lib.to_device(fs, device="cpu")
    for n in (10, 30):
        sel = lib.Selector(n, default_params(), device="cpu")
        with pytest.raises(ValueError, match="frames"):
            sel.run(hits)


def test_fit_autograd_rejects_wrong_coordinates(L):
    """The hit-coordinate autograd wrapper refuses coordinate tensors that
    are not float32 GPU tensors of length n_hits, before any library call
    (host tensors here: nothing reaches a GPU)."""
    import torch
    from paper_2206_11535_amd import lib, synth
    from paper_2206_11535_amd.params import default_params
    fs = synth.generate(2, n_frames=5)
    hits = lib.to_device(fs, device="cpu")
    trip = torch.zeros((1, 3), dtype=torch.int32)
    x = torch.zeros(fs.n_hits - 1)
    with pytest.raises(ValueError, match="x"):
        lib.fit_chi2_autograd(x, hits.y, hits.z, hits, trip, default_params())
    with pytest.raises(ValueError, match="x"):
        lib.fit_chi2_autograd(hits.x, hits.y, hits.z, hits, trip, default_params())   # host tensors


def test_chunk_layout_and_validation(L):
    """The chunk a readout writes (records from the front, the layer offsets
    and the frame count at the tail) as the binding packs it, and the host
    checks of mu3e_chunk_unpack (nothing is launched)."""
    import numpy as np
    from paper_2206_11535_amd import lib, synth
    fs = synth.generate(2, n_frames=40)
    buf = np.full(1 << 16, 0xAB, np.uint8)
    n = lib.pack_chunk(fs, 5, 25, buf)
    lo = fs.layer_offsets
    assert n == lo[100] - lo[20]
    rec = buf[:12 * n].view(np.float32).reshape(-1, 3)
    assert np.array_equal(rec[:, 0], fs.x[lo[20]:lo[100]]) and np.array_equal(rec[:, 2], fs.z[lo[20]:lo[100]])
    tail = buf[len(buf) - 4 * 82:].view(np.int32)
    assert tail[-1] == 20 and tail[0] == 0 and tail[-2] == n
    assert np.array_equal(tail[:-1], lo[20:101] - lo[20])
    assert lib.chunk_capacity(1 << 16, 20) == ((1 << 16) - 4 - 4 * 81) // 12
    with pytest.raises(ValueError):
        lib.pack_chunk(fs, 0, 40, np.zeros(4096, np.uint8))
    P = ctypes.c_void_p
    # null chunk, too short, misaligned, negative sizes, null outputs
    assert L.mu3e_chunk_unpack(None, 1024, 10, 100, 16, 32, 48, 64, 80, None) == -1
    assert L.mu3e_chunk_unpack(P(4096), 2, 10, 100, 16, 32, 48, 64, 80, None) == -1
    assert L.mu3e_chunk_unpack(P(4098), 1024, 10, 100, 16, 32, 48, 64, 80, None) == -1
    assert L.mu3e_chunk_unpack(P(4096), 1024, -1, 100, 16, 32, 48, 64, 80, None) == -1
    assert L.mu3e_chunk_unpack(P(4096), 1024, 10, 100, None, 32, 48, 64, 80, None) == -1
    assert L.mu3e_chunk_unpack(P(4096), 1024, 10, 100, 16, 32, 48, None, 80, None) == -1
