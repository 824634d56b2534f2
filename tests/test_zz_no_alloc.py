"""The selection entry point that allocates nothing (library-owned static
workspace) against the workspace entry point, through the C ABI: two calls
in a row, the second on fewer frames, each compared with
mu3e_select_frames on the same hits (flags, counts and vertices identical)."""
import numpy as np
import pytest

from paper_2206_11535_amd import synth
from paper_2206_11535_amd.params import default_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_11535_amd import lib as L
    L.load()
    return L


def _compare(L, fs, p, tcap, kcap):
    import torch
    print(f"case: static workspace, {fs.n_frames} frames, capacities {tcap}/{kcap}", flush=True)
    dh = L.to_device(fs)
    ref = L.select_frames(dh, p, triplet_capacity=tcap, track_capacity=kcap)
    fl, co, vx = L.select_frames_static(dh, p, tcap, kcap)
    torch.cuda.synchronize()
    assert ref.counters()[2] == 0
    rf, rc, rv = ref.result()
    F = fs.n_frames
    sf = fl[:F].cpu().numpy().view(np.uint32)
    sc = co[:F].cpu().numpy()
    sv = vx[:F].cpu().numpy()
    assert np.array_equal(rf, sf)
    assert np.array_equal(rc, sc)
    assert np.array_equal(np.isnan(rv), np.isnan(sv))
    assert np.array_equal(np.nan_to_num(rv), np.nan_to_num(sv))
    assert rc[:, 0].sum() > 0 and rc[:, 1].sum() > 0
    return rf, rc


def test_static_workspace_two_calls(lib):
    p = default_params()
    big = synth.generate(2, n_frames=20000, salt=11)
    small = synth.generate(1, n_frames=1000, salt=12)
    _compare(lib, big, p, 1 << 19, 16384)
    # second call: fewer frames; stale counters and lists of the first call
    # must not leak into it
    _compare(lib, small, p, 1 << 16, 4096)


def test_static_workspace_refuses_oversize(lib):
    p = default_params()
    fs = synth.generate(1, n_frames=10)
    dh = lib.to_device(fs)
    with pytest.raises(lib.Mu3eError) as e:
        lib.select_frames_static(dh, p, 1 << 30, 1 << 20)
    assert e.value.status == -3
