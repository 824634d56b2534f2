"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Every case runs the same seeded inputs through libmu3e.so on the GPU and
through the oracle on the CPU and compares with tests/parity.py: exact sets
apart from oracle-marked ambiguous candidates (and descendants); float
results within 1e-4 relative.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle
from paper_2206_11535_amd import synth
from paper_2206_11535_amd.params import default_params, lifted_caps
from parity import assert_parity, compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_11535_amd import lib as L
    L.load()
    return L


def run_both(L, fs, params, frames_subset=None, **kw):
    print(f"case: {fs.n_frames} frames, {fs.n_hits} hits, caps "
          f"{params['max_triplets']}/{params['max_tracks']}/{params['max_combos']}", flush=True)
    import torch
    dh = L.to_device(fs)
    sel = L.select_frames(dh, params, **kw)
    torch.cuda.synchronize()
    flags, counts, vtx = sel.result()
    trips, tracks, kf, c = sel.lists(fs.layer_offsets)
    assert c[2] == 0, f"list capacity status {c}"
    orc = oracle.run(fs, params)
    return orc, flags, counts, vtx, trips, tracks, kf, sel


def check(L, fs, params, what, **kw):
    orc, flags, counts, vtx, trips, tracks, kf, _ = run_both(L, fs, params, **kw)
    bad, stats = compare(orc, flags, counts, vtx, trips, tracks, kf)
    print(what, stats, flush=True)
    assert_parity(bad, stats, what)
    return orc, flags, counts


def test_cfg1_full(lib):
    orc, flags, counts = check(lib, synth.generate(1), default_params(), "cfg1")
    assert counts[:, 0].sum() > 1000 and counts[:, 1].sum() > 500 and (flags & 16).sum() > 5


def test_cfg2_subset(lib):
    check(lib, synth.generate(2, n_frames=3000), default_params(), "cfg2[:3000]")


def test_cfg3_mixed_subset(lib):
    check(lib, synth.generate(3, n_frames=3000), default_params(), "cfg3[:3000]")


def test_cfg4_lifted_caps(lib):
    fs = synth.generate(4, n_frames=120)
    p = lifted_caps()
    orc, flags, counts = check(lib, fs, p, "cfg4[:120] lifted", triplet_capacity=1000 * 120,
                               track_capacity=80 * 120)
    assert counts[:, 0].sum() > 20000


def test_triplet_stream_path(lib):
    """Wide windows and a lifted triplet cap: thousands of survivors per
    frame stream through the LDS buffer to the global list."""
    from paper_2206_11535_amd.params import INT32_MAX
    fs = synth.generate(4, n_frames=40)
    p = default_params(dlambda=(-3.0, 3.0), cosphi01=(0.5, 2.0), max_triplets=INT32_MAX)
    orc, flags, counts = check(lib, fs, p, "cfg4[:40] wide windows", triplet_capacity=60000 * 40,
                               track_capacity=4000 * 40)
    assert counts[:, 0].max() > 2000


def test_cfg4_paper_caps(lib):
    check(lib, synth.generate(4, n_frames=200), default_params(), "cfg4[:200] paper caps",
          triplet_capacity=1000 * 200)


@pytest.mark.parametrize("cap", ["max_triplets", "max_tracks", "max_combos"])
@pytest.mark.parametrize("value", [0, 1])
def test_caps_zero_one(lib, cap, value):
    check(lib, synth.generate(1, n_frames=400), default_params(**{cap: value}), f"{cap}={value}")


def test_layer_hit_overflow(lib):
    fs = synth.generate(2, n_frames=500)
    orc, flags, counts = check(lib, fs, default_params(max_layer_hits=10), "max_layer_hits=10")
    assert (flags & 32).sum() > 10


# hits per layer (0..3) of frames around the LDS tile sizes (64 and 128
# hits per layer): one full tile (128: 16,384 pairs per layer pair), one
# less, one more on each kind of layer (two tiles), and frames that need
# several tiles per layer up to the layer capacity (1023 hits)
LIMIT_FILL = [(128, 128, 128, 128), (128, 128, 128, 40), (129, 20, 20, 20), (20, 20, 20, 129),
              (30, 128, 30, 30), (128, 30, 128, 30), (127, 128, 127, 128), (128, 129, 128, 128)]
TILE_FILL = [(64, 64, 64, 64), (65, 63, 65, 20), (20, 65, 20, 20), (20, 20, 129, 20), (200, 150, 140, 90),
             (300, 64, 130, 40), (1023, 12, 12, 12), (12, 12, 1023, 1023), (30, 30, 30, 1024), (1024, 5, 5, 5)]


def limit_frames(fill=LIMIT_FILL, seed=5):
    """High-rate Michel frames with each layer cut or padded with noise hits
    (pixel centres on the layer's cylinder) to the counts of `fill`, the hits
    of a layer in random order."""
    from helpers import Frames
    base = synth.generate(dataclasses.replace(synth.CONFIGS[1], lam=22.0, noise_per_layer=0),
                          n_frames=len(fill), salt=21)
    rng = np.random.default_rng(seed)
    frames = []
    for f, want in enumerate(fill):
        fr = []
        for l in range(4):
            a, b = base.layer_offsets[4 * f + l], base.layer_offsets[4 * f + l + 1]
            pts = np.stack([base.x[a:b], base.y[a:b], base.z[a:b]], 1)[:want[l]].astype(float)
            k = want[l] - len(pts)
            phi = rng.uniform(-np.pi, np.pi, k)
            zt = rng.uniform(-1.0, 1.0, k) * synth.Z_HALF[l]
            x, y, z = synth.quantise(phi, zt, synth.R_LAYER[l])
            z = np.where(np.abs(z) > synth.Z_HALF[l], z - np.sign(z) * synth.PIXEL, z)
            pts = np.concatenate([pts, np.stack([x, y, z], 1)])
            fr.append(pts[rng.permutation(len(pts))])
        frames.append(fr)
    fs = Frames(frames)
    assert np.array_equal(np.diff(fs.layer_offsets).reshape(-1, 4), np.asarray(fill))
    return fs


def batched_equal_plain(lib, dh, p, tiles=(64, 128)):
    """Every batched shape that matters for tiling (both LDS tile sizes,
    fused or not, stolen tail) gives the plain form's outputs."""
    import torch
    a = lib.select_frames(dh, p)
    for tile in tiles:
        for fuse in (0, 1):
            print(f"case: batched tile {tile} fuse {fuse}", flush=True)
            b = lib.BatchedSelector(dh, p, waves_per_cu=4, frames_per_claim=1, fuse_fits=fuse, steal_percent=50,
                                    tile_hits=tile)
            b.run()
            torch.cuda.synchronize()
            fa, ca, va = a.result()
            fb, cb, vb = b.result()
            assert np.array_equal(fa, fb) and np.array_equal(ca, cb)
            assert np.array_equal(np.nan_to_num(va), np.nan_to_num(vb))
            assert b.counters()[2] == 0
            assert b.effective[4] == tile


@pytest.mark.parametrize("n_sub", [2, 3, 4])
def test_sub_batches_equal_plain_and_oracle(lib, n_sub):
    """A plan split into sub-batches (cuts of one overlapping the fits and
    vertex stage of the one before, on the plan's streams) gives exactly the
    plain form's outputs and lists, matches the oracle, and repeats."""
    import torch
    fs = synth.generate(2, n_frames=3001, salt=31)
    p = default_params()
    dh = lib.to_device(fs)
    a = lib.select_frames(dh, p)
    torch.cuda.synchronize()
    ta, ka, kfa, _ = a.lists(fs.layer_offsets)
    orc = oracle.run(fs, p)
    for fuse, tile in ((0, 128), (1, 64)):
        print(f"case: {n_sub} sub-batches, fuse {fuse}, tile {tile}", flush=True)
        b = lib.BatchedSelector(dh, p, waves_per_cu=8, frames_per_claim=4, fuse_fits=fuse, steal_percent=25,
                                tile_hits=tile, sub_batches=n_sub)
        assert b.effective[5] == n_sub and len(b.parts) == n_sub
        assert sum(n for _, _, n in b.parts) == fs.n_frames
        for _ in range(2):
            b.run()
        torch.cuda.synchronize()
        fa, ca, va = a.result()
        fb, cb, vb = b.result()
        assert np.array_equal(fa, fb) and np.array_equal(ca, cb)
        assert np.array_equal(np.nan_to_num(va), np.nan_to_num(vb))
        tb, kb, kfb, c = b.lists(fs.layer_offsets)
        assert c[2] == 0
        assert sorted(map(tuple, ta.tolist())) == sorted(map(tuple, tb.tolist()))
        assert sorted(map(tuple, ka.tolist())) == sorted(map(tuple, kb.tolist()))
        bad, stats = compare(orc, fb, cb, vb, tb, kb, kfb)
        assert_parity(bad, stats, f"{n_sub} sub-batches")


def test_layers_at_the_tile_limit(lib):
    """Layers that fill one 128-hit tile, one below and one above it (two
    tiles), with the paper's caps and with lifted caps (then the full-size
    frames reach the vertex stage), in the plain form and in the batched
    form with both tile sizes."""
    fs = limit_frames()
    for what, p in (("limit frames", default_params()), ("limit frames lifted", lifted_caps())):
        orc, flags, counts = check(lib, fs, p, what)
        assert not (flags & 32).any()
        batched_equal_plain(lib, lib.to_device(fs), p)
    assert counts[:, 0].max() > 2000 and counts[:, 2].max() > 500 and (flags & 16).any()


def test_layers_over_several_tiles(lib):
    """Frames whose layers need several LDS tiles (up to the 1023-hit layer
    capacity) against the oracle, with every triplet kept (no triplet cap)
    and the paper's track and combination caps; layers of 1024 hits are over
    the capacity: flagged and kept unprocessed."""
    fs = limit_frames(TILE_FILL, seed=6)
    p = default_params(max_triplets=2 ** 31 - 1)
    orc, flags, counts = check(lib, fs, p, "tiled frames")
    over = np.asarray([max(w) > 1023 for w in TILE_FILL])
    assert np.array_equal((flags & 32) != 0, over)
    assert counts[~over, 0].min() > 0 and counts[:, 0].max() > 5000
    batched_equal_plain(lib, lib.to_device(fs), p)
    # a lower capacity given as a parameter flags the frames above it
    q = default_params(max_triplets=2 ** 31 - 1, max_layer_hits=200)
    orc, flags, counts = check(lib, fs, q, "tiled frames, capacity 200")
    assert np.array_equal((flags & 32) != 0, np.asarray([max(w) > 200 for w in TILE_FILL]))


def test_empty_and_tiny_frames(lib):
    from helpers import Frames
    frames = [[[], [], [], []],
              [[(25.0, 0.0, 1.0)], [], [(73.0, 0.0, 2.0)], []],
              [[(25.0, 0.0, 1.0)], [(31.0, 0.5, 1.2)], [(73.0, 2.0, 2.0)], []],
              [[], [], [], [(85.0, 0.0, 0.0)]]]
    fs = Frames(frames)
    check(lib, fs, default_params(), "tiny frames")


def test_batches_in_flight(lib):
    """Distinct batches in flight on their own streams, as bench.py times
    them: after three interleaved rounds every plan's outputs equal the plain
    form on its own batch."""
    import torch
    p = default_params()
    hs = [lib.to_device(synth.generate(2, n_frames=3000, salt=s)) for s in range(3)]
    refs = [lib.select_frames(h, p) for h in hs]
    torch.cuda.synchronize()
    shapes = [(8, 4, 0, 0, 128, 1), (12, 4, 1, 25, 64, 2), (16, 8, 0, 50, 128, 3)]
    plans = [lib.BatchedSelector(h, p, waves_per_cu=w, frames_per_claim=c, fuse_fits=u, steal_percent=st,
                                 tile_hits=t, sub_batches=n)
             for h, (w, c, u, st, t, n) in zip(hs, shapes)]
    streams = [torch.cuda.Stream() for _ in plans]
    print("case: three plans on three streams, three rounds", flush=True)
    for _ in range(3):
        for b, st in zip(plans, streams):
            b.run(None, st)
    torch.cuda.synchronize()
    for k, (r, b) in enumerate(zip(refs, plans)):
        fr, cr, vr = r.result()
        fb, cb, vb = b.result()
        assert np.array_equal(fr, fb) and np.array_equal(cr, cb), k
        assert np.array_equal(np.nan_to_num(vr), np.nan_to_num(vb)), k
        assert b.counters()[2] == 0


def test_batched_empty_and_tiny(lib):
    """The batched form on a batch without frames, on one frame, and on the
    tiny frames above (every shape), against the plain form."""
    import torch
    from helpers import Frames
    frames = [[[], [], [], []],
              [[(25.0, 0.0, 1.0)], [], [(73.0, 0.0, 2.0)], []],
              [[(25.0, 0.0, 1.0)], [(31.0, 0.5, 1.2)], [(73.0, 2.0, 2.0)], []],
              [[], [], [], [(85.0, 0.0, 0.0)]]]
    p = default_params()
    for sub in ([], frames[2:3], frames):
        fs = Frames(sub) if sub else None
        if fs is None:
            empty = Frames(frames[:1])
            empty.layer_offsets = np.zeros(1, np.int32)
            empty.x = empty.y = empty.z = np.zeros(0, np.float32)
            empty.sensor = empty.layer = np.zeros(0, np.uint16)
            fs = empty
        print(f"case: batched tiny, {fs.n_frames} frames", flush=True)
        dh = lib.to_device(fs)
        a = lib.select_frames(dh, p)
        for fuse in (0, 1):
            b = lib.BatchedSelector(dh, p, waves_per_cu=4, frames_per_claim=1, fuse_fits=fuse, steal_percent=50)
            b.run()
            torch.cuda.synchronize()
            fa, ca, va = a.result()
            fb, cb, vb = b.result()
            assert np.array_equal(fa, fb) and np.array_equal(ca, cb)
            assert np.array_equal(np.nan_to_num(va), np.nan_to_num(vb))
            assert b.counters()[2] == 0


def test_malformed_layer_offsets(lib):
    """Frames whose layer offsets are negative, decreasing or beyond n_hits
    are skipped (no flag, no count) and reported in status bit 4, in both
    forms; every other frame gives what it gives with correct offsets."""
    import torch
    fs = synth.generate(2, n_frames=300)
    p = default_params()
    lo = fs.layer_offsets.copy()
    F = fs.n_frames
    lo[4 * 10 + 1] = lo[4 * 10] - 1              # layer 0 count negative
    lo[4 * 20 + 2] = lo[4 * 20 + 1] - 3          # layer 1 count negative
    lo[4 * 30 + 3] = lo[4 * 30 + 4] + 2          # layer 3 count negative
    lo[4 * 40] = -1                              # frame 40 starts below 0, frame 39 ends below its start
    lo[4 * F] = fs.n_hits + 5                    # the last frame ends beyond n_hits
    skip = np.zeros(F, bool)
    skip[[10, 20, 30, 39, 40, F - 1]] = True
    bad = dataclasses.replace(fs, layer_offsets=lo)
    print(f"case: malformed offsets, frames {np.flatnonzero(skip).tolist()}", flush=True)
    ref = lib.select_frames(lib.to_device(fs), p)
    dh = lib.to_device(bad)
    a = lib.select_frames(dh, p)
    torch.cuda.synchronize()
    fr, cr, vr = ref.result()
    fa, ca, va = a.result()
    assert np.all(fa[skip] == 0) and np.all(ca[skip] == 0)
    assert np.array_equal(fa[~skip], fr[~skip]) and np.array_equal(ca[~skip], cr[~skip])
    assert np.array_equal(np.nan_to_num(va[~skip]), np.nan_to_num(vr[~skip]))
    assert a.counters()[2] & 4 and not ref.counters()[2] & 4
    for fuse in (0, 1):
        b = lib.BatchedSelector(dh, p, waves_per_cu=4, frames_per_claim=2, fuse_fits=fuse, steal_percent=50)
        b.run()
        torch.cuda.synchronize()
        fb, cb, vb = b.result()
        assert np.array_equal(fa, fb) and np.array_equal(ca, cb)
        assert b.counters()[2] & 4


def test_misaligned_frames(lib):
    check(lib, synth.generate(5, n_frames=2000), default_params(), "cfg5[:2000]")


def test_signal_only_frames(lib):
    cfg = dataclasses.replace(synth.CONFIGS[1], lam=0.5, noise_per_layer=0, signal_frac=1.0)
    orc, flags, counts = check(lib, synth.generate(cfg, n_frames=1500, salt=9), default_params(), "signal")
    assert (flags & 16).sum() > 300


def test_busy_signal_frames(lib):
    """Signal decays on top of a high Michel rate: vertex-candidate frames
    with more tracks than the per-frame slot row (the vertex stage then
    gathers them from the whole triplet list)."""
    cfg = dataclasses.replace(synth.CONFIGS[1], lam=22.0, noise_per_layer=2, signal_frac=1.0)
    fs = synth.generate(cfg, n_frames=500, salt=13)
    orc, flags, counts = check(lib, fs, default_params(), "busy signal frames", triplet_capacity=400 * 500)
    many = (counts[:, 1] > 16) & ((flags & (2 | 4 | 32)) == 0)
    assert many.sum() > 50
    assert ((flags & 16) != 0)[many].sum() > 10


@pytest.mark.parametrize("fuse", [0, 1])
def test_batched_small_chunks(lib, fuse):
    """A small triplet capacity makes the chunks 64 entries long, so frames
    span chunks, fused fits leave entries of closed chunks to k_tracks, and
    an overflowing frame leaves entries behind in closed chunks."""
    import torch
    fs = synth.generate(2, n_frames=3000)
    p = default_params(max_triplets=30)
    dh = lib.to_device(fs)
    print(f"case: batched small chunks fused={fuse}", flush=True)
    a = lib.select_frames(dh, p, triplet_capacity=400000)
    b = lib.BatchedSelector(dh, p, triplet_capacity=120000, waves_per_cu=4, frames_per_claim=2, fuse_fits=fuse,
                            steal_percent=50)
    b.run()
    torch.cuda.synchronize()
    assert b.dbg.chunk_size == 64
    assert a.counters()[2] == 0
    fa, ca, va = a.result()
    fb, cb, vb = b.result()
    assert np.array_equal(fa, fb) and np.array_equal(ca, cb)
    assert np.array_equal(np.nan_to_num(va), np.nan_to_num(vb))
    assert (fb & 2).sum() > 20   # frames over max_triplets
    tb, kb, kfb, c = b.lists(fs.layer_offsets)
    assert c[2] == 0
    # counters[0], summed from the waves' tallies: the triplets of frames
    # that did not overflow, in both forms
    kept = (fb & 2) == 0
    for sel in (a, b):
        assert int(sel.counters()[0]) == int(cb[:, 0][kept].sum()) == len(tb)
    orc = oracle.run(fs, p)
    bad, stats = compare(orc, fb, cb, vb, tb, kb, kfb)
    assert_parity(bad, stats, f"batched small chunks fused={fuse}")


def test_edges_on_candidates(lib):
    """Cut windows whose edges sit on the float32-rounded value of a true
    triplet's Delta lambda, cos Phi01, cos Phi12 or |r_tc|: float32 cannot
    decide those candidates, so every float64 decision of the cuts runs
    (the Phi12 and Delta lambda ones deferred to the r_tc stage).  A
    float32-rounded edge lies ~1e-8 (relative) from the float64 value, so
    the oracle, run with an ambiguity band of 1e-12 instead of 1e-5, decides
    them, and both forms must agree with it."""
    import torch
    fs = synth.generate(2, n_frames=400, salt=21)
    p = default_params()
    tt, _, _ = synth.true_triplets(fs)
    h = np.stack([np.stack([fs.x[tt[:, k]], fs.y[tt[:, k]], fs.z[tt[:, k]]], 1) for k in range(3)], 1)
    q, dec = oracle.cut_quantities(h.astype(np.float64), p)
    q = q[dec == 1]
    assert len(q) > 100

    def at(v, frac):   # the float32 value of the element at this rank
        return float(np.float32(np.sort(v)[int(frac * (len(v) - 1))]))

    dl, c01, c12, rt = q[:, 0], q[:, 1], q[:, 2], np.abs(q[:, 3])
    pe = dict(p, amb=1e-12, dlambda=(at(dl[dl < 0], 0.3), at(dl[dl > 0], 0.7)),
              cosphi01=(at(c01, 0.3), 2.0), cosphi12=(at(c12, 0.3), 2.0), rtc_abs=(at(rt, 0.2), at(rt, 0.8)))
    orc, flags, counts = check(lib, fs, pe, "edges on candidates, plain")
    assert int((orc.namb).sum()) == 0
    dh = lib.to_device(fs)
    b = lib.BatchedSelector(dh, pe, waves_per_cu=4, frames_per_claim=2, steal_percent=25)
    b.run()
    torch.cuda.synchronize()
    fb, cb, vb = b.result()
    assert np.array_equal(fb, flags) and np.array_equal(cb, counts)


@pytest.mark.parametrize("cap", [40, 3000])
def test_triplet_list_full(lib, cap):
    """A triplet list too small for the batch (below one chunk, and a few
    chunks): both forms report it in the status word (bit 1) instead of
    writing past it, and the per-frame triplet counts stay exact."""
    import torch
    fs = synth.generate(2, n_frames=2000)
    p = default_params()
    dh = lib.to_device(fs)
    ref = lib.select_frames(dh, p)
    print(f"case: triplet list of {cap} entries", flush=True)
    a = lib.select_frames(dh, p, triplet_capacity=cap)
    b = lib.BatchedSelector(dh, p, triplet_capacity=cap, waves_per_cu=4, frames_per_claim=2, steal_percent=25)
    b.run()
    torch.cuda.synchronize()
    fr, cr, vr = ref.result()
    assert ref.counters()[2] == 0
    for sel in (a, b):
        c = sel.counters()
        assert c[2] & 1, c
        fs_, cs, vs = sel.result()
        assert np.array_equal(cs[:, 0], cr[:, 0])
        # every frame whose triplets the list could not hold is flagged and
        # kept; every other frame is processed fully, as with a large list
        full = (fs_ & lib.LIST_FULL) != 0
        assert full.any() and np.all(fs_[full] & lib.KEEP) and np.all(cs[full, 0] > 0)
        assert np.array_equal(fs_[~full], fr[~full]) and np.array_equal(cs[~full], cr[~full])
        assert np.array_equal(np.nan_to_num(vs[~full]), np.nan_to_num(vr[~full]))
    # the plan runs again, still reporting the full list
    b.run()
    torch.cuda.synchronize()
    assert b.counters()[2] & 1


def test_fit_triplets(lib):
    import torch
    fs = synth.generate(2, n_frames=3000)
    tt, _, tab = synth.true_triplets(fs)
    rng = np.random.default_rng(0)
    # true triplets, second triplets (layers 1-3) and random combinations
    t2 = tab[np.all(tab[:, 1:4] >= 0, axis=1)][:, 1:4]
    lo = fs.layer_offsets
    f = rng.integers(0, fs.n_frames, 4000)
    ok = np.all([lo[4 * f + l + 1] > lo[4 * f + l] for l in range(3)], axis=0)
    f = f[ok]
    rnd = np.stack([rng.integers(lo[4 * f + l], lo[4 * f + l + 1]) for l in range(3)], 1)
    trip = np.concatenate([tt, t2, rnd]).astype(np.int32)
    print(f"case: fit_triplets n={len(trip)}", flush=True)
    dh = lib.to_device(fs)
    out = lib.fit_triplets(dh, torch.from_numpy(trip).cuda(), default_params()).cpu().numpy()
    h = np.stack([np.stack([fs.x[trip[:, k]], fs.y[trip[:, k]], fs.z[trip[:, k]]], 1) for k in range(3)], 1)
    ref, rok = oracle.fit(h.astype(np.float64), default_params())
    assert np.all(np.isfinite(out[rok, 0]))
    names = ["kappa", "sigma2_kappa", "chi2", "r_star", "sigma2_r", "rtc", "theta1", "theta2"]
    for i, k in enumerate(names):
        g, o = out[rok, i].astype(np.float64), ref[k][rok]
        floor = 1.0 if k == "chi2" else 0.0
        err = np.abs(g - o) / np.maximum(np.abs(o), floor)
        assert np.max(err) <= 1e-4, (k, float(np.max(err)), int(np.argmax(err)))


def test_fit_triplets_degenerate_and_out_of_range(lib):
    """Triplets the fit cannot take give NaN in all eight fields: collinear
    in the transverse plane (along x, along y), a repeated hit, and hit
    indices outside [0, n_hits) (a kernel-side bounds check, no read);
    an ordinary triplet among them matches the oracle; no triplets is a
    valid call."""
    import torch
    from helpers import Frames
    fs = Frames([[[(25.0, 0.0, 1.0), (0.0, 25.0, 1.0)],
                  [(31.0, 0.0, 2.0), (0.0, 31.0, 2.0), (31.0, 0.5, 2.0)],
                  [(73.0, 0.0, 5.0), (0.0, 73.0, 5.0), (73.0, 2.0, 5.0)], []]])
    big, small = np.iinfo(np.int32).max, np.iinfo(np.int32).min
    trip = np.array([[0, 2, 5], [1, 3, 6], [0, 0, 5], [0, 4, 7], [-1, 2, 5], [0, 2, fs.n_hits],
                     [0, big, 7], [small, 4, 7]], np.int32)
    print(f"case: fit_triplets degenerate, n={len(trip)}", flush=True)
    dh = lib.to_device(fs)
    p = default_params()
    out = lib.fit_triplets(dh, torch.from_numpy(trip).cuda(), p).cpu().numpy()
    good = np.zeros(len(trip), bool)
    good[3] = True
    assert np.all(np.isnan(out[~good]))
    h = np.stack([np.stack([fs.x[trip[good, k]], fs.y[trip[good, k]], fs.z[trip[good, k]]], 1)
                  for k in range(3)], 1)
    ref, rok = oracle.fit(h.astype(np.float64), p)
    assert rok.all()
    names = ["kappa", "sigma2_kappa", "chi2", "r_star", "sigma2_r", "rtc", "theta1", "theta2"]
    for i, k in enumerate(names):
        floor = 1.0 if k == "chi2" else 0.0
        assert abs(float(out[good][0, i]) - ref[k][0]) <= 1e-4 * max(abs(ref[k][0]), floor), k
    # the oracle rejects the in-range degenerate ones as well
    hd = np.stack([np.stack([fs.x[trip[:3, k]], fs.y[trip[:3, k]], fs.z[trip[:3, k]]], 1) for k in range(3)], 1)
    assert not oracle.fit(hd.astype(np.float64), p)[1].any()
    assert lib.fit_triplets(dh, torch.zeros((0, 3), dtype=torch.int32, device="cuda"), p).shape == (0, 8)


def test_fit_triplets_backward(lib):
    """Adjoint of the fit chi2 with respect to the hit coordinates against
    FP64 central differences of the oracle's fit chi2 (step 1e-4 mm), on
    true triplets sharing hits, with random upstream gradients; an invalid
    triplet adds nothing, a given buffer is added to, n = 0 is valid."""
    import torch
    fs = synth.generate(2, n_frames=1200)
    assert fs.n_hits < 65536   # one alignment "sensor" per hit below
    tt, _, tab = synth.true_triplets(fs)
    t2 = tab[np.all(tab[:, 1:4] >= 0, axis=1)][:, 1:4]
    trip = np.concatenate([tt, t2]).astype(np.int32)
    p = default_params()
    h = np.stack([np.stack([fs.x[trip[:, k]], fs.y[trip[:, k]], fs.z[trip[:, k]]], 1) for k in range(3)], 1)
    h = h.astype(np.float64)
    ref, rok = oracle.fit(h, p)
    trip, h = trip[rok], h[rok]
    rng = np.random.default_rng(11)
    w = rng.uniform(0.0, 2.0, len(trip))
    eps = 1e-4
    hp = np.repeat(h[:, None], 9, 1).copy()
    hm = hp.copy()
    for j in range(9):
        hp[:, j, j // 3, j % 3] += eps
        hm[:, j, j // 3, j % 3] -= eps
    cp, okp = oracle.fit(hp.reshape(-1, 3, 3), p)
    cm, okm = oracle.fit(hm.reshape(-1, 3, 3), p)
    assert okp.all() and okm.all()
    d = ((cp["chi2"] - cm["chi2"]) / (2 * eps)).reshape(-1, 9) * w[:, None]
    gref = np.zeros((fs.n_hits, 3))
    for k in range(3):
        np.add.at(gref, trip[:, k], d[:, 3 * k:3 * k + 3])
    bad = np.array([[-1, trip[0, 1], trip[0, 2]]], np.int32)
    print(f"case: fit_triplets_backward n={len(trip)}", flush=True)
    dh = lib.to_device(fs)
    tg = torch.from_numpy(np.concatenate([trip, bad])).cuda()
    wg = torch.from_numpy(np.concatenate([w, [1.0]]).astype(np.float32)).cuda()
    g = lib.fit_triplets_backward(dh, tg, p, wg)
    torch.cuda.synchronize()
    gn = g.cpu().numpy().astype(np.float64)
    err = np.linalg.norm(gn - gref) / np.linalg.norm(gref)
    print("fit adjoint vs central differences: norm-wise", err, flush=True)
    assert err <= 1e-3
    # exact reference: the oracle's forward-mode (dual number) gradient of the
    # same weighted sum, with every hit on a sensor of its own, so that the
    # gradient with respect to a sensor's translation at zero alignment is
    # the gradient with respect to that hit's coordinates
    fs1 = dataclasses.replace(fs, sensor=np.arange(fs.n_hits, dtype=np.uint16))
    _, gs = oracle.align_loss_grad(fs1, trip, np.zeros((fs.n_hits, 4)), p, weight=w)
    gex = gs[:, :3]
    err = np.linalg.norm(gn - gex) / np.linalg.norm(gex)
    floor = 1e-3 * np.abs(gex).max()
    elem = np.max(np.abs(gn - gex) / np.maximum(np.abs(gex), floor))
    print("fit adjoint vs exact dual gradient: norm-wise", err, "element-wise (floored)", elem, flush=True)
    assert err <= 1e-3 and elem <= 1e-3
    # the two references agree with each other
    assert np.linalg.norm(gref - gex) / np.linalg.norm(gex) <= 1e-4
    used = np.zeros(fs.n_hits, bool)
    used[trip.ravel()] = True
    assert np.count_nonzero(gn[~used]) == 0
    g2 = lib.fit_triplets_backward(dh, tg, p, wg, grad_xyz=g.clone())
    assert torch.allclose(g2, 2 * g, rtol=1e-5, atol=1e-6 * float(g.abs().max()))
    z = lib.fit_triplets_backward(dh, torch.zeros((0, 3), dtype=torch.int32, device="cuda"), p,
                                  torch.zeros(0, dtype=torch.float32, device="cuda"))
    assert z.shape == (fs.n_hits, 3) and torch.count_nonzero(z).item() == 0


def test_fit_chi2_autograd(lib):
    """The autograd wrapper over the hit coordinates: chi2 as from
    mu3e_fit_triplets, gradients as from mu3e_fit_triplets_backward, and a
    small step along the gradient lowers the summed chi2."""
    import torch
    fs = synth.generate(2, n_frames=300)
    tt, _, _ = synth.true_triplets(fs)
    trip = torch.from_numpy(np.ascontiguousarray(tt, dtype=np.int32)).cuda()
    p = default_params()
    dh = lib.to_device(fs)
    x, y, z = (t.clone().requires_grad_(True) for t in (dh.x, dh.y, dh.z))
    c = lib.fit_chi2_autograd(x, y, z, dh, trip, p)
    ref = lib.fit_triplets(dh, trip, p)[:, 2]
    ok = torch.isfinite(ref)
    assert ok.sum() > 500 and torch.equal(c[ok], ref[ok])
    w = torch.where(ok, torch.rand(len(ok), device="cuda"), torch.zeros_like(ref))
    (torch.nan_to_num(c) * w).sum().backward()
    g = lib.fit_triplets_backward(dh, trip, p, w)
    gxyz = torch.stack([x.grad, y.grad, z.grad], 1)
    assert torch.allclose(gxyz, g, rtol=1e-5, atol=1e-6 * float(g.abs().max()))
    with torch.no_grad():
        step = 1e-4 / float(gxyz.abs().max())
        h2 = lib.DeviceHits(x - step * x.grad, y - step * y.grad, z - step * z.grad, dh.layer, dh.sensor,
                            dh.layer_offsets, dh.n_frames, dh.n_hits)
        after = lib.fit_triplets(h2, trip, p)[:, 2]
    assert float((after[ok] * w[ok]).sum()) < float((ref[ok] * w[ok]).sum())


def test_vertex_entry_point(lib):
    """mu3e_vertex on the oracle's accepted tracks reproduces the oracle's
    vertex decisions for frames without an overflow."""
    import torch
    cfg = dataclasses.replace(synth.CONFIGS[1], lam=1.0, noise_per_layer=1, signal_frac=0.6)
    fs = synth.generate(cfg, n_frames=1500, salt=11)
    p = default_params()
    orc = oracle.run(fs, p)
    k = orc.tracks[(orc.tracks[:, 6] == 1) & (orc.tracks[:, 7] == 0)]
    F = fs.n_frames
    off = np.searchsorted(k[:, 0], np.arange(F + 1)).astype(np.int32)
    hits = k[:, 1:5].astype(np.int32)
    print(f"case: vertex n_tracks={len(hits)}", flush=True)
    dh = lib.to_device(fs)
    gf, gc, gv = lib.vertex(dh, torch.from_numpy(hits).cuda(), torch.from_numpy(off).cuda(), p)
    gf, gc, gv = gf.cpu().numpy(), gc.cpu().numpy(), gv.cpu().numpy()
    ok = (orc.amb == 0) & ((orc.flags & (2 | 4 | 32)) == 0)
    assert ok.sum() > 1000
    assert np.array_equal(gf[ok] & 24, orc.flags[ok] & 24)
    assert np.array_equal(gc[ok], orc.counts[ok, 2])
    v = ok & ((orc.flags & 16) != 0)
    assert v.sum() > 100
    assert np.allclose(gv[v, :3], orc.vertex[v, :3], rtol=1e-4, atol=1e-3)


def test_energy_passing_triples_equal_oracle(lib):
    """The e+e+e- triples passing the energy test (Alg. 4, preliminary
    check), as a set: the GPU's own accepted tracks of each frame go through
    mu3e_vertex_debug, and its triple list equals the oracle's energy-passing
    triples (keyed by the first triplets of the three tracks, the e+ pair
    unordered) on every frame whose tracks are decided without ambiguity;
    triples the oracle marks ambiguous are dropped from both sides."""
    import torch
    cfg = dataclasses.replace(synth.CONFIGS[2], lam=12.0, signal_frac=0.3)
    fs = synth.generate(cfg, n_frames=600, salt=17)
    p = lifted_caps()
    dh = lib.to_device(fs)
    sel = lib.select_frames(dh, p)
    torch.cuda.synchronize()
    _, tracks, kf, c = sel.lists(fs.layer_offsets)
    assert c[2] == 0
    order = np.lexsort((tracks[:, 3], tracks[:, 2], tracks[:, 1], tracks[:, 0]))
    tracks, kf = tracks[order], kf[order]
    F = fs.n_frames
    off = np.searchsorted(tracks[:, 0], np.arange(F + 1)).astype(np.int32)
    th = np.ascontiguousarray(tracks[:, 1:5], dtype=np.int32)
    print(f"case: energy-passing triples, {len(th)} GPU tracks", flush=True)
    gf, gc, gv, rows, m = lib.vertex(dh, torch.from_numpy(th).cuda(), torch.from_numpy(off).cuda(), p,
                                     triple_capacity=2_000_000)
    rows = rows.cpu().numpy()
    assert m == len(rows) and m > 1000
    assert np.array_equal(gc.cpu().numpy(), sel.result()[1][:, 2])
    orc = oracle.run(fs, p)
    # frames compared: no ambiguous track, no overflow before the vertex stage
    okf = (orc.namb[:, 0] == 0) & (orc.namb[:, 1] == 0) & ((orc.flags & (2 | 4 | 32)) == 0)
    assert okf.sum() > 0.8 * F

    def key(f, a, b, e):
        pa, pb = tuple(a), tuple(b)
        return (int(f), min(pa, pb), max(pa, pb), tuple(e))
    trip_of = tracks[:, 1:4]
    g = {key(r[0], trip_of[r[1]], trip_of[r[2]], trip_of[r[3]]) for r in rows.tolist() if okf[r[0]]}
    t = orc.triples
    sure = {key(r[0], r[1:4], r[4:7], r[7:10]) for r in t.tolist() if r[10] == 1 and r[11] == 0 and okf[r[0]]}
    amb = {key(r[0], r[1:4], r[4:7], r[7:10]) for r in t.tolist() if r[11] == 1}
    g -= amb
    assert len(sure) > 1000
    assert sure == g, (len(sure - g), len(g - sure), sorted(sure - g)[:3], sorted(g - sure)[:3])
    # the e+ / e- roles: charges of the GPU's tracks
    ch = np.sign(kf[:, 0])
    assert np.all(ch[rows[:, 1]] > 0) and np.all(ch[rows[:, 2]] > 0) and np.all(ch[rows[:, 3]] < 0)


def test_chunks_unpacked_equal_batch(lib):
    """Frames packed into chunks (records and tail offsets, as the readout
    writes them), copied to the GPU and unpacked give the same selection as
    the frames given as SoA arrays; the frames that pad a chunk to its frame
    table stay empty.  Through ChunkStream with three slots in flight, in
    both forms, over more chunks than slots."""
    import torch
    fs = synth.generate(2, n_frames=7000, salt=41)
    p = default_params()
    dh = lib.to_device(fs)
    ref = lib.select_frames(dh, p)
    torch.cuda.synchronize()
    rf, rc, rv = ref.result()
    bounds = [0, 1000, 2500, 2501, 4000, 5200, 6500, 7000, 7000]   # uneven chunks, one of one frame, one empty
    for form in ("batched", "plain"):
        print(f"case: chunk stream, {form}", flush=True)
        cs = lib.ChunkStream(p, 1 << 21, 1500, n_buffers=3, form=form)
        slots = []
        for a, b in zip(bounds[:-1], bounds[1:]):
            slots.append((a, b, cs.submit(lambda v, a=a, b=b: lib.pack_chunk(fs, a, b, v))))
            if len(slots) >= 3:   # results of the oldest chunk before its slot is refilled
                a0, b0, k0 = slots.pop(0)
                F, fl = cs.result(k0)
                assert F == b0 - a0 and np.array_equal(fl, rf[a0:b0])
        for a0, b0, k0 in slots:
            F, fl = cs.result(k0)
            assert F == b0 - a0 and np.array_equal(fl, rf[a0:b0])
        # the last chunk's full outputs, padding frames included
        sl = cs.slots[k0]
        fb, cb, vb = sl["sel"].result()
        assert not fb[b0 - a0:].any() and not cb[b0 - a0:].any()
        cs.synchronize()
    # one chunk through the plain form with the debug lists: same triplets
    print("case: one chunk, lists", flush=True)
    cs = lib.ChunkStream(p, 1 << 22, 3000, n_buffers=1, form="plain")
    k = cs.submit(lambda v: lib.pack_chunk(fs, 2000, 5000, v))
    F, fl = cs.result(k)
    sel = cs.slots[k]["sel"]
    lo_chunk = cs.slots[k]["hits"].layer_offsets.cpu().numpy()
    t, tr, kf, c = sel.lists(lo_chunk)
    assert c[2] == 0
    tr_ref, _, _, _ = ref.lists(fs.layer_offsets)
    base = fs.layer_offsets[4 * 2000]
    m = (tr_ref[:, 0] >= 2000) & (tr_ref[:, 0] < 5000)
    want = tr_ref[m].copy()
    want[:, 0] -= 2000
    want[:, 1:] -= base
    assert sorted(map(tuple, t.tolist())) == sorted(map(tuple, want.tolist()))


def test_malformed_chunks(lib):
    """Chunks whose tail is inconsistent (frame count above the table,
    offsets overlapping the records, a first offset other than 0, more hits
    than the buffers hold) are unpacked to no frames with info -1; offsets
    that decrease inside a consistent tail reach the selection, which skips
    those frames and reports them."""
    import torch
    fs = synth.generate(2, n_frames=300, salt=42)
    p = default_params()
    cs = lib.ChunkStream(p, 1 << 20, 400, n_buffers=1, form="plain")

    def bad_count(v):
        lib.pack_chunk(fs, 0, 300, v)
        v[len(v) // 4 * 4 - 4:len(v) // 4 * 4].view(np.int32)[0] = 401

    def overlapping(v):
        v[:] = 0
        v[len(v) // 4 * 4 - 4:len(v) // 4 * 4].view(np.int32)[0] = (len(v) // 4) // 4

    def first_not_zero(v):
        lib.pack_chunk(fs, 0, 300, v)
        t = v[len(v) // 4 * 4 - 4 * (4 * 300 + 2):len(v) // 4 * 4].view(np.int32)
        t[0] = 1

    def too_many_hits(v):
        lib.pack_chunk(fs, 0, 300, v)
        t = v[len(v) // 4 * 4 - 4 * (4 * 300 + 2):len(v) // 4 * 4].view(np.int32)
        t[-2] = cs.max_hits + 1

    for what, fill in (("count", bad_count), ("overlap", overlapping), ("first", first_not_zero),
                       ("hits", too_many_hits)):
        print(f"case: malformed chunk ({what})", flush=True)
        k = cs.submit(fill)
        F, fl = cs.result(k)
        assert F == -1 and len(fl) == 0, what
        fb, cb, _ = cs.slots[k]["sel"].result()
        assert not fb.any() and not cb.any(), what

    def decreasing(v):
        lib.pack_chunk(fs, 0, 300, v)
        t = v[len(v) // 4 * 4 - 4 * (4 * 300 + 2):len(v) // 4 * 4].view(np.int32)
        t[4 * 10 + 2] = t[4 * 10 + 1] - 1   # frame 10, layer 1 count negative
    print("case: chunk with decreasing offsets", flush=True)
    k = cs.submit(decreasing)
    F, fl = cs.result(k)
    assert F == 300
    assert cs.slots[k]["sel"].counters()[2] & 4
    dh = lib.to_device(fs)
    ref = lib.select_frames(dh, p)
    torch.cuda.synchronize()
    rf = ref.result()[0]
    assert fl[10] == 0 and fl[9] == rf[9] and np.array_equal(fl[12:], rf[12:])


def test_frame_pairs_find_tracks_across_frames(lib):
    """Tracks across a frame boundary (Section VII): the merged frame pairs
    built on the GPU equal their host definition bit for bit; the selection
    on them matches the oracle run on the host-built pairs; and of the
    generator's particles that cross a frame boundary with a hit on every
    layer, the frame pairs find most as tracks with exactly their four hits,
    which the frames on their own cannot (their hits sit in two frames)."""
    import torch
    from helpers import Frames, merge_pairs
    fs = synth.generate(7, n_frames=2000, salt=51)
    p = default_params()
    dh = lib.to_device(fs)
    print("case: frame pairs of 2000 frames", flush=True)
    ph = lib.pair_frames(dh)
    torch.cuda.synchronize()
    x, y, z, off, orig = merge_pairs(fs)
    n = int(off[-1])
    assert np.array_equal(ph.layer_offsets.cpu().numpy(), off)
    assert np.array_equal(ph.x[:n].cpu().numpy(), x) and np.array_equal(ph.y[:n].cpu().numpy(), y)
    assert np.array_equal(ph.z[:n].cpu().numpy(), z)
    pf = synth.FrameSet(x, y, z, np.zeros(n, np.uint16), np.zeros(n, np.uint16), off, fs.pid[orig], {},
                        np.zeros(fs.n_frames - 1, bool))
    sel = lib.select_frames(ph, p)
    torch.cuda.synchronize()
    flags, counts, vtx = sel.result()
    trips, tracks, kf, c = sel.lists(off)
    assert c[2] == 0
    orc = oracle.run(pf, p)
    bad, stats = compare(orc, flags, counts, vtx, trips, tracks, kf)
    print("frame pairs", stats, flush=True)
    assert_parity(bad, stats, "frame pairs")
    # recovery of the particles that cross a frame boundary
    _, _, table = synth.true_triplets(fs)
    st = fs.particles["straddle"][:len(table)]
    cross = (st >= 0) & np.all(table >= 0, axis=1)
    assert cross.sum() > 100
    want = {tuple(r) for r in table[cross].tolist()}
    found_pairs = {tuple(r) for r in orig[tracks[:, 1:5]].tolist()} & want
    single = lib.select_frames(dh, p)
    torch.cuda.synchronize()
    _, tr1, _, _ = single.lists(fs.layer_offsets)
    found_single = {tuple(r) for r in tr1[:, 1:5].tolist()} & want
    eff_pairs, eff_single = len(found_pairs) / len(want), len(found_single) / len(want)
    print(f"crossing particles {len(want)}: found by the pairs {eff_pairs:.3f}, by the frames {eff_single:.3f}",
          flush=True)
    assert eff_single == 0.0 and eff_pairs > 0.7


def test_vertex_entry_point_malformed(lib):
    """mu3e_vertex on hand-made track ranges: a track with a hit index
    outside [0, n_hits) is ignored (the frame gives what it gives without
    that track), a decreasing range and a range past n_tracks form no
    triple (no flag, no combination, NaN vertex); the other frames match
    the oracle."""
    import torch
    cfg = dataclasses.replace(synth.CONFIGS[1], lam=1.0, noise_per_layer=1, signal_frac=0.6)
    fs = synth.generate(cfg, n_frames=300, salt=11)
    p = default_params()
    orc = oracle.run(fs, p)
    k = orc.tracks[(orc.tracks[:, 6] == 1) & (orc.tracks[:, 7] == 0)]
    cand = [f for f in range(fs.n_frames) if orc.amb[f] == 0 and (orc.flags[f] & (2 | 4 | 32)) == 0
            and (orc.flags[f] & 16) and (k[:, 0] == f).sum() >= 4]
    assert len(cand) >= 2
    fa, fb = cand[0], cand[1]
    ta = k[k[:, 0] == fa][:, 1:5].astype(np.int32)
    tb = k[k[:, 0] == fb][:, 1:5].astype(np.int32)
    bad = ta.copy()
    bad[1, 2] = fs.n_hits
    bad2 = ta.copy()
    bad2[1, 0] = -1
    drop = np.delete(ta, 1, axis=0)
    hits = np.concatenate([ta, bad, bad2, drop, tb])
    n = len(hits)
    ends = np.cumsum([len(ta), len(bad), len(bad2), len(drop), len(tb)])
    off = np.array([0, *ends, 5, n + 7], np.int32)       # frame 5 decreasing, frame 6 past the end
    print(f"case: vertex malformed, {n} tracks, offsets {off.tolist()}", flush=True)
    dh = lib.to_device(fs)
    gf, gc, gv = lib.vertex(dh, torch.from_numpy(hits).cuda(), torch.from_numpy(off).cuda(), p)
    gf, gc, gv = gf.cpu().numpy(), gc.cpu().numpy(), gv.cpu().numpy()
    for g, f in ((0, fa), (4, fb)):
        assert gf[g] & 24 == orc.flags[f] & 24 and gc[g] == orc.counts[f, 2]
        assert np.allclose(gv[g, :3], orc.vertex[f, :3], rtol=1e-4, atol=1e-3)
    for g in (1, 2):
        assert gf[g] == gf[3] and gc[g] == gc[3]
        assert np.array_equal(np.isnan(gv[g]), np.isnan(gv[3]))
        assert np.allclose(gv[g], gv[3], rtol=1e-6, atol=1e-6, equal_nan=True)
    assert np.all(gf[5:] == 0) and np.all(gc[5:] == 0) and np.all(np.isnan(gv[5:]))


def test_deterministic_outputs(lib):
    import torch
    fs = synth.generate(2, n_frames=2000)
    dh = lib.to_device(fs)
    p = default_params()
    a = lib.select_frames(dh, p)
    b = lib.select_frames(dh, p)
    torch.cuda.synchronize()
    fa, ca, va = a.result()
    fb, cb, vb = b.result()
    assert np.array_equal(fa, fb) and np.array_equal(ca, cb)
    assert np.array_equal(np.nan_to_num(va), np.nan_to_num(vb))
    ta, ka, kfa, _ = a.lists(fs.layer_offsets)
    tb, kb, kfb, _ = b.lists(fs.layer_offsets)
    assert sorted(map(tuple, ta.tolist())) == sorted(map(tuple, tb.tolist()))
    assert sorted(map(tuple, ka.tolist())) == sorted(map(tuple, kb.tolist()))


def sampled_parity(fs, p, sel, what, n_pick=2000, seed=7):
    """Compare a selector's outputs over a whole batch with the oracle run
    frame by frame on n_pick sampled frames; check properties that hold
    for every frame."""
    flags, counts, vtx = sel.result()
    trips, tracks, kf, c = sel.lists(fs.layer_offsets)
    assert c[2] == 0
    rng = np.random.default_rng(seed)
    pick = np.sort(rng.choice(fs.n_frames, n_pick, replace=False))
    # group the lists by frame once (a stable sort keeps each frame's rows in
    # list order), so each picked frame's rows are one contiguous slice
    ot = np.argsort(trips[:, 0], kind="stable")
    trips = trips[ot]
    ok_ = np.argsort(tracks[:, 0], kind="stable")
    tracks, kf = tracks[ok_], kf[ok_]
    t_lo, t_hi = np.searchsorted(trips[:, 0], pick, "left"), np.searchsorted(trips[:, 0], pick, "right")
    k_lo, k_hi = np.searchsorted(tracks[:, 0], pick, "left"), np.searchsorted(tracks[:, 0], pick, "right")
    # oracle on the picked frames, one sub-batch per frame (hit indices rebased)
    sub_trips, sub_tracks, sub_kf = [], [], []
    orcs = []
    for i, f in enumerate(pick):
        sub = fs.subset(int(f), int(f) + 1)
        orcs.append(oracle.run(sub, p))
        base = fs.layer_offsets[4 * f]
        t = trips[t_lo[i]:t_hi[i]].copy(); t[:, 0] = i; t[:, 1:] -= base
        sub_trips.append(t)
        k = tracks[k_lo[i]:k_hi[i]].copy(); k[:, 0] = i; k[:, 1:] -= base
        sub_tracks.append(k)
        sub_kf.append(kf[k_lo[i]:k_hi[i]])
    # merge the per-frame oracle results into one result over len(pick) frames
    orc = oracle.OracleResult(
        np.concatenate([o.flags for o in orcs]), np.concatenate([o.amb for o in orcs]),
        np.concatenate([o.counts for o in orcs]), np.concatenate([o.namb for o in orcs]),
        np.concatenate([o.vertex for o in orcs]), sum(o.stats for o in orcs), 0.0)

    def cat(name, idx_cols):
        out = []
        for i, o in enumerate(orcs):
            a = getattr(o, name).copy()
            a[:, 0] = i
            out.append(a)
        return np.concatenate(out) if out else np.zeros((0, idx_cols))
    orc.trips = cat("trips", 6)
    orc.trip_rtc = np.concatenate([o.trip_rtc for o in orcs])
    orc.tracks = cat("tracks", 8)
    orc.track_f = np.concatenate([o.track_f for o in orcs])
    orc.triples = cat("triples", 12)
    bad, stats = compare(orc, flags, counts, vtx, np.concatenate(sub_trips), np.concatenate(sub_tracks),
                         np.concatenate(sub_kf), frames=pick)
    print(what, stats, flush=True)
    assert_parity(bad, stats, what)
    # properties over all frames: counts non-negative, KEEP iff another bit
    keep = (flags & 1) != 0
    assert np.array_equal(keep, (flags & 62) != 0)
    assert np.all(counts >= 0)


def test_full_nominal_sampled(lib):
    """The benchmark workload (100,000 nominal frames) in both forms, each in
    the launch configuration the benchmark times (the batched form with the
    autotuned shape), compared with the oracle on 2,000 sampled frames."""
    import torch
    from paper_2206_11535_amd import autotune
    fs = synth.generate(2)
    p = default_params()
    print(f"case: full cfg2 {fs.n_frames} frames", flush=True)
    dh = lib.to_device(fs)
    sel = lib.select_frames(dh, p)
    torch.cuda.synchronize()
    sampled_parity(fs, p, sel, "full cfg2 sampled, plain")
    shape, _, _ = autotune.tune(dh, p)
    print(f"case: full cfg2 batched shape {shape}", flush=True)
    b = lib.BatchedSelector(dh, p, **autotune.as_kwargs(shape))
    b.run()
    torch.cuda.synchronize()
    sampled_parity(fs, p, b, "full cfg2 sampled, batched", seed=8)


def test_full_mixed_sampled(lib):
    """The mixed-rate 1,000,000-frame batch in the batched form with the
    autotuned shape, compared with the oracle on 2,000 sampled frames."""
    import torch
    from paper_2206_11535_amd import autotune
    fs = synth.generate(3)
    p = default_params()
    print(f"case: full cfg3 {fs.n_frames} frames", flush=True)
    dh = lib.to_device(fs)
    shape, _, _ = autotune.tune(dh, p)
    print(f"case: full cfg3 batched shape {shape}", flush=True)
    b = lib.BatchedSelector(dh, p, **autotune.as_kwargs(shape))
    b.run()
    torch.cuda.synchronize()
    sampled_parity(fs, p, b, "full cfg3 sampled, batched", seed=9)


# triplet-list and vertex-track capacities of the full lifted-cap batches
# (about twice what they produce)
FULL_CAPS = {4: (1 << 26, 1 << 23), 6: (1 << 27, 1 << 23)}


@pytest.mark.parametrize("cfg", [4, 6])
def test_full_lifted_sampled(lib, cfg):
    """The full pile-up batch (200,000 frames, lambda = 30, 20 noise hits per
    layer) and the full phase-II batch (100,000 frames at lambda = 64), caps
    lifted so that every frame runs every stage (no frame kept for
    overflowing): the plain form and the batched form with the autotuned
    shape give identical outputs, and both match the oracle on 2,000 sampled
    frames."""
    import torch
    from paper_2206_11535_amd import autotune
    fs = synth.generate(cfg)
    p = lifted_caps()
    tc, kc = FULL_CAPS[cfg]
    print(f"case: full cfg{cfg} {fs.n_frames} frames, lifted caps", flush=True)
    dh = lib.to_device(fs)
    sel = lib.Selector(fs.n_frames, p, triplet_capacity=tc, track_capacity=kc)
    sel.run(dh)
    torch.cuda.synchronize()
    sampled_parity(fs, p, sel, f"full cfg{cfg} sampled, plain", seed=10 + cfg)
    shape, _, _ = autotune.tune(dh, p, tc, kc)
    print(f"case: full cfg{cfg} batched shape {shape}", flush=True)
    b = lib.BatchedSelector(dh, p, tc, kc, **autotune.as_kwargs(shape))
    b.run()
    torch.cuda.synchronize()
    fa, ca, va = sel.result()
    fb, cb, vb = b.result()
    assert np.array_equal(fa, fb) and np.array_equal(ca, cb)
    assert np.array_equal(np.nan_to_num(va), np.nan_to_num(vb))
    sampled_parity(fs, p, b, f"full cfg{cfg} sampled, batched", seed=20 + cfg)
    # nothing is kept for overflowing; only signal-like vertices keep frames
    assert not (fa & (2 | 4 | 8 | 32)).any()
    assert ca[:, 0].mean() > 100


@pytest.mark.parametrize("cfg,n,fuse,steal", [(2, 3000, 0, 25), (3, 5000, 1, 50), (1, 1000, 0, 0), (2, 2000, 1, 100)])
def test_batched_equals_plain_and_oracle(lib, cfg, n, fuse, steal):
    """The batched persistent form gives exactly the plain form's outputs
    and matches the oracle."""
    import torch
    fs = synth.generate(cfg, n_frames=n)
    p = default_params()
    dh = lib.to_device(fs)
    print(f"case: batched cfg{cfg}[:{n}] fused={fuse} steal={steal}%", flush=True)
    a = lib.select_frames(dh, p)
    b = lib.BatchedSelector(dh, p, waves_per_cu=8, frames_per_claim=4, fuse_fits=fuse, steal_percent=steal)
    b.run()
    torch.cuda.synchronize()
    fa, ca, va = a.result()
    fb, cb, vb = b.result()
    assert np.array_equal(fa, fb) and np.array_equal(ca, cb)
    assert np.array_equal(np.nan_to_num(va), np.nan_to_num(vb))
    ta, ka, kfa, _ = a.lists(fs.layer_offsets)
    tb, kb, kfb, c = b.lists(fs.layer_offsets)
    assert c[2] == 0
    assert sorted(map(tuple, ta.tolist())) == sorted(map(tuple, tb.tolist()))
    assert sorted(map(tuple, ka[:, :5].tolist())) == sorted(map(tuple, kb[:, :5].tolist()))
    orc = oracle.run(fs, p)
    bad, stats = compare(orc, fb, cb, vb, tb, kb, kfb)
    assert_parity(bad, stats, f"batched cfg{cfg}")


@pytest.mark.parametrize("w,c,fuse,steal", [(1, 1, 1, 100), (2, 32, 0, 50), (20, 3, 1, 0), (32, 8, 0, 12)])
def test_batched_shapes_and_repeat(lib, w, c, fuse, steal):
    """Any shape gives the same result, also on a second run of the plan."""
    import torch
    fs = synth.generate(3, n_frames=4000)
    p = default_params()
    dh = lib.to_device(fs)
    ref = lib.select_frames(dh, p)
    print(f"case: batched shape {w} waves/CU, {c} frames/claim, fused={fuse}, steal={steal}%", flush=True)
    b = lib.BatchedSelector(dh, p, waves_per_cu=w, frames_per_claim=c, fuse_fits=fuse, steal_percent=steal)
    for rep in range(3):
        # outputs overwritten with sentinels, so that every replay of the
        # graph must write them all again; eager work between the replays
        b.flags.fill_(-1)
        b.counts.fill_(-1)
        b.vertex.fill_(7.0)
        b.run()
        torch.cuda.synchronize()
        fr, cr, vr = ref.result()
        fb, cb, vb = b.result()
        assert np.array_equal(fr, fb) and np.array_equal(cr, cb), (w, c, rep)
        assert np.array_equal(np.nan_to_num(vr), np.nan_to_num(vb)), (w, c, rep)
        ref.run(dh)
        torch.cuda.synchronize()
    # the eager, event-bracketed launch of the same plan (outputs cleared first)
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
    hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
    ev = (ctypes.c_void_p * 4)()
    for i in range(4):
        e = ctypes.c_void_p()
        assert hip.hipEventCreate(ctypes.byref(e)) == 0
        ev[i] = e
    b.flags.fill_(-1)
    b.counts.fill_(-1)
    b.run(None, torch.cuda.current_stream(), events=ev)
    torch.cuda.synchronize()
    fb, cb, vb = b.result()
    assert np.array_equal(fr, fb) and np.array_equal(cr, cb) and np.array_equal(np.nan_to_num(vr), np.nan_to_num(vb))
    ms = ctypes.c_float()
    assert hip.hipEventElapsedTime(ctypes.byref(ms), ev[0], ev[1]) == 0 and ms.value > 0
    assert hip.hipEventElapsedTime(ctypes.byref(ms), ev[1], ev[2]) == 0 and ms.value >= 0
    assert hip.hipEventElapsedTime(ctypes.byref(ms), ev[2], ev[3]) == 0 and ms.value >= 0
    for i in range(4):
        hip.hipEventDestroy(ev[i])
