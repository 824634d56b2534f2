"""Host logic of the autotuner of the batched form: the candidate shapes,
the cache key, and the source tag that invalidates cached shapes when the
kernel sources or build flags change."""
import json
import os
import shutil
from types import SimpleNamespace

from paper_2206_11535_amd import autotune


def test_candidates():
    c = autotune.cyclic_candidates()
    assert len(c) == len(set(c))
    # the purely cyclic schedule at every wave count, tile size and fusion
    for t in autotune.TILE_HITS:
        for u in autotune.FUSE_FITS:
            for w in autotune.WAVES_PER_CU:
                assert (w, 0, u, 0, t, 1) in c
    assert set(autotune.TILE_HITS) == {64, 128}
    best = (20, 0, 1, 0, 64, 1)
    s = autotune.steal_candidates(best)
    assert len(s) == len(set(s))
    for w, claim, u, st, t, n in s:
        assert (u, t, n) == (1, 64, 1)
        assert st in autotune.STEAL_PERCENT and claim in autotune.FRAMES_PER_CLAIM
        assert w in autotune.STEAL_WAVES_PER_CU or w == 20
    sp = autotune.split_candidates((8, 4, 0, 25, 128, 1))
    assert sp == [(8, 4, 0, 25, 128, n) for n in autotune.SUB_BATCHES if n > 1]
    assert autotune.as_kwargs((8, 4, 0, 25, 128, 2)) == dict(waves_per_cu=8, frames_per_claim=4, fuse_fits=0,
                                                            steal_percent=25, tile_hits=128, sub_batches=2)


def test_workload_key_rounds_hits_per_frame():
    import torch
    k = autotune.workload_key(SimpleNamespace(n_frames=100000, n_hits=4_270_000), "gfx950")
    assert k == f"gfx950|rocm{torch.version.hip}|src{autotune.source_tag()}|F100000|hpf44"
    # frames without hits, and a batch without frames
    assert autotune.workload_key(SimpleNamespace(n_frames=10, n_hits=0), "gfx950").endswith("|F10|hpf0")
    assert autotune.workload_key(SimpleNamespace(n_frames=0, n_hits=0), "gfx950").endswith("|F0|hpf0")


def test_source_tag_follows_kernel_sources(tmp_path, monkeypatch):
    tag = autotune.source_tag()
    assert len(tag) == 10 and int(tag, 16) >= 0
    assert autotune.source_tag() == tag
    pkg = tmp_path / "pkg"
    shutil.copytree(os.path.join(autotune.PKG, "csrc"), pkg / "csrc",
                    ignore=shutil.ignore_patterns("__pycache__", "*.o", "*.so"))
    shutil.copy(os.path.join(autotune.PKG, "build.py"), pkg / "build.py")
    monkeypatch.setattr(autotune, "PKG", str(pkg))
    assert autotune.source_tag() == tag
    (pkg / "build.py").write_text((pkg / "build.py").read_text() + "\n# changed\n")
    t2 = autotune.source_tag()
    assert t2 != tag
    hip = sorted(p for p in (pkg / "csrc").iterdir() if p.suffix == ".hip")[0]
    hip.write_text(hip.read_text() + "\n// changed\n")
    assert autotune.source_tag() not in (tag, t2)
    # files other than kernel sources do not count
    (pkg / "csrc" / "notes.txt").write_text("x")
    t3 = autotune.source_tag()
    (pkg / "csrc" / "notes.txt").write_text("y")
    assert autotune.source_tag() == t3


def test_committed_cache_is_well_formed():
    with open(autotune.CACHE) as f:
        cache = json.load(f)
    assert cache
    for key, e in cache.items():
        arch, rocm, src, frames, hpf = key.split("|")
        assert arch.startswith("gfx") and rocm.startswith("rocm") and src.startswith("src")
        assert frames.startswith("F") and hpf.startswith("hpf")
        assert set(e) == set(autotune.FIELDS) | {"ms"}
        assert e["ms"] > 0
        # the shape in effect may be capped by occupancy below the one asked
        # for, so only the schedule parameters are checked against the lists
        assert e["tile_hits"] in autotune.TILE_HITS and e["fuse_fits"] in autotune.FUSE_FITS
        assert e["sub_batches"] in autotune.SUB_BATCHES
        assert 1 <= e["waves_per_cu"] <= max(autotune.WAVES_PER_CU)
        if e["steal_percent"]:
            assert e["steal_percent"] in autotune.STEAL_PERCENT
            assert e["frames_per_claim"] in autotune.FRAMES_PER_CLAIM
