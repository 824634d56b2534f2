"""Set comparison of the HIP path's outputs with the oracle's.

Candidates the oracle marks ambiguous (a tested quantity within 1e-5
relative of a window edge, a near-tie in the nearest-hit choice, a circle
tangency) are dropped from both sides together with everything derived from
them; the rest must match exactly:
  * passing triplets (frame, h0, h1, h2);
  * tracks keyed by their triplet: layer-3 hit and charge;
  * frame flags (bits the oracle marks ambiguous are skipped);
  * per-stage counts within [sure, sure + ambiguous];
  * track kappa_bar and chi2 within 1e-4 relative (chi2 with an absolute
    floor of 1), reported vertex within 1e-4 relative / 1e-3 mm.
"""
from __future__ import annotations

import numpy as np

KEEP, TRIPLET_OVF, TRACK_OVF, COMBO_OVF, VERTEX, HITS_OVF = 1, 2, 4, 8, 16, 32


def compare(orc, gflags, gcounts, gvertex, gtrips=None, gtracks=None, gkf=None, frames=None,
            rel=1e-4, vtx_abs=1e-3):
    """orc: OracleResult over frames 0..n-1 (optionally a subset of the GPU
    frames: `frames[i]` is the GPU frame index of oracle frame i, and the
    list inputs are then already restricted and renumbered).  Returns a dict
    of mismatch lists (all empty on parity) and statistics."""
    F = len(orc.flags)
    fmap = np.arange(F) if frames is None else np.asarray(frames)
    gflags = np.asarray(gflags).astype(np.uint32)[fmap]
    gcounts = np.asarray(gcounts)[fmap]
    gvertex = np.asarray(gvertex)[fmap]
    bad = {"flags": [], "counts": [], "vertex": [], "triplets_missing": [], "triplets_extra": [],
           "tracks_missing": [], "tracks_extra": [], "tracks_diff": [], "track_params": []}
    stats = {"frames": F, "amb_frames": int(np.sum(orc.amb != 0))}
    # ---- flags
    for f in range(F):
        amb = int(orc.amb[f])
        mask = ~amb & 0x3F
        if amb:
            mask &= ~KEEP
        if (int(gflags[f]) ^ int(orc.flags[f])) & mask:
            bad["flags"].append((int(fmap[f]), int(gflags[f]), int(orc.flags[f]), amb))
    # ---- counts
    for f in range(F):
        c, n = orc.counts[f], orc.namb[f]
        up = 0
        for s in range(3):
            if up:
                break
            if s == 1 and orc.flags[f] & (TRIPLET_OVF | HITS_OVF):
                break
            if s == 2 and orc.flags[f] & (TRACK_OVF | TRIPLET_OVF | HITS_OVF):
                break
            g = int(gcounts[f, s])
            if not (c[s] <= g <= c[s] + n[s]):
                bad["counts"].append((int(fmap[f]), s, g, int(c[s]), int(n[s])))
            up += n[s]
    # ---- vertex
    for f in range(F):
        if orc.amb[f] & VERTEX or not (orc.flags[f] & VERTEX) or not (gflags[f] & VERTEX):
            continue
        o, g = orc.vertex[f], gvertex[f].astype(np.float64)
        tol_xyz = np.maximum(vtx_abs, rel * np.abs(o[:3]))
        if np.any(np.abs(g[:3] - o[:3]) > tol_xyz) or abs(g[3] - o[3]) > rel * max(abs(o[3]), 1.0):
            bad["vertex"].append((int(fmap[f]), g.tolist(), o.tolist()))
    if gtrips is None:
        return bad, stats
    # frames where either side stopped after the cuts are compared on flags only
    ovf = ((orc.flags | gflags) & (TRIPLET_OVF | HITS_OVF)) != 0
    # ---- triplets
    t = orc.trips
    amb_keys = {tuple(r) for r in t[t[:, 5] == 1][:, 0:4].tolist()}
    sure = {tuple(r) for r in t[(t[:, 4] == 1) & (t[:, 5] == 0)][:, 0:4].tolist() if not ovf[r[0]]}
    g = {tuple(r) for r in np.asarray(gtrips)[:, 0:4].tolist() if not ovf[r[0]]}
    bad["triplets_missing"] = sorted(sure - g)
    bad["triplets_extra"] = sorted(g - sure - amb_keys)
    stats["triplets"] = len(sure)
    stats["triplets_amb"] = len(amb_keys)
    # ---- tracks keyed by (frame, h0, h1, h2)
    k = orc.tracks
    amb_trk = amb_keys | {tuple(r) for r in k[k[:, 7] == 1][:, 0:4].tolist()}
    o_trk = {}
    for r, kf in zip(k.tolist(), orc.track_f.tolist()):
        if r[6] == 1 and r[7] == 0 and tuple(r[0:4]) not in amb_trk and not ovf[r[0]]:
            o_trk[tuple(r[0:4])] = (r[4], r[5], kf[0], kf[1])
    g_trk = {}
    for r, kf in zip(np.asarray(gtracks).tolist(), np.asarray(gkf).tolist()):
        if not ovf[r[0]]:
            g_trk[tuple(r[0:4])] = (r[4], 1 if kf[0] > 0 else -1, kf[0], kf[1])
    gk = {key for key in g_trk if key not in amb_trk}
    bad["tracks_missing"] = sorted(set(o_trk) - gk)
    bad["tracks_extra"] = sorted(gk - set(o_trk))
    for key in set(o_trk) & gk:
        o, gg = o_trk[key], g_trk[key]
        if o[0] != gg[0] or o[1] != gg[1]:
            bad["tracks_diff"].append((key, gg[:2], o[:2]))
            continue
        if abs(gg[2] - o[2]) > rel * abs(o[2]) or abs(gg[3] - o[3]) > rel * max(abs(o[3]), 1.0):
            bad["track_params"].append((key, gg[2:], o[2:]))
    stats["tracks"] = len(o_trk)
    stats["tracks_amb"] = len(amb_trk)
    return bad, stats


def assert_parity(bad, stats, what=""):
    msg = {k: v[:5] for k, v in bad.items() if len(v)}
    n = {k: len(v) for k, v in bad.items() if len(v)}
    assert not msg, f"{what} parity failures {n}: {msg} stats={stats}"
