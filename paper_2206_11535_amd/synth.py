"""Seeded synthetic Mu3e-shaped readout frames.

This module is the single input source shared by the HIP path and the FP64
oracle.  It simulates the detector (helices in a solenoid field, multiple
scattering, pixel quantisation, noise, sensor misalignment); it contains none
of the selection method's arithmetic (no cuts, no triplet fit, no vertex
estimate).

Physics and geometry (paper, Sections III-B and IV):
  * four cylindrical pixel layers at r = 25, 31, 73, 85 mm (the setup macros
    and the Selection Cuts figure), |z| acceptance 62 mm (inner) / 175 mm
    (outer);
  * a hollow double-cone target, radius 19 mm, half length 50 mm (Selection
    Cuts figure, Section IV-C "target ... disk with a radius of 19mm");
  * a 1 T solenoid field parallel to the beam line (Section III-B); positive
    charges turn clockwise seen from +z;
  * Michel positrons mu+ -> e+ nu nu and signal decays mu+ -> e+ e- e+ at
    rest with sum p = 0, sum E = m_mu (Section III-A, eq. conservation-laws);
  * frames are 64 ns snapshots; at 1e8 mu/s a frame holds Poisson(6.4) decays.

Multiple scattering uses the Highland formula with 0.1 % X0 per layer; hits
are quantised to 80 um pixel centres in (r*phi, z) and put back on the
cylinder.  A particle records the first outward crossing of each layer that
falls inside that layer's z acceptance; there are no recurl re-hits and no
energy loss.

Draw order (fixed, one PCG64 stream per configuration):
  1 per-frame lambda (mixed-rate configuration only), 2 Michel counts,
  3 signal flags, 4 decay vertices, 5 Michel momenta, 6 Michel directions,
  7 signal kinematics (Dalitz point, orientation), 8 scattering angles
  (per layer, two per particle), 9 noise hits, 10 in-layer shuffle keys,
  11 misalignment, 12 frame-straddling particles and their first layer in
  the next frame (only when straddle_frac > 0, so that other configurations
  draw nothing).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

# ---------------------------------------------------------------- constants
R_LAYER = np.array([25.0, 31.0, 73.0, 85.0])
Z_HALF = np.array([62.0, 62.0, 175.0, 175.0])
B_TESLA = 1.0
C_LIGHT = 0.299792458          # p[MeV] = C_LIGHT * B[T] * R[mm]
PIXEL = 0.08                   # mm
X_OVER_X0 = 0.001              # per layer
M_E = 0.51099895               # MeV
M_MU = 105.6583755             # MeV
P_MICHEL_MAX = (M_MU ** 2 + M_E ** 2) / (2.0 * M_MU)   # 52.83 MeV
P_MICHEL_MIN = 10.0
TARGET_R = 19.0
TARGET_HALF = 50.0
# sensor grid per layer: ladders in phi (8/10/24/28, Selection Cuts figure)
# times sensors along z
N_PHI = np.array([8, 10, 24, 28])
N_Z = np.array([6, 6, 18, 18])
SENSOR_BASE = np.concatenate([[0], np.cumsum(N_PHI * N_Z)])[:4]
N_SENSORS = int(np.sum(N_PHI * N_Z))   # 1044


@dataclasses.dataclass
class SynthConfig:
    name: str
    n_frames: int
    lam: float | tuple            # decays per frame, or a tuple to draw from
    noise_per_layer: int
    signal_frac: float
    cfg_id: int
    misalign: bool = False
    misalign_t: float = 0.05      # mm
    misalign_alpha: float = 0.5e-3  # rad
    straddle_frac: float = 0.0    # particles whose later hits fall into the next frame


CONFIGS = {
    1: SynthConfig("nominal-small lambda=2", 1_000, 2.0, 2, 0.10, 1),
    2: SynthConfig("nominal lambda=6.4", 100_000, 6.4, 5, 0.01, 2),
    3: SynthConfig("mixed-rate lambda in {2,6.4,12,20}", 1_000_000,
                   (2.0, 6.4, 12.0, 20.0), 5, 0.01, 3),
    4: SynthConfig("pile-up lambda=30", 200_000, 30.0, 20, 0.01, 4),
    5: SynthConfig("nominal lambda=6.4 misaligned", 100_000, 6.4, 5, 0.01, 5,
                   misalign=True),
    # phase II of the experiment: 1e9 mu/s, ten times the nominal rate
    6: SynthConfig("phase-II lambda=64", 100_000, 64.0, 5, 0.01, 6),
    # nominal rate with 5 % of the particles crossing a frame boundary
    # between two layers (their hits from that layer on belong to the next
    # 64 ns frame)
    7: SynthConfig("nominal lambda=6.4, frame-straddling", 100_000, 6.4, 5, 0.01, 7, straddle_frac=0.05),
}


@dataclasses.dataclass
class FrameSet:
    """Hits of a batch of frames, sorted by (frame, layer).

    x, y, z     float32 [n_hits], mm, global frame
    layer       uint16  [n_hits]
    sensor      uint16  [n_hits]
    layer_offsets int32 [4*n_frames+1]: hits of frame f on layer l are
                [layer_offsets[4f+l], layer_offsets[4f+l+1])
    pid         int32   [n_hits] truth particle index, -1 for noise
    particles   dict of per-particle truth arrays
    frame_signal bool [n_frames]
    align       float64 [N_SENSORS, 4] true (tx, ty, tz, alpha) per sensor
    """
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    layer: np.ndarray
    sensor: np.ndarray
    layer_offsets: np.ndarray
    pid: np.ndarray
    particles: dict
    frame_signal: np.ndarray
    align: Optional[np.ndarray] = None

    @property
    def n_frames(self) -> int:
        return (len(self.layer_offsets) - 1) // 4

    @property
    def n_hits(self) -> int:
        return len(self.x)

    def hits_per_layer(self) -> np.ndarray:
        lo = self.layer_offsets
        return (lo[1:] - lo[:-1]).reshape(-1, 4)

    def subset(self, f0: int, f1: int) -> "FrameSet":
        """Frames [f0, f1) as a new FrameSet (hit indices rebased)."""
        lo = self.layer_offsets
        h0, h1 = int(lo[4 * f0]), int(lo[4 * f1])
        sel = slice(h0, h1)
        return FrameSet(self.x[sel].copy(), self.y[sel].copy(),
                        self.z[sel].copy(), self.layer[sel].copy(),
                        self.sensor[sel].copy(),
                        (lo[4 * f0:4 * f1 + 1] - h0).astype(np.int32),
                        self.pid[sel].copy(), self.particles,
                        self.frame_signal[f0:f1].copy(), self.align)


def _rng(cfg_id: int, salt: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([2206, 11535, cfg_id, salt])))


def highland(p, x_over_x0):
    """Highland width of the projected scattering angle [rad] (beta = 1)."""
    return 13.6 / p * np.sqrt(x_over_x0) * (1.0 + 0.038 * np.log(x_over_x0))


def sample_michel(rng, n):
    """Michel momenta [MeV] with density x^2 (3 - 2x), x = p / p_max, on
    [P_MICHEL_MIN, P_MICHEL_MAX], by rejection (the density peaks at x=1)."""
    out = np.empty(n)
    filled = 0
    xmin = P_MICHEL_MIN / P_MICHEL_MAX
    while filled < n:
        m = max(2 * (n - filled), 64)
        x = rng.uniform(xmin, 1.0, m)
        u = rng.uniform(0.0, 1.0, m)
        acc = x[u <= x * x * (3.0 - 2.0 * x)]
        k = min(len(acc), n - filled)
        out[filled:filled + k] = acc[:k] * P_MICHEL_MAX
        filled += k
    return out


def sample_target(rng, n):
    """Points uniform on the double-cone surface r(z) = R (1 - |z|/L)."""
    # |z| has density proportional to r(|z|): triangular on [0, L]
    u = rng.uniform(0.0, 1.0, n)
    az = TARGET_HALF * (1.0 - np.sqrt(1.0 - u))
    sgn = np.where(rng.uniform(0.0, 1.0, n) < 0.5, -1.0, 1.0)
    phi = rng.uniform(-np.pi, np.pi, n)
    r = TARGET_R * (1.0 - az / TARGET_HALF)
    return np.stack([r * np.cos(phi), r * np.sin(phi), sgn * az], axis=1)


def isotropic(rng, n):
    cz = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(-np.pi, np.pi, n)
    sz = np.sqrt(1.0 - cz * cz)
    return np.stack([sz * np.cos(ph), sz * np.sin(ph), cz], axis=1)


def random_rotations(rng, n):
    """Uniform random rotation matrices (from uniform unit quaternions)."""
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1),
    ], axis=1)


def sample_signal(rng, n):
    """mu+ -> e+ e- e+ at rest, flat three-body phase space.

    Returns momenta [n, 3(particle), 3(xyz)] and charges (+1, -1, +1).
    The Dalitz point (m12^2, m23^2) is uniform inside the kinematic boundary.
    """
    M, m = M_MU, M_E
    lo12, hi12 = (2 * m) ** 2, (M - m) ** 2
    out_s12 = np.empty(n)
    out_s23 = np.empty(n)
    filled = 0
    while filled < n:
        k = max(2 * (n - filled), 64)
        s12 = rng.uniform(lo12, hi12, k)
        s23 = rng.uniform(lo12, hi12, k)
        # boundary of s23 at fixed s12 (particles 1,2,3 all of mass m)
        e2s = s12 / (2 * np.sqrt(s12))                      # E2 in 12 frame
        e3s = (M * M - s12 - m * m) / (2 * np.sqrt(s12))    # E3 in 12 frame
        p2s = np.sqrt(np.maximum(e2s ** 2 - m * m, 0.0))
        p3s = np.sqrt(np.maximum(e3s ** 2 - m * m, 0.0))
        s23min = (e2s + e3s) ** 2 - (p2s + p3s) ** 2
        s23max = (e2s + e3s) ** 2 - (p2s - p3s) ** 2
        ok = (s23 >= s23min) & (s23 <= s23max)
        acc12, acc23 = s12[ok], s23[ok]
        t = min(len(acc12), n - filled)
        out_s12[filled:filled + t] = acc12[:t]
        out_s23[filled:filled + t] = acc23[:t]
        filled += t
    s12, s23 = out_s12, out_s23
    s13 = M * M + 3 * m * m - s12 - s23
    E1 = (M * M + m * m - s23) / (2 * M)
    E2 = (M * M + m * m - s13) / (2 * M)
    E3 = M - E1 - E2
    p1 = np.sqrt(np.maximum(E1 ** 2 - m * m, 0.0))
    p2 = np.sqrt(np.maximum(E2 ** 2 - m * m, 0.0))
    p3 = np.sqrt(np.maximum(E3 ** 2 - m * m, 0.0))
    # p1 along x, p2 in the xy plane; p3 = -(p1 + p2)
    c12 = np.clip((p3 ** 2 - p1 ** 2 - p2 ** 2) / (2 * p1 * p2), -1.0, 1.0)
    s12a = np.sqrt(1.0 - c12 ** 2)
    v1 = np.stack([p1, np.zeros(n), np.zeros(n)], 1)
    v2 = np.stack([p2 * c12, p2 * s12a, np.zeros(n)], 1)
    v3 = -(v1 + v2)
    rot = random_rotations(rng, n)
    mom = np.stack([np.einsum('nij,nj->ni', rot, v) for v in (v1, v2, v3)], 1)
    return mom


def quantise(phi_true, z_true, R):
    """80 um pixel centres in (u = R phi, z); returns (x, y, z)."""
    u = R * phi_true
    uq = (np.floor(u / PIXEL) + 0.5) * PIXEL
    zq = (np.floor(z_true / PIXEL) + 0.5) * PIXEL
    return R * np.cos(uq / R), R * np.sin(uq / R), zq


def propagate(rng, pos, mom, charge, ms=True, quant=True, accept=True, ms_layers=(0, 1, 2, 3)):
    """Propagate particles through the four layers.

    pos, mom: [n, 3]; charge: [n] (+1/-1).  Returns hit arrays
    (pid, layer, x, y, z) for the recorded crossings.  ms / quant / accept
    switch multiple scattering, pixel quantisation and the z acceptance off
    (noiseless helices for closed-form checks); ms_layers restricts the
    scattering to the listed layers (the angles are drawn for every layer
    either way, so the draw order does not change).
    """
    n = len(charge)
    pos = pos.copy()
    mom = mom.copy()
    alive = np.ones(n, bool)
    rec = []
    for layer in range(4):
        R = R_LAYER[layer]
        pt = np.hypot(mom[:, 0], mom[:, 1])
        rho = pt / (C_LIGHT * B_TESLA)
        ux, uy = mom[:, 0] / pt, mom[:, 1] / pt
        # centre on the right of the motion for q > 0 (clockwise)
        cx = pos[:, 0] + charge * rho * uy
        cy = pos[:, 1] - charge * rho * ux
        cn = np.hypot(cx, cy)
        ax, ay = pos[:, 0] - cx, pos[:, 1] - cy
        with np.errstate(invalid='ignore', divide='ignore'):
            C = (R * R - cn * cn - rho * rho) / (2.0 * rho * cn)
        reach = alive & (np.abs(C) <= 1.0)
        psi0 = np.arctan2(ay, ax)
        gam = np.arctan2(cy, cx)
        acC = np.arccos(np.clip(C, -1.0, 1.0))
        # the position angle psi(phi) = psi0 - q*phi; solutions of
        # cos(psi - gam) = C: psi = gam +- acos(C)
        two_pi = 2.0 * np.pi
        phiA = np.mod(charge * (psi0 - (gam + acC)), two_pi)
        phiB = np.mod(charge * (psi0 - (gam - acC)), two_pi)
        dphi = np.minimum(phiA, phiB)
        psi = psi0 - charge * dphi
        nx = cx + rho * np.cos(psi)
        ny = cy + rho * np.sin(psi)
        nz = pos[:, 2] + rho * dphi * mom[:, 2] / pt
        # direction after turning by dphi
        cd, sd = np.cos(-charge * dphi), np.sin(-charge * dphi)
        npx = cd * mom[:, 0] - sd * mom[:, 1]
        npy = sd * mom[:, 0] + cd * mom[:, 1]
        inside = reach & ((np.abs(nz) <= Z_HALF[layer]) | (not accept))
        # scattering angles are drawn for every particle (fixed draw order)
        th = rng.normal(size=(n, 2))
        pos = np.where(reach[:, None], np.stack([nx, ny, nz], 1), pos)
        mom = np.where(reach[:, None], np.stack([npx, npy, mom[:, 2]], 1), mom)
        alive = reach
        idx = np.nonzero(inside)[0]
        if len(idx):
            if quant:
                phi_t = np.arctan2(pos[idx, 1], pos[idx, 0])
                hx, hy, hz = quantise(phi_t, pos[idx, 2], R)
            else:
                hx, hy, hz = pos[idx, 0].copy(), pos[idx, 1].copy(), pos[idx, 2].copy()
            rec.append((idx, np.full(len(idx), layer), hx, hy, hz))
            if not ms or layer not in ms_layers:
                continue
            # multiple scattering in the sensor material
            p = np.linalg.norm(mom[idx], axis=1)
            t = mom[idx] / p[:, None]
            nr = np.stack([pos[idx, 0] / R, pos[idx, 1] / R, np.zeros(len(idx))], 1)
            cosinc = np.abs(np.sum(t * nr, axis=1))
            theta0 = highland(p, X_OVER_X0 / np.maximum(cosinc, 1e-3))
            e1 = np.cross(t, np.array([0.0, 0.0, 1.0]))
            e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
            e2 = np.cross(t, e1)
            a1 = theta0 * th[idx, 0]
            a2 = theta0 * th[idx, 1]
            ang = np.hypot(a1, a2)
            with np.errstate(invalid='ignore', divide='ignore'):
                k = np.where(ang > 0, np.sin(ang) / ang, 1.0)
            tn = np.cos(ang)[:, None] * t + k[:, None] * (a1[:, None] * e1 + a2[:, None] * e2)
            tn /= np.linalg.norm(tn, axis=1, keepdims=True)
            mom[idx] = tn * p[:, None]
    if not rec:
        e = np.zeros(0)
        return e.astype(np.int64), e.astype(np.int64), e, e, e
    pid = np.concatenate([r[0] for r in rec])
    lay = np.concatenate([r[1] for r in rec])
    hx = np.concatenate([r[2] for r in rec])
    hy = np.concatenate([r[3] for r in rec])
    hz = np.concatenate([r[4] for r in rec])
    return pid, lay, hx, hy, hz


def sensor_of(layer, x, y, z):
    phi = np.arctan2(y, x)
    nphi = N_PHI[layer]
    nz = N_Z[layer]
    iphi = np.clip(np.floor((phi + np.pi) / (2 * np.pi) * nphi), 0, nphi - 1).astype(np.int64)
    zh = Z_HALF[layer]
    iz = np.clip(np.floor((z + zh) / (2 * zh) * nz), 0, nz - 1).astype(np.int64)
    return SENSOR_BASE[layer] + iphi * nz + iz


def generate(cfg: SynthConfig | int, n_frames: Optional[int] = None,
             salt: int = 0) -> FrameSet:
    """Generate a configuration (optionally only its first n_frames).

    Generation is vectorised over all particles of all frames; a prefix of
    n_frames is produced from the same stream layout but is not a prefix of
    the full configuration's frames (the streams are consumed in bulk).
    """
    if isinstance(cfg, int):
        cfg = CONFIGS[cfg]
    F = cfg.n_frames if n_frames is None else int(n_frames)
    rng = _rng(cfg.cfg_id, salt)
    # 1 per-frame lambda
    if isinstance(cfg.lam, tuple):
        lam = np.asarray(cfg.lam)[rng.integers(0, len(cfg.lam), F)]
    else:
        lam = np.full(F, float(cfg.lam))
    # 2 Michel counts, 3 signal flags
    n_mich = rng.poisson(lam)
    sig = rng.uniform(0.0, 1.0, F) < cfg.signal_frac
    n_sig = 3 * sig.astype(np.int64)
    n_tot = n_mich + n_sig
    P = int(n_tot.sum())
    frame_of = np.repeat(np.arange(F), n_tot)
    # particle order inside a frame: Michel positrons, then the signal triple
    first = np.concatenate([[0], np.cumsum(n_tot)[:-1]])
    local = np.arange(P) - first[frame_of]
    is_sig = local >= n_mich[frame_of]
    # 4 vertices: one per Michel decay, one per signal decay
    n_vert_m = int(n_mich.sum())
    n_sigf = int(sig.sum())
    vert = sample_target(rng, n_vert_m + n_sigf)
    pos = np.empty((P, 3))
    pos[~is_sig] = vert[:n_vert_m]
    sig_frames = np.nonzero(sig)[0]
    pos[is_sig] = np.repeat(vert[n_vert_m:], 3, axis=0)
    # 5-6 Michel momenta and directions
    pm = sample_michel(rng, n_vert_m)
    dirs = isotropic(rng, n_vert_m)
    mom = np.empty((P, 3))
    mom[~is_sig] = dirs * pm[:, None]
    charge = np.ones(P)
    # 7 signal kinematics
    if n_sigf:
        sm = sample_signal(rng, n_sigf)
        mom[is_sig] = sm.reshape(-1, 3)
        charge[is_sig] = np.tile([1.0, -1.0, 1.0], n_sigf)
    # 8 propagation with scattering
    pid, lay, hx, hy, hz = propagate(rng, pos, mom, charge)
    hit_frame = frame_of[pid]
    # 12 frame-straddling particles (own stream, so the main draw order is
    # unchanged): a particle crossing the boundary between layers s - 1 and
    # s leaves its hits on layers >= s in the next frame
    straddle = np.full(P, -1, np.int64)
    if cfg.straddle_frac > 0:
        rs = _rng(cfg.cfg_id, 2000 + salt)
        cross = rs.uniform(0.0, 1.0, P) < cfg.straddle_frac
        first = rs.integers(1, 4, P)
        straddle = np.where(cross & (frame_of < F - 1), first, -1)
        hit_frame = hit_frame + ((straddle[pid] >= 0) & (lay >= straddle[pid]))
    # 9 noise
    nn = cfg.noise_per_layer
    nlay = np.tile(np.repeat(np.arange(4), nn), F)
    nframe = np.repeat(np.arange(F), 4 * nn)
    nphi = rng.uniform(-np.pi, np.pi, len(nlay))
    nzt = rng.uniform(-1.0, 1.0, len(nlay)) * Z_HALF[nlay]
    Rn = R_LAYER[nlay]
    nx_, ny_, nz_ = quantise(nphi, nzt, Rn)
    # a pixel centre just outside the acceptance moves one pixel inward
    nz_ = np.where(np.abs(nz_) > Z_HALF[nlay], nz_ - np.sign(nz_) * PIXEL, nz_)
    # assemble and sort by (frame, layer, shuffle key)
    all_frame = np.concatenate([hit_frame, nframe])
    all_layer = np.concatenate([lay, nlay]).astype(np.int64)
    all_x = np.concatenate([hx, nx_])
    all_y = np.concatenate([hy, ny_])
    all_z = np.concatenate([hz, nz_])
    all_pid = np.concatenate([pid, np.full(len(nlay), -1)])
    key = rng.uniform(0.0, 1.0, len(all_x))          # 10 shuffle keys
    order = np.lexsort((key, all_layer, all_frame))
    all_frame, all_layer = all_frame[order], all_layer[order]
    all_x, all_y, all_z, all_pid = all_x[order], all_y[order], all_z[order], all_pid[order]
    sensor = sensor_of(all_layer, all_x, all_y, all_z)
    # 11 misalignment: the reported hit is A_s^-1(true hit) with
    # A_s(h) = R_z(alpha_s) h + t_s
    align = None
    if cfg.misalign:
        ra = _rng(cfg.cfg_id, 1000 + salt)
        align = np.concatenate([ra.normal(0.0, cfg.misalign_t, (N_SENSORS, 3)),
                                ra.normal(0.0, cfg.misalign_alpha, (N_SENSORS, 1))], 1)
        t = align[sensor, :3]
        a = align[sensor, 3]
        dx, dy, dz = all_x - t[:, 0], all_y - t[:, 1], all_z - t[:, 2]
        ca, sa = np.cos(-a), np.sin(-a)
        all_x, all_y, all_z = ca * dx - sa * dy, sa * dx + ca * dy, dz
    seg = all_frame * 4 + all_layer
    lo = np.searchsorted(seg, np.arange(4 * F + 1)).astype(np.int32)
    parts = dict(frame=frame_of, charge=charge.astype(np.int8), p0=mom,
                 vertex=pos, signal=is_sig, lam=lam, straddle=straddle)
    return FrameSet(all_x.astype(np.float32), all_y.astype(np.float32),
                    all_z.astype(np.float32), all_layer.astype(np.uint16),
                    sensor.astype(np.uint16), lo, all_pid.astype(np.int32),
                    parts, sig, align)


def true_triplets(fs: FrameSet, first_layer: int = 0):
    """Global hit indices (h_l, h_l+1, h_l+2) of particles that left one hit
    on each of three consecutive layers, with the particle index."""
    pid = fs.pid
    ok = pid >= 0
    P = int(pid[ok].max()) + 1 if ok.any() else 0
    table = np.full((P, 4), -1, np.int64)
    idx = np.nonzero(ok)[0]
    table[pid[idx], fs.layer[idx].astype(np.int64)] = idx
    L = first_layer
    good = np.all(table[:, L:L + 3] >= 0, axis=1)
    return table[good][:, L:L + 3], np.nonzero(good)[0], table
