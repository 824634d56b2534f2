"""The differentiable form: per-sensor alignment gradient of the summed
triplet-fit chi2 (hand-written adjoint behind a torch.autograd.Function)
against the oracle's exact forward-mode gradient and FP64 central finite
differences (step 1 um for translations, 1 um / R for rotations); relative
error <= 1e-3."""
import numpy as np
import pytest

from oracle import oracle
from paper_2206_11535_amd import synth
from paper_2206_11535_amd.params import default_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_11535_amd import lib
    lib.load()
    fs = synth.generate(5, n_frames=4000)
    p = default_params()
    r = oracle.run(fs, p)
    tr = r.tracks[(r.tracks[:, 6] == 1) & (r.tracks[:, 7] == 0)]
    trip = np.concatenate([tr[:, [1, 2, 3]], tr[:, [2, 3, 4]]]).astype(np.int32)
    print(f"case: alignment, {len(trip)} triplets", flush=True)
    dh = lib.to_device(fs)
    return lib, fs, p, trip, dh


def test_forward_matches_oracle(setup):
    import torch
    lib, fs, p, trip, dh = setup
    S = synth.N_SENSORS
    rng = np.random.default_rng(1)
    theta = np.concatenate([rng.normal(0, 0.02, (S, 3)), rng.normal(0, 2e-4, (S, 1))], 1)
    th32 = theta.astype(np.float32)
    chi2 = lib.align_chi2(dh, torch.from_numpy(trip).cuda(), torch.from_numpy(th32).cuda(), p).cpu().numpy()
    L, _ = oracle.align_loss_grad(fs, trip, th32.astype(np.float64), p, grad=False)
    assert np.all(np.isfinite(chi2))
    assert abs(chi2.astype(np.float64).sum() - L) <= 1e-4 * L
    # element by element: the oracle's chi2 of each triplet on its own (the
    # one-triplet loss), within 1e-4 relative with an absolute floor of 1
    rng = np.random.default_rng(3)
    pick = rng.choice(len(trip), 3000, replace=False)
    ref = np.array([oracle.align_loss_grad(fs, trip[i:i + 1], th32.astype(np.float64), p, grad=False)[0]
                    for i in pick])
    dev = np.abs(chi2[pick].astype(np.float64) - ref) / np.maximum(np.abs(ref), 1.0)
    print("alignment forward, element-wise relative deviation (floor 1): max", dev.max(), flush=True)
    assert dev.max() <= 1e-4


@pytest.mark.parametrize("at", ["zero", "random"])
def test_gradient_vs_oracle_and_fd(setup, at):
    import torch
    lib, fs, p, trip, dh = setup
    S = synth.N_SENSORS
    rng = np.random.default_rng(2)
    theta = np.zeros((S, 4)) if at == "zero" else \
        np.concatenate([rng.normal(0, 0.02, (S, 3)), rng.normal(0, 2e-4, (S, 1))], 1)
    th32 = theta.astype(np.float32)
    th = torch.from_numpy(th32).cuda().requires_grad_(True)
    tt = torch.from_numpy(trip).cuda()
    chi2 = lib.align_chi2_autograd(th, dh, tt, p)
    chi2.sum().backward()
    g = th.grad.cpu().numpy().astype(np.float64)
    _, gref = oracle.align_loss_grad(fs, trip, th32.astype(np.float64), p)
    err = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    print("norm-wise relative error vs oracle", err, flush=True)
    assert err <= 1e-3
    floor = 1e-3 * np.abs(gref).max()
    assert np.all(np.abs(g - gref) <= 1e-3 * np.maximum(np.abs(gref), floor))
    # FP64 central differences on a sample of parameters (triplets touching the sensor only)
    sens = fs.sensor.astype(np.int64)
    used = np.unique(sens[trip.ravel()])
    for s in rng.choice(used, 16, replace=False):
        m = np.any(sens[trip] == s, axis=1)
        sub = trip[m]
        layer = np.searchsorted(synth.SENSOR_BASE, s, "right") - 1
        for j in range(4):
            step = 1e-3 if j < 3 else 1e-3 / synth.R_LAYER[layer]
            tp, tm = th32.astype(np.float64), th32.astype(np.float64)
            tp[s, j] += step
            tm[s, j] -= step
            Lp, _ = oracle.align_loss_grad(fs, sub, tp, p, grad=False)
            Lm, _ = oracle.align_loss_grad(fs, sub, tm, p, grad=False)
            fd = (Lp - Lm) / (2 * step)
            assert abs(g[s, j] - fd) <= 1e-3 * max(abs(fd), floor), (s, j, g[s, j], fd)


def test_weighted_backward(setup):
    """Per-triplet upstream gradients flow through: the gradient of
    sum_t w_t chi2_t with random w against the oracle's weighted gradient."""
    import torch
    lib, fs, p, trip, dh = setup
    S = synth.N_SENSORS
    rng = np.random.default_rng(3)
    w = rng.uniform(0.0, 2.0, len(trip)).astype(np.float32)
    th = torch.zeros((S, 4), dtype=torch.float32, device="cuda")
    g = lib.align_backward(dh, torch.from_numpy(trip).cuda(), th, p, torch.from_numpy(w).cuda()).cpu().numpy()
    _, gref = oracle.align_loss_grad(fs, trip, np.zeros((S, 4)), p, weight=w.astype(np.float64))
    assert np.linalg.norm(g - gref) <= 1e-3 * np.linalg.norm(gref)


def test_strided_inputs(setup):
    """Tensors that are not row-major (a Fortran-ordered triplet array, a
    transposed theta) give the same results: the binding hands the C ABI
    contiguous copies."""
    import torch
    lib, fs, p, trip, dh = setup
    S = synth.N_SENSORS
    rng = np.random.default_rng(4)
    th32 = np.concatenate([rng.normal(0, 0.02, (S, 3)), rng.normal(0, 2e-4, (S, 1))], 1).astype(np.float32)
    tc = torch.from_numpy(np.ascontiguousarray(trip)).cuda()
    tf = torch.from_numpy(np.asfortranarray(trip)).cuda()
    assert not tf.is_contiguous()
    thc = torch.from_numpy(th32).cuda()
    tht = torch.from_numpy(np.ascontiguousarray(th32.T)).cuda().t()
    assert not tht.is_contiguous()
    a = lib.align_chi2(dh, tc, thc, p).cpu().numpy()
    b = lib.align_chi2(dh, tf, tht, p).cpu().numpy()
    assert np.array_equal(a, b)
    w = torch.ones(len(trip), dtype=torch.float32, device="cuda")
    ga = lib.align_backward(dh, tc, thc, p, w).cpu().numpy()
    gb = lib.align_backward(dh, tf, tht, p, w).cpu().numpy()
    # float64 accumulation in arbitrary atomic order: equal up to its rounding
    assert np.allclose(ga, gb, rtol=1e-6, atol=1e-6 * np.abs(ga).max())


def test_empty_and_single_triplet(setup):
    """No triplets: an empty chi2, a zero gradient (also through autograd).
    One triplet: chi2 and gradient against the oracle (one block of the
    backward pass has work, every other block contributes zero rows)."""
    import torch
    lib, fs, p, trip, dh = setup
    S = synth.N_SENSORS
    rng = np.random.default_rng(5)
    th32 = np.concatenate([rng.normal(0, 0.02, (S, 3)), rng.normal(0, 2e-4, (S, 1))], 1).astype(np.float32)
    thc = torch.from_numpy(th32).cuda()
    none = torch.zeros((0, 3), dtype=torch.int32, device="cuda")
    assert lib.align_chi2(dh, none, thc, p).numel() == 0
    g0 = lib.align_backward(dh, none, thc, p, torch.zeros(0, dtype=torch.float32, device="cuda"))
    assert torch.count_nonzero(g0).item() == 0
    th = thc.clone().requires_grad_(True)
    lib.align_chi2_autograd(th, dh, none, p).sum().backward()
    assert th.grad is not None and torch.count_nonzero(th.grad).item() == 0
    one = trip[len(trip) // 2:len(trip) // 2 + 1]
    c1 = lib.align_chi2(dh, torch.from_numpy(one).cuda(), thc, p).cpu().numpy()
    L1, gref = oracle.align_loss_grad(fs, one, th32.astype(np.float64), p)
    assert c1.shape == (1,) and abs(float(c1[0]) - L1) <= 1e-4 * max(L1, 1.0)
    g1 = lib.align_backward(dh, torch.from_numpy(one).cuda(), thc, p,
                            torch.ones(1, dtype=torch.float32, device="cuda")).cpu().numpy()
    touched = np.unique(fs.sensor[one.ravel()].astype(np.int64))
    assert np.count_nonzero(np.abs(g1).sum(1)) <= 3
    assert set(np.flatnonzero(np.abs(g1).sum(1))) <= set(touched.tolist())
    assert np.linalg.norm(g1 - gref) <= 1e-3 * np.linalg.norm(gref)


def test_invalid_indices_and_sensors(setup):
    """A triplet with a hit index outside [0, n_hits), or a hit on a sensor
    beyond theta's rows, gives NaN chi2 and adds nothing to the gradient
    (bounds checks in the kernels: nothing outside the buffers is read)."""
    import torch
    lib, fs, p, trip, dh = setup
    S = synth.N_SENSORS
    rng = np.random.default_rng(6)
    th32 = np.concatenate([rng.normal(0, 0.02, (S, 3)), rng.normal(0, 2e-4, (S, 1))], 1).astype(np.float32)
    sub = trip[rng.choice(len(trip), 2000, replace=False)]
    bad = np.array([[-1, sub[0, 1], sub[0, 2]], [sub[1, 0], sub[1, 1], fs.n_hits]], np.int32)
    mixed = np.concatenate([sub, bad])
    cm = lib.align_chi2(dh, torch.from_numpy(mixed).cuda(), torch.from_numpy(th32).cuda(), p).cpu().numpy()
    cs = lib.align_chi2(dh, torch.from_numpy(sub).cuda(), torch.from_numpy(th32).cuda(), p).cpu().numpy()
    assert np.all(np.isnan(cm[-2:])) and np.array_equal(cm[:-2], cs)
    ones = lambda n: torch.ones(n, dtype=torch.float32, device="cuda")
    gm = lib.align_backward(dh, torch.from_numpy(mixed).cuda(), torch.from_numpy(th32).cuda(), p, ones(len(mixed)))
    gs = lib.align_backward(dh, torch.from_numpy(sub).cuda(), torch.from_numpy(th32).cuda(), p, ones(len(sub)))
    assert torch.allclose(gm, gs, rtol=1e-6, atol=1e-9 * float(gs.abs().max()))
    # theta with fewer rows than the largest sensor id of the hits
    smax = fs.sensor[sub].astype(np.int64).max(axis=1)
    cut = int(np.median(smax))
    inside = smax < cut
    assert 100 < inside.sum() < len(sub) - 100
    ts = torch.from_numpy(np.ascontiguousarray(th32[:cut])).cuda()
    cc = lib.align_chi2(dh, torch.from_numpy(sub).cuda(), ts, p).cpu().numpy()
    assert np.all(np.isnan(cc[~inside])) and np.array_equal(cc[inside], cs[inside])
    gc = lib.align_backward(dh, torch.from_numpy(sub).cuda(), ts, p, ones(len(sub)))
    gi = lib.align_backward(dh, torch.from_numpy(np.ascontiguousarray(sub[inside])).cuda(),
                            torch.from_numpy(th32).cuda(), p, ones(int(inside.sum())))
    assert gc.shape == (cut, 4)
    assert torch.allclose(gc, gi[:cut], rtol=1e-6, atol=1e-9 * float(gi.abs().max()))
    assert torch.count_nonzero(gi[cut:]).item() == 0


def test_gradient_deterministic_and_reused_workspace(setup):
    """The backward pass sums in a fixed order (per-block rows, then group
    sums, then the sum of the group sums): repeated calls, also on one
    workspace reused across calls and with another triplet set in between,
    give bitwise the same gradient."""
    import torch
    lib, fs, p, trip, dh = setup
    S = synth.N_SENSORS
    tt = torch.from_numpy(trip).cuda()
    th = torch.zeros((S, 4), dtype=torch.float32, device="cuda")
    g = torch.ones(len(trip), dtype=torch.float32, device="cuda")
    a = lib.align_backward(dh, tt, th, p, g).cpu().numpy()
    b = lib.align_backward(dh, tt, th, p, g).cpu().numpy()
    lib.align_backward(dh, tt[: len(trip) // 3], th, p, g[: len(trip) // 3])
    c = lib.align_backward(dh, tt, th, p, g).cpu().numpy()
    assert np.array_equal(a, b) and np.array_equal(a, c)
    assert np.count_nonzero(a) > 1000


def test_padded_sensor_table(setup):
    """Padding theta with unused sensors (2000 in all) leaves the chi2 and
    the gradient of the sensors in use unchanged and gives the unused ones a
    zero gradient (the sensors' cos, sin tables and the accumulators are
    indexed by sensor)."""
    import torch
    lib, fs, p, trip, dh = setup
    S = synth.N_SENSORS
    rng = np.random.default_rng(5)
    theta = np.concatenate([rng.normal(0, 0.02, (S, 3)), rng.normal(0, 2e-4, (S, 1))], 1).astype(np.float32)
    big = np.zeros((2000, 4), np.float32)
    big[:S] = theta
    tt = torch.from_numpy(trip).cuda()
    g = torch.ones(len(trip), dtype=torch.float32, device="cuda")
    ts, tb = torch.from_numpy(theta).cuda(), torch.from_numpy(big).cuda()
    a = lib.align_backward(dh, tt, ts, p, g).cpu().numpy()
    b = lib.align_backward(dh, tt, tb, p, g).cpu().numpy()
    assert np.count_nonzero(a) > 1000
    assert not np.any(b[S:])
    np.testing.assert_allclose(b[:S], a, rtol=1e-6, atol=1e-9 * np.abs(a).max())
    ca = lib.align_chi2(dh, tt, ts, p).cpu().numpy()
    cb = lib.align_chi2(dh, tt, tb, p).cpu().numpy()
    assert np.array_equal(ca, cb)
