"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars: relative L2 <= 1e-5 for signals, <= 1e-4 per gradient group.  Inputs are
seeded synthetic scenes; the 'measured' data is the oracle forward of a
perturbed scene.  Full-size workloads are compared on a sampled subset of
sensors (the oracle runs the same subset); smaller ones element by element.
"""

import sys

import numpy as np
import pytest

import oracle
from helpers import rel_l2, tiny_scene, with_
from paper_2412_03898_amd import synth

pytestmark = pytest.mark.gpu

SIG_TOL = 1e-5
GRAD_TOL = 1e-4


def _say(msg):
    print(f"[gpu-parity] {msg}", flush=True)
    sys.stdout.flush()


def gpu_forward(wl):
    from paper_2412_03898_amd import ops
    pb, balls, deform, ft, sens = ops.to_device(wl)
    y = ops.forward(pb, balls, deform, ft, sens)
    flags = ops.check()
    return y.cpu().numpy().astype(np.float64), flags


def gpu_adjoint(wl, residual):
    import torch
    from paper_2412_03898_amd import ops
    pb, balls, deform, ft, sens = ops.to_device(wl)
    res = torch.from_numpy(np.ascontiguousarray(residual.astype(np.float32))).cuda()
    gb, gd = ops.adjoint(pb, balls, deform, ft, sens, res)
    ops.check()
    return gb.cpu().numpy().astype(np.float64), (None if gd is None else gd.cpu().numpy().astype(np.float64))


def gpu_loss(wl, y, d):
    import torch
    from paper_2412_03898_amd import ops
    pb = ops.Problem.from_workload(wl)
    yt = torch.from_numpy(np.ascontiguousarray(y.astype(np.float32))).cuda()
    dt = torch.from_numpy(np.ascontiguousarray(d.astype(np.float32))).cuda()
    L, r = ops.loss(pb, yt, dt)
    return float(L.item()), r.cpu().numpy().astype(np.float64)


def grad_groups(wl, gb, gd):
    """Named parameter groups (units differ between groups)."""
    out = {"pos": gb[0:3], "R": gb[3], "P": gb[4]}
    if gd is not None:
        if wl.basis == 2:
            for kind, name in ((0, "w"), (1, "theta"), (2, "sigma")):
                out[f"def_pos_{name}"] = gd[0:3, kind::3]
                out[f"def_R_{name}"] = gd[3, kind::3]
                out[f"def_P_{name}"] = gd[4, kind::3]
        else:
            out["def_pos"] = gd[0:3]
            out["def_R"] = gd[3]
            out["def_P"] = gd[4]
    return out


def assert_grads(wl, got, ref, tol=GRAD_TOL):
    g = grad_groups(wl, *got)
    r = grad_groups(wl, *ref)
    errs = {k: rel_l2(g[k], r[k]) for k in r}
    _say(f"grad rel-L2 {errs}")
    for k, e in errs.items():
        assert e <= tol, (k, e)


def measured_for(wl, seed=1):
    return oracle.forward(wl, balls=synth.perturbed(wl.balls, seed)).astype(np.float32)


# ---------------------------------------------------------------- plain single frame
@pytest.fixture(scope="module")
def plain():
    return synth.workload_plain()


@pytest.mark.parametrize("order", ["unsorted", "morton"])
def test_forward_plain(plain, order):
    wl = plain if order == "unsorted" else synth.apply_order(plain)
    _say(f"forward plain {order} B={wl.n_balls} S={wl.n_sensors} T={wl.n_samples}")
    y, flags = gpu_forward(wl)
    ref = oracle.forward(wl)
    err = rel_l2(y, ref)
    _say(f"forward rel-L2 {err:.3e} flags={flags}")
    assert flags == 0
    assert err <= SIG_TOL


def test_loss_and_adjoint_plain(plain):
    wl = synth.apply_order(plain)
    d = measured_for(wl)
    y_ref = oracle.forward(wl)
    L_ref, r_ref = oracle.loss(y_ref, d)
    # loss on identical FP32 inputs
    y32 = y_ref.astype(np.float32)
    L_gpu, r_gpu = gpu_loss(wl, y32, d)
    L_same, _ = oracle.loss(y32, d)
    assert L_gpu == pytest.approx(L_same, rel=1e-6)
    # the residual is one FP32 subtraction per element: bit-exact against numpy's
    np.testing.assert_array_equal(r_gpu.astype(np.float32), y32 - d)
    # adjoint only: the same FP32 residual into both
    res32 = r_ref.astype(np.float32)
    _say("adjoint plain (same residual)")
    assert_grads(wl, gpu_adjoint(wl, res32), oracle.adjoint(wl, res32.astype(np.float64)))
    # end to end: each side its own forward and residual
    y_gpu, _ = gpu_forward(wl)
    L_e2e, r_e2e = gpu_loss(wl, y_gpu, d)
    assert L_e2e == pytest.approx(L_ref, rel=2e-5)
    _say("adjoint plain (end to end)")
    assert_grads(wl, gpu_adjoint(wl, r_e2e), oracle.adjoint(wl, r_ref))


# ---------------------------------------------------------------- 4D and variants
def test_4d_fourier_small():
    wl = synth.apply_order(synth.workload_vessel_4d(n_balls=4000, n_sensors=130, n_frames=16))
    _say(f"4d fourier B={wl.n_balls} S={wl.n_sensors} F={wl.n_frames} T={wl.n_samples}")
    y, flags = gpu_forward(wl)
    ref = oracle.forward(wl)
    err = rel_l2(y, ref)
    _say(f"forward rel-L2 {err:.3e}")
    assert err <= SIG_TOL
    rng = np.random.default_rng(3)
    res = (ref - ref * (1.0 + 0.05 * rng.normal(size=ref.shape))).astype(np.float32)
    assert_grads(wl, gpu_adjoint(wl, res), oracle.adjoint(wl, res.astype(np.float64)))


VARIANTS = [
    dict(basis=1, pos_mode=1),
    dict(basis=2, pos_mode=0),
    dict(basis=2, pos_mode=1),
    dict(kernel=1, basis=0),
    dict(kernel=1, basis=1),
    dict(kernel=1, basis=2, pos_mode=1),
    # the two-phase chain rule: Fourier series beyond 2 harmonics, and Eq. 2 with 13 and
    # 65 bases per attribute (the two readings of the 65 Gaussian basis functions)
    dict(basis=1, K=3),
    dict(kernel=1, basis=1, K=5, pos_mode=1),
    dict(basis=2, pos_mode=1, N=13),
    dict(basis=2, pos_mode=1, N=65),
    dict(kernel=1, basis=2, pos_mode=1, N=13),
    dict(kernel=1, basis=2, pos_mode=0, N=65),
]


@pytest.mark.parametrize("var", VARIANTS, ids=lambda c: "-".join(f"{k}{v}" for k, v in c.items()))
def test_variants(var):
    wl = tiny_scene(n_balls=700, n_sensors=69, n_frames=3, seed=61, **var)
    wl = with_(wl, balls=wl.balls.copy())
    order = synth.morton_order(wl.balls)
    wl.balls = np.ascontiguousarray(wl.balls[:, order])
    if wl.deform is not None:
        wl.deform = np.ascontiguousarray(wl.deform[:, :, order])
    _say(f"variant {var}")
    y, flags = gpu_forward(wl)
    ref = oracle.forward(wl)
    err = rel_l2(y, ref)
    _say(f"forward rel-L2 {err:.3e}")
    assert err <= SIG_TOL
    rng = np.random.default_rng(4)
    res = rng.normal(size=ref.shape).astype(np.float32) * np.float32(np.abs(ref).max())
    assert_grads(wl, gpu_adjoint(wl, res), oracle.adjoint(wl, res.astype(np.float64)))


# ---------------------------------------------------------------- batching and edge cases
def test_uneven_batch_with_empty_scene():
    a = tiny_scene(n_balls=300, n_sensors=70, n_frames=2, basis=1, seed=71)
    b = tiny_scene(n_balls=1000, n_sensors=70, n_frames=1, basis=1, seed=72)
    wl = with_(a, balls=np.concatenate([a.balls, b.balls], axis=1),
               deform=np.concatenate([a.deform, b.deform], axis=2),
               frame_t=np.concatenate([a.frame_t, np.array([0.3, 0.7, 0.9], np.float32), b.frame_t]),
               ball_offset=np.array([0, 300, 300, 1300]), frame_offset=np.array([0, 2, 5, 6]))
    _say("uneven batch 3 scenes (one empty)")
    y, _ = gpu_forward(wl)
    ref = oracle.forward(wl)
    assert np.abs(y[2:5]).max() == 0.0
    assert rel_l2(y, ref) <= SIG_TOL
    rng = np.random.default_rng(5)
    res = rng.normal(size=ref.shape).astype(np.float32)
    assert_grads(wl, gpu_adjoint(wl, res), oracle.adjoint(wl, res.astype(np.float64)))


def test_uneven_batch_two_phase_chain_rule():
    """The two-phase chain rule's per-scene layout: four scenes with the Eq. 2 deformation
    (4 bases per attribute, multiplicative positions) -- 300 balls x 2 frames, an empty
    scene with 3 frames, 500 balls with no frame, 700 balls x 1 frame -- against the oracle."""
    parts = [tiny_scene(n_balls=n, n_sensors=70, n_frames=1, basis=2, N=4, pos_mode=1, seed=s)
             for n, s in ((300, 91), (500, 92), (700, 93))]
    a, c, d = parts
    wl = with_(a, balls=np.concatenate([a.balls, c.balls, d.balls], axis=1),
               deform=np.concatenate([a.deform, c.deform, d.deform], axis=2),
               frame_t=np.array([0.1, 0.6, 0.2, 0.5, 0.8, 0.35], np.float32),
               ball_offset=np.array([0, 300, 300, 800, 1500]), frame_offset=np.array([0, 2, 5, 5, 6]))
    _say("uneven batch, Eq. 2 (two-phase chain rule): 4 scenes, one empty, one without frames")
    y, _ = gpu_forward(wl)
    ref = oracle.forward(wl)
    assert np.abs(y[2:5]).max() == 0.0
    assert rel_l2(y, ref) <= SIG_TOL
    rng = np.random.default_rng(94)
    res = rng.normal(size=ref.shape).astype(np.float32) * np.float32(np.abs(ref).max())
    got = gpu_adjoint(wl, res)
    # the scene without frames has no gradient
    assert np.abs(got[0][:, 300:800]).max() == 0.0 and np.abs(got[1][:, :, 300:800]).max() == 0.0
    assert_grads(wl, got, oracle.adjoint(wl, res.astype(np.float64)))


def test_single_ball_single_sensor():
    wl = tiny_scene(n_balls=1, n_sensors=1, seed=81)
    y, _ = gpu_forward(wl)
    ref = oracle.forward(wl)
    assert rel_l2(y, ref) <= SIG_TOL
    assert abs(y.sum()) < 1e-6 * np.abs(y).max()


def test_adjoint_windows_outside_the_staged_row_and_at_the_record_end():
    """Unordered balls (each chunk spans the whole cube, so almost every window lies outside
    the staged residual row and takes the global-memory path) and a record cut 40 samples
    before the latest window ends: windows near, across and past the last sample."""
    wl = tiny_scene(n_balls=700, n_sensors=70, seed=87)
    b = wl.balls.astype(np.float64)
    S = wl.sensors.astype(np.float64)
    delta = wl.c / wl.fs
    r = np.sqrt(((b[0:3, :, None] - S[:, None, :]) ** 2).sum(0))
    rho = b[3] / delta
    kl = np.floor(r / delta - wl.t0 * wl.fs - rho[:, None] + 0.5).astype(int)
    end = kl + (np.floor(2 * rho).astype(int) + 2)[:, None]
    T = int(end.max()) - 40
    assert (end > T).sum() > 5 and (kl >= T).sum() > 0
    wl = with_(wl, n_samples=T)
    rng = np.random.default_rng(9)
    res = rng.normal(size=(1, S.shape[1], T)).astype(np.float32)
    _say(f"adjoint unordered, record cut at T={T}")
    assert_grads(wl, gpu_adjoint(wl, res), oracle.adjoint(wl, res.astype(np.float64)))


def test_gaussian_adjoint_windows_outside_the_row_and_at_the_record_end():
    """Gaussian balls in an order unrelated to their positions: a wave's 64 balls span the
    whole cube, so most windows miss the wave's staged residual row and take the
    global-memory path (eight loads at a time); the record ends 40 samples before the
    latest window does."""
    wl = tiny_scene(n_balls=700, n_sensors=70, seed=88, kernel=1)
    b = wl.balls.astype(np.float64)
    S = wl.sensors.astype(np.float64)
    delta = wl.c / wl.fs
    r = np.sqrt(((b[0:3, :, None] - S[:, None, :]) ** 2).sum(0))
    h = 6.0 * b[3] / delta                       # the kernels' window half-width (6 std)
    kl = np.floor(r / delta - wl.t0 * wl.fs - h[:, None] + 0.5).astype(int)
    end = kl + (np.floor(2 * h).astype(int) + 2)[:, None]
    T = int(end.max()) - 40
    assert (end > T).sum() > 5 and (kl >= T).sum() > 0
    wl = with_(wl, n_samples=T)
    rng = np.random.default_rng(10)
    res = rng.normal(size=(1, S.shape[1], T)).astype(np.float32)
    _say(f"gaussian adjoint unordered, record cut at T={T}")
    assert_grads(wl, gpu_adjoint(wl, res), oracle.adjoint(wl, res.astype(np.float64)))


def _morton(wl):
    order = synth.morton_order(wl.balls)
    return with_(wl, balls=np.ascontiguousarray(wl.balls[:, order]))


def test_window_lengths_two_to_forty():
    """Uniform spheres from R = 0.005 mm to 0.75 mm: window lengths W = 2 .. 42 samples
    (the short windows take the four-sample second-difference form), amplitudes over
    three decades in one chunk."""
    wl = tiny_scene(n_balls=600, n_sensors=70, seed=85)
    b = wl.balls.copy()
    rng = np.random.default_rng(85)
    delta = wl.c / wl.fs
    W = rng.integers(2, 43, size=b.shape[1])
    b[3] = ((W - 2 + rng.uniform(0.05, 0.95, size=W.size)) * delta / 2).astype(np.float32)
    b[4] = (10.0 ** rng.uniform(-3, 0, size=W.size)).astype(np.float32)
    k0 = synth.record_start(0.060, 0.010, 0.8e-3, 0.5e-3)
    n = synth.record_length_needed(0.060, 0.010, 0.8e-3, 0.5e-3, k0)
    wl = _morton(with_(wl, balls=b, t0=k0 / wl.fs, n_samples=n))
    Wk = np.floor(2 * wl.balls[3].astype(np.float64) / delta).astype(int) + 2
    assert {2, 3, 4, 5, 6}.issubset(set(Wk.tolist()))
    y, flags = gpu_forward(wl)
    ref = oracle.forward(wl)
    err = rel_l2(y, ref)
    _say(f"window lengths 2..42 rel-L2 {err:.3e}")
    assert flags == 0
    assert err <= SIG_TOL


@pytest.mark.parametrize("kernel", [0, 1])
def test_sensors_among_the_balls(kernel):
    """Sensors inside the cloud's box, all among the first 64: the wave holding them keeps
    the FP32 tile, the other waves take the integer one.  Uniform spheres: every inner
    sensor lies 0.5 mm outside every ball; Gaussian balls: farther than 10 std from every
    centre, where the trace term the kernel leaves out is below 1e-21 of the peak."""
    wl = tiny_scene(n_balls=900, n_sensors=200, seed=86, kernel=kernel)
    sens = wl.sensors.copy()
    rng = np.random.default_rng(86)
    inner = rng.choice(64, size=40, replace=False)     # all in the first 64-sensor wave
    b = wl.balls.astype(np.float64)
    margin = b[3] + 0.5e-3 if kernel == 0 else 10.0 * b[3]
    for s in inner:
        while True:
            p = rng.uniform(-0.012, 0.012, size=3)
            if np.min(np.linalg.norm(b[0:3] - p[:, None], axis=0) - margin) > 0.0:
                break
        sens[:, s] = p.astype(np.float32)
    k0 = 0
    reach = 0.4e-3 if kernel == 0 else 2.0e-3            # largest radius, or 6 std x 2 (+10%)
    n = synth.record_length_needed(0.060, 0.010, reach, 0.5e-3, k0)
    wl = _morton(with_(wl, sensors=sens, t0=0.0, n_samples=n))
    y, flags = gpu_forward(wl)
    ref = oracle.forward(wl)
    err = rel_l2(y, ref)
    err_in = rel_l2(y[:, inner], ref[:, inner])
    _say(f"sensors among the balls rel-L2 {err:.3e} (inner sensors {err_in:.3e}) flags={flags}")
    assert flags == 0
    assert err <= SIG_TOL and err_in <= SIG_TOL


def test_clipped_record_is_dropped_and_flagged():
    wl = tiny_scene(n_balls=50, n_sensors=10, seed=82)
    wl = with_(wl, n_samples=200, t0=wl.t0 + 150 / wl.fs)   # record too short: most traces clipped
    y, flags = gpu_forward(wl)
    ref = oracle.forward(wl)
    assert flags & 4
    assert rel_l2(y, ref) <= SIG_TOL


def test_sensor_inside_ball_raises_flag():
    from paper_2412_03898_amd import binding
    wl = tiny_scene(n_balls=5, n_sensors=3, seed=83)
    sens = wl.sensors.copy()
    sens[:, 1] = wl.balls[0:3, 2]     # sensor 1 sits at the centre of ball 2
    wl = with_(wl, sensors=sens)
    with pytest.raises(binding.SlingbagError) as ei:
        gpu_forward(wl)
    assert ei.value.status == binding.SB_ERR_DEVICE_FLAG


def test_nonfinite_ball_is_skipped_and_flagged():
    from paper_2412_03898_amd import binding
    wl = tiny_scene(n_balls=20, n_sensors=8, seed=84)
    bad = wl.balls.copy()
    bad[3, 7] = np.nan
    with pytest.raises(binding.SlingbagError):
        gpu_forward(with_(wl, balls=bad))
    # the remaining balls still produced the right signal
    from paper_2412_03898_amd import ops
    import torch
    pb, balls, deform, ft, sens = ops.to_device(with_(wl, balls=bad))
    y = ops.forward(pb, balls, deform, ft, sens)
    torch.cuda.synchronize()
    try:
        ops.check()
    except binding.SlingbagError:
        pass
    keep = np.r_[0:7, 8:20]
    ref = oracle.forward(with_(wl, balls=wl.balls[:, keep], ball_offset=np.array([0, 19])))
    assert rel_l2(y.cpu().numpy(), ref) <= SIG_TOL


@pytest.mark.parametrize("kernel", [0, 1])
def test_nonfinite_size_is_skipped_by_the_adjoint(kernel):
    """A NaN and a +inf size inside one 256-ball chunk (the Gaussian-ball adjoint ranks the
    chunk's balls by size): both balls are skipped and flagged, their gradients stay zero,
    and every other ball's gradient matches the oracle without them."""
    import torch
    from paper_2412_03898_amd import binding, ops
    wl = tiny_scene(n_balls=300, n_sensors=70, seed=85, kernel=kernel)
    bad = wl.balls.copy()
    bad[3, 7] = np.nan
    bad[3, 130] = np.inf
    keep = np.r_[0:7, 8:130, 131:300]
    sub = with_(wl, balls=wl.balls[:, keep], ball_offset=np.array([0, len(keep)]))
    rng = np.random.default_rng(86)
    ref_y = oracle.forward(sub)
    res = (rng.normal(size=ref_y.shape) * np.abs(ref_y).max()).astype(np.float32)
    _say(f"nonfinite sizes in the adjoint, kernel={kernel}")
    pb, balls, deform, ft, sens = ops.to_device(with_(wl, balls=bad))
    gb, _ = ops.adjoint(pb, balls, deform, ft, sens, torch.from_numpy(res).cuda())
    torch.cuda.synchronize()
    with pytest.raises(binding.SlingbagError) as ei:
        ops.check()
    assert ei.value.status == binding.SB_ERR_DEVICE_FLAG
    g = gb.cpu().numpy().astype(np.float64)
    assert np.all(g[:, [7, 130]] == 0.0)
    ref_gb, _ = oracle.adjoint(sub, res.astype(np.float64))
    assert_grads(sub, (g[:, keep], None), (ref_gb, None))


def test_ball_longer_than_any_record_is_skipped_and_flagged():
    """A ball whose window would span more than a million samples (radius 100 m) is left
    out with the clipped flag; the other balls still match the oracle without it."""
    wl = tiny_scene(n_balls=300, n_sensors=70, seed=93)
    big = wl.balls.copy()
    big[3, 17] = 100.0
    y, flags = gpu_forward(with_(wl, balls=big))
    keep = np.r_[0:17, 18:300]
    ref = oracle.forward(with_(wl, balls=wl.balls[:, keep], ball_offset=np.array([0, 299])))
    err = rel_l2(y, ref)
    _say(f"ball longer than any record: rel-L2 {err:.3e} flags={flags}")
    assert flags & 4
    assert err <= SIG_TOL


# ---------------------------------------------------------------- full sizes, sampled outputs
# The GPU runs the whole problem (every ball, sensor and frame, default knobs);
# the oracle computes the sampled (frame, sensor) rows.  For the adjoint the
# GPU's residual is zero outside those rows, so its gradient equals the oracle
# adjoint of the sub-problem made of just those rows.
def _full_size_sampled(wl, s_step, f_step, seed):
    import torch
    from paper_2412_03898_amd import ops
    F = wl.n_frames
    s_idx = np.arange(0, wl.n_sensors, s_step)
    if len(wl.ball_offset) == 2:
        f_idx = np.arange(0, F, f_step)
        sub = with_(wl, sensors=wl.sensors[:, s_idx].copy(), frame_t=wl.frame_t[f_idx].copy(),
                    frame_offset=np.array([0, len(f_idx)]), n_frames=len(f_idx))
    else:                       # batch of scenes: every frame of every scene
        f_idx = np.arange(F)
        sub = with_(wl, sensors=wl.sensors[:, s_idx].copy())
    pb, balls, deform, ft, sens = ops.to_device(wl)
    fi = torch.from_numpy(f_idx).cuda()[:, None]
    si = torch.from_numpy(s_idx).cuda()[None, :]
    y = ops.forward(pb, balls, deform, ft, sens)
    assert ops.check() == 0
    got = y[fi, si].cpu().numpy().astype(np.float64)
    del y
    ref = oracle.forward(sub)
    err = rel_l2(got, ref)
    _say(f"forward sampled rel-L2 {err:.3e} ({len(f_idx)} frames x {len(s_idx)} sensors)")
    assert err <= SIG_TOL
    rng = np.random.default_rng(seed)
    rows = (rng.normal(size=ref.shape) * np.abs(ref).max()).astype(np.float32)
    res = torch.zeros((F, wl.n_sensors, wl.n_samples), dtype=torch.float32, device="cuda")
    res[fi, si] = torch.from_numpy(rows).cuda()
    gb, gd = ops.adjoint(pb, balls, deform, ft, sens, res)
    assert ops.check() == 0
    got_g = (gb.cpu().numpy().astype(np.float64), None if gd is None else gd.cpu().numpy().astype(np.float64))
    del res, gb, gd
    assert_grads(sub, got_g, oracle.adjoint(sub, rows.astype(np.float64)))


def test_vessel_static_full_size_sampled():
    wl = synth.apply_order(synth.workload_vessel_static())
    _say(f"vessel static full B={wl.n_balls} S={wl.n_sensors} T={wl.n_samples}")
    _full_size_sampled(wl, 16, 1, 6)


def test_heart_ellipsoid_full_size_sampled():
    """The heart phantom's Gaussian ellipsoid (10,667 Gaussian balls, Fourier pulsation, 17 frames,
    1,024 sensors, 2,560 samples) at full size, with the default Gaussian knobs (256-row forward
    column, 384-sample adjoint row); sampled every 64th sensor and 4th frame."""
    slabs, ell = synth.heart_phantom()
    wl = synth.apply_order(ell)
    _say(f"heart ellipsoid full B={wl.n_balls} F={wl.n_frames} S={wl.n_sensors} T={wl.n_samples}")
    _full_size_sampled(wl, 64, 4, 8)


def test_vessel_4d_full_size_sampled():
    wl = synth.apply_order(synth.workload_vessel_4d())
    _say(f"vessel 4d full B={wl.n_balls} S={wl.n_sensors} F={wl.n_frames} T={wl.n_samples}")
    _full_size_sampled(wl, 16, 1, 7)


def test_uneven_batch_full_size_sampled():
    wl = synth.apply_order(synth.workload_uneven_batch())
    _say(f"uneven batch full: scenes={len(wl.ball_offset) - 1} B={wl.n_balls} F={wl.n_frames} "
         f"S={wl.n_sensors} T={wl.n_samples}")
    _full_size_sampled(wl, 64, 1, 11)


def test_per_frame_path_matches_4d_oracle():
    """The frame-by-frame comparison path (each frame's attributes evaluated in FP64 and
    stored as FP32, then one static forward per frame) against the oracle's FP64 4D
    forward of the same scene: the 50,000-ball 16-frame scene with its Fourier
    deformation, every 16th sensor of every frame, within the signal bar (the FP32
    positions cost a few 1e-6)."""
    import torch
    from paper_2412_03898_amd import ir, ops
    wl = synth.apply_order(synth.workload_vessel_4d())
    s_idx = np.arange(0, wl.n_sensors, 16)
    sub = with_(wl, sensors=wl.sensors[:, s_idx].copy())
    ref = oracle.forward(sub)
    pf = ops.Problem(wl.kernel, 0, 0, 0, wl.n_sensors, wl.n_samples, wl.c, wl.fs, wl.t0,
                     np.array([0, wl.n_balls]), np.array([0, 1]))
    sens = torch.from_numpy(wl.sensors).cuda()
    t0 = torch.zeros(1, dtype=torch.float32, device="cuda")
    got = np.empty_like(ref)
    for f, x in enumerate(ir.materialise_frames(wl, wl.balls, wl.deform)):
        y = ops.forward(pf, torch.from_numpy(x).cuda(), None, t0, sens)
        got[f] = y[0, torch.from_numpy(s_idx).cuda()].cpu().numpy()
    assert ops.check() == 0
    err = rel_l2(got, ref)
    _say(f"per-frame path vs 4D oracle: rel-L2 {err:.3e}")
    assert err <= SIG_TOL


def test_large_ir_scene_full_size_sampled():
    wl = synth.apply_order(synth.workload_large_ir())
    _say(f"large 4D full B={wl.n_balls} F={wl.n_frames} S={wl.n_sensors} T={wl.n_samples}")
    _full_size_sampled(wl, 128, 8, 12)


# ---------------------------------------------------------------- ordering (performance only)
def test_order_matches_morton_definition():
    """The GPU order is the stable sort by the Morton code of the fixed grid, per scene
    (integer result: bit-exact against the definition written in numpy)."""
    import torch
    from paper_2412_03898_amd import ops
    a = synth.workload_vessel_static(n_balls=30_000, n_sensors=4, n_samples=4096, seed=12)
    b = synth.workload_plain(n_balls=7_000, n_sensors=4, seed=13)
    balls = np.concatenate([a.balls, b.balls], axis=1)
    wl = with_(a, balls=balls, ball_offset=np.array([0, 30_000, 37_000]),
               frame_offset=np.array([0, 1, 2]), frame_t=np.zeros(2, np.float32))
    pb = ops.Problem.from_workload(wl)
    bt = torch.from_numpy(balls).cuda()
    perm = ops.order(pb, bt).cpu().numpy()
    ref = np.concatenate([synth.morton_order(a.balls), synth.morton_order(b.balls) + 30_000])
    np.testing.assert_array_equal(perm, ref)
    nb = ops.permute(bt, torch.from_numpy(perm).cuda()).cpu().numpy()
    np.testing.assert_array_equal(nb, balls[:, perm])


@pytest.mark.parametrize("sizes", [[1], [5, 4096, 4097], [1_100_000], [300] * 32, [0, 300, 0, 5000, 0]],
                         ids=["one", "ragged", "nine-scan-groups", "32-scenes", "empty-scenes"])
def test_order_ties_clamps_and_sizes(sizes):
    """Stable order with many equal keys (balls sharing a grid cell, balls clamped to the
    grid's faces), ragged tile counts, a table of 269 tiles (the column scan in nine groups
    of at most 32), the largest scene index and empty scenes; bit-exact against the numpy
    definition."""
    import torch
    from paper_2412_03898_amd import ops
    rng = np.random.default_rng(sum(sizes) + len(sizes))
    B = int(sum(sizes))
    pos = rng.uniform(-0.01, 0.01, size=(3, B))
    pos[:, ::3] = 0.004                                        # one shared cell
    pos[:, 1::7] = rng.choice([-3.0, 2.5], size=(3, len(range(1, B, 7))))   # outside the grid
    pos[:, 2::5] = np.round(pos[:, 2::5], 4)                   # a few hundred shared cells
    balls = np.zeros((5, B), np.float32)
    balls[:3] = pos
    balls[3] = 2e-4
    balls[4] = 1.0
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    base = synth.workload_plain(n_balls=4, n_sensors=4)
    wl = with_(base, balls=balls, ball_offset=off, frame_offset=np.arange(len(sizes) + 1),
               frame_t=np.zeros(len(sizes), np.float32))
    _say(f"order B={B} scenes={len(sizes)}")
    pb = ops.Problem.from_workload(wl)
    perm = ops.order(pb, torch.from_numpy(balls).cuda()).cpu().numpy()
    ref = np.concatenate([synth.morton_order(balls[:, a:b]) + a for a, b in zip(off[:-1], off[1:])])
    np.testing.assert_array_equal(perm, ref)


def test_result_independent_of_order():
    """Forward and gradients of a 4D scene are the same (up to the permutation) in any ball order."""
    wl = synth.workload_vessel_4d(n_balls=3000, n_sensors=70, n_frames=3)
    y0, _ = gpu_forward(wl)
    ws = synth.apply_order(wl)
    y1, _ = gpu_forward(ws)
    # The uniform sphere's integer tile rounds every sample to 2^-30 of its chunk's
    # amplitude bound, and which balls share a chunk depends on the order: each run
    # lies about 1e-6 (relative L2) from the exact signal, so the two may differ by twice that.
    assert rel_l2(y1, y0) <= 3e-6
    rng = np.random.default_rng(8)
    res = rng.normal(size=y0.shape).astype(np.float32)
    g0 = gpu_adjoint(wl, res)
    g1 = gpu_adjoint(ws, res)
    perm = synth.morton_order(wl.balls)
    assert rel_l2(g1[0], g0[0][:, perm]) <= 1e-5
    assert rel_l2(g1[1], g0[1][:, :, perm]) <= 1e-5


def test_autotune_then_parity():
    """The autotuner picks a candidate setting and the tuned kernels still match the oracle."""
    import torch
    from paper_2412_03898_amd import binding, ops, tune
    wl = synth.apply_order(synth.workload_vessel_4d(n_balls=3000, n_sensors=70, n_frames=4))
    pb, balls, deform, ft, sens = ops.to_device(wl)
    saved = {k: binding.tune_get(k) for k in (1, 2, 3, 4)}
    try:
        choice = tune.autotune(pb, balls, deform, ft, sens, cache=None)
        assert choice[0] in (64, 128, 1, 2) and choice[1] in (2, 3, 4) and choice[2] in (2048, 4096, 8192, 16384)
        y = ops.forward(pb, balls, deform, ft, sens)
        ops.check()
        ref = oracle.forward(wl)
        assert rel_l2(y.cpu().numpy(), ref) <= SIG_TOL
        rng = np.random.default_rng(9)
        res = rng.normal(size=ref.shape).astype(np.float32)
        assert_grads(wl, gpu_adjoint(wl, res), oracle.adjoint(wl, res.astype(np.float64)))
    finally:
        for k, v in saved.items():
            binding.tune(k, v)


@pytest.mark.parametrize("col,occ", [(64, 2), (64, 4), (128, 3), (128, 4), (1, 4), (2, 3)])
def test_every_knob_setting_matches_oracle(col, occ):
    """Every kernel instance the tuner can pick gives oracle-parity results."""
    from paper_2412_03898_amd import binding
    wl = synth.apply_order(synth.workload_vessel_static(n_balls=6000, n_sensors=130, n_samples=4096))
    saved = {k: binding.tune_get(k) for k in (1, 2, 3, 4)}
    try:
        binding.tune(binding.SB_TUNE_FWD_COLUMN, col)
        binding.tune(binding.SB_TUNE_ADJ_OCCUPANCY, occ)
        y, flags = gpu_forward(wl)
        ref = oracle.forward(wl)
        assert rel_l2(y, ref) <= SIG_TOL
        rng = np.random.default_rng(10)
        res = (rng.normal(size=ref.shape) * np.abs(ref).max()).astype(np.float32)
        assert_grads(wl, gpu_adjoint(wl, res), oracle.adjoint(wl, res.astype(np.float64)))
    finally:
        for k, v in saved.items():
            binding.tune(k, v)


@pytest.mark.parametrize("col", [64, 128, 1, 2])     # 1, 2: the shared columns
def test_windows_longer_than_the_column(col):
    """Uniform spheres whose windows need more tile rows than the column holds (W from 55
    to 150 samples, R up to 2.8 mm) mixed with ordinary ones: the long windows go to the
    global trace directly, the chunk's integer-tile bound leaves them out."""
    from paper_2412_03898_amd import binding
    wl = tiny_scene(n_balls=400, n_sensors=70, seed=88)
    b = wl.balls.copy()
    rng = np.random.default_rng(88)
    delta = wl.c / wl.fs
    W = np.where(rng.uniform(size=b.shape[1]) < 0.3, rng.integers(55, 151, size=b.shape[1]),
                 rng.integers(7, 20, size=b.shape[1]))
    b[3] = ((W - 2 + rng.uniform(0.05, 0.95, size=W.size)) * delta / 2).astype(np.float32)
    k0 = synth.record_start(0.060, 0.010, 3.0e-3, 0.5e-3)
    n = synth.record_length_needed(0.060, 0.010, 3.0e-3, 0.5e-3, k0)
    wl = _morton(with_(wl, balls=b, t0=k0 / wl.fs, n_samples=n))
    saved = binding.tune_get(binding.SB_TUNE_FWD_COLUMN)
    try:
        binding.tune(binding.SB_TUNE_FWD_COLUMN, col)
        y, flags = gpu_forward(wl)
    finally:
        binding.tune(binding.SB_TUNE_FWD_COLUMN, saved)
    ref = oracle.forward(wl)
    err = rel_l2(y, ref)
    _say(f"windows longer than the column ({col}): rel-L2 {err:.3e} flags={flags}")
    assert flags == 0
    assert err <= SIG_TOL


@pytest.mark.parametrize("col", [128, 256, 1])     # 1: a lane per sample
def test_gaussian_ball_both_columns(col):
    """Gaussian balls (Fourier 4D, windows of 20 to 125 samples) at both column lengths
    of their forward: 128 rows in blocks of four waves, 256 rows in blocks of two."""
    from paper_2412_03898_amd import binding
    wl = tiny_scene(n_balls=600, n_sensors=140, n_frames=2, kernel=1, basis=1, seed=89)
    b = wl.balls.copy()
    rng = np.random.default_rng(89)
    b[3] = rng.uniform(0.05e-3, 0.35e-3, size=b.shape[1]).astype(np.float32)   # 6 sigma: up to 125 samples
    k0 = synth.record_start(0.060, 0.010, 0.35e-3 * 12, 0.5e-3)
    n = synth.record_length_needed(0.060, 0.010, 0.35e-3 * 12, 0.5e-3, k0)
    wl = with_(wl, balls=b, t0=k0 / wl.fs, n_samples=n)
    order = synth.morton_order(wl.balls)
    wl = with_(wl, balls=np.ascontiguousarray(wl.balls[:, order]),
               deform=np.ascontiguousarray(wl.deform[:, :, order]))
    saved = binding.tune_get(binding.SB_TUNE_FWD_GAUSS_COLUMN)
    try:
        binding.tune(binding.SB_TUNE_FWD_GAUSS_COLUMN, col)
        y, flags = gpu_forward(wl)
    finally:
        binding.tune(binding.SB_TUNE_FWD_GAUSS_COLUMN, saved)
    ref = oracle.forward(wl)
    err = rel_l2(y, ref)
    _say(f"gaussian column {col}: forward rel-L2 {err:.3e} flags={flags}")
    assert flags == 0
    assert err <= SIG_TOL


@pytest.mark.parametrize("col", [1, 256])     # 1: a lane per sample
def test_gaussian_ball_spread_chunks_and_windows_longer_than_the_row(col):
    """Gaussian balls in random order over a 20 mm cube (every 256-ball chunk spreads its
    arrivals at a sensor over ≈900 samples, more than the lane layout's 512-sample row, so
    the row is flushed and restarted) and a few balls whose windows exceed the row (520 to
    700 samples: added to the trace directly), against the oracle."""
    from paper_2412_03898_amd import binding
    wl = tiny_scene(n_balls=700, n_sensors=70, n_frames=2, kernel=1, basis=1, seed=91)
    b = wl.balls.copy()
    rng = np.random.default_rng(91)
    delta = wl.c / wl.fs
    big = rng.choice(b.shape[1], size=6, replace=False)
    W = rng.integers(520, 701, size=big.size)
    b[3, big] = ((W - 2 + 0.5) * delta / (2 * 6.0)).astype(np.float32)    # W = floor(12 rho) + 2
    k0 = synth.record_start(0.060, 0.010, float(b[3].max()) * 12 * 1.1, 0.5e-3)
    n = synth.record_length_needed(0.060, 0.010, float(b[3].max()) * 12 * 1.1, 0.5e-3, k0)
    wl = with_(wl, balls=b, t0=k0 / wl.fs, n_samples=n)               # unsorted on purpose
    saved = binding.tune_get(binding.SB_TUNE_FWD_GAUSS_COLUMN)
    try:
        binding.tune(binding.SB_TUNE_FWD_GAUSS_COLUMN, col)
        y, flags = gpu_forward(wl)
    finally:
        binding.tune(binding.SB_TUNE_FWD_GAUSS_COLUMN, saved)
    ref = oracle.forward(wl)
    err = rel_l2(y, ref)
    _say(f"gaussian spread chunks, long windows (column {col}): rel-L2 {err:.3e} flags={flags}")
    assert flags == 0
    assert err <= SIG_TOL
