"""Pins of the FP64 oracle against facts fixed by physics and mathematics.

None of these re-types the oracle's formulas: each checks it against an
independent route (exact rational arithmetic of the N-wave, brute-force
quadrature of Poisson's spherical-means formula, invariances of the wave
equation, finite differences, special values of the deformation functions).
"""

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
from helpers import rel_l2, tiny_scene, with_
from paper_2412_03898_amd import synth


def single(kernel, R, P=1.0, r_samples=1600, t0=0.0, T=2048, ball=(0.0, 0.0, 0.0), sensor_dir=(1, 0, 0)):
    delta = synth.C_SOUND / synth.FS
    sd = np.asarray(sensor_dir, dtype=np.float64)
    sd = sd / np.linalg.norm(sd)
    sens = (np.asarray(ball) + sd * r_samples * delta).reshape(3, 1)
    return tiny_scene(n_balls=1, n_sensors=1) if False else with_(
        tiny_scene(n_balls=1, n_sensors=1), kernel=kernel, t0=t0, n_samples=T,
        sensors=sens, balls=np.array([[ball[0]], [ball[1]], [ball[2]], [R], [P]], dtype=np.float64))


# ---------------------------------------------------------------- closed forms (Sec. 2.1 radiator)
def test_nwave_exact_rationals():
    """Uniform ball, R = 8 delta, r = 1600 delta, t0 = 0: every sample is the average of
    the N-wave P(r-ct)/(2r) over its interval, which for a linear profile is the
    overlap length times the midpoint value - exact rationals in units of delta."""
    delta = synth.C_SOUND / synth.FS
    wl = single(0, R=8 * delta, P=1.0)
    y = oracle.forward(wl)[0, 0]
    R = Fraction(8)
    r = Fraction(1600)
    for k in range(1585, 1616):
        u = r - k                      # (r - c t_k)/delta
        lo, hi = max(u - Fraction(1, 2), -R), min(u + Fraction(1, 2), R)
        exact = Fraction(0) if lo >= hi else (hi - lo) * ((lo + hi) / 2) / (2 * r)   # x delta/delta
        assert y[k] == pytest.approx(float(exact), abs=1e-15), k
    # worked numbers in closed form: edge = P(2R - delta/2)/(8r), interior = P u/(2r)
    assert y[1592] == pytest.approx((2 * 8 - 0.5) / (8 * 1600), rel=1e-12)
    assert y[1593] == pytest.approx(7 / (2 * 1600), rel=1e-12)
    assert abs(y[1600]) < 1e-15
    assert np.count_nonzero(np.abs(y) > 1e-15) == 16


@pytest.mark.parametrize("kernel,R", [(0, 0.3e-3), (1, 0.2e-3)])
def test_zero_sum(kernel, R):
    """The sampled trace of one ball telescopes: its samples sum to zero."""
    wl = single(kernel, R=R, P=0.7)
    y = oracle.forward(wl)[0, 0]
    assert abs(y.sum()) < 1e-12 * np.abs(y).max()


def test_gauss_ball_values():
    """Gaussian ball (std a, r = 1600 delta, t0 = 0): the centre sample is 0 (odd
    profile) and samples at +-m from the centre are opposite; a far sample equals
    the closed-form difference of exp terms evaluated here independently."""
    delta = synth.C_SOUND / synth.FS
    a = 0.2e-3
    wl = single(1, R=a, P=1.0)
    y = oracle.forward(wl)[0, 0]
    assert abs(y[1600]) < 1e-16
    for m in range(1, 12):
        assert y[1600 + m] == pytest.approx(-y[1600 - m], rel=1e-12, abs=1e-18)
    # sample at u = 5 delta: (1/delta) * integral of (1/2r) s exp(-s^2/2a^2) ds over [4.5, 5.5] delta
    r = 1600 * delta
    g = lambda s: -(a * a / (2 * r)) * math.exp(-s * s / (2 * a * a))
    assert y[1595] == pytest.approx((g(5.5 * delta) - g(4.5 * delta)) / delta, rel=1e-12)


# ---------------------------------------------------------------- brute force (Poisson)
@pytest.mark.parametrize("kernel,n_mu,tol", [(1, 20_000, 5e-6), (0, 200_000, 1e-4)])
def test_bruteforce_poisson(kernel, n_mu, tol):
    """Two balls, two sensors, nonzero t0: closed form vs quadrature of Poisson's formula."""
    wl = tiny_scene(n_balls=2, n_sensors=2, kernel=kernel, seed=3)
    y = oracle.forward(wl)[0]
    amax = np.abs(y).max()
    nz = np.nonzero(np.abs(y).max(axis=0) > 1e-9 * amax)[0]
    kr = (int(nz.min()) - 2, int(nz.max()) + 2)
    yb = brute.forward_bruteforce(wl.balls, wl.sensors, wl.c, wl.fs, wl.t0, wl.n_samples,
                                  kernel, k_range=kr, n_mu=n_mu, n_phi=2)
    for j in range(2):
        sel = np.abs(y[j]) > 0
        assert rel_l2(yb[j][sel], y[j][sel]) < tol
    # nothing (uniform) or only the far Gaussian tail outside the evaluated range
    outside = max(np.abs(y[:, :kr[0]]).max(initial=0), np.abs(y[:, kr[1] + 1:]).max(initial=0))
    assert outside <= (0.0 if kernel == 0 else 1e-9 * amax)


# ---------------------------------------------------------------- Gaussian ball, sensor near the ball
# The Gaussian ball's incoming (r + ct) term is below the double range at every sensor of
# the workloads; these pins put the sensor 2.5 std from the centre, with the record
# starting at t = 0, where that term carries half of the pressure.
def _near_gauss(fs, a=0.2e-3, r_over_a=2.5, T=None, P=1.3):
    delta = synth.C_SOUND / fs
    r = r_over_a * a
    if T is None:
        T = int(math.ceil((r + 12 * a) / delta)) + 4
    return with_(tiny_scene(n_balls=1, n_sensors=1, kernel=1), fs=fs, t0=0.5 / fs, n_samples=T,
                 sensors=np.array([[r], [0.0], [0.0]]),
                 balls=np.array([[0.0], [0.0], [0.0], [a], [P]], dtype=np.float64))


def test_gauss_ball_initial_condition_at_the_sensor():
    """The wave equation's solution starts from the initial pressure: p(x_s, 0+) =
    P exp(-r^2/2a^2) at a sensor r from the centre (zero initial velocity, so p changes as
    t^2).  The first sample averages p over [0, dt]; with c dt = a/53 the t^2 term moves it
    by ~2e-4 relative.  The outgoing (r - ct) term alone gives half of p0, a sign error in
    the incoming term gives ~0, so either mistake fails by orders of magnitude."""
    fs = 400e6
    wl = _near_gauss(fs)
    y = oracle.forward(wl)[0, 0]
    r, a, P = float(wl.sensors[0, 0]), float(wl.balls[3, 0]), float(wl.balls[4, 0])
    p0 = P * math.exp(-r * r / (2 * a * a))
    assert y[0] == pytest.approx(p0, rel=1e-3)
    assert y[0] != pytest.approx(0.5 * p0, rel=0.1)


def test_gauss_ball_near_sensor_bruteforce():
    """Sensor 2.5 std from a Gaussian ball, record from t = 0: the closed form (both
    terms) against quadrature of Poisson's formula over every sample."""
    wl = _near_gauss(synth.FS)
    y = oracle.forward(wl)[0]
    yb = brute.forward_bruteforce(wl.balls, wl.sensors, wl.c, wl.fs, wl.t0, wl.n_samples, 1,
                                  n_mu=20_000, n_phi=2)
    assert rel_l2(yb, y) < 5e-6
    # the incoming term is not negligible here: the first samples carry a large share
    assert abs(y[0, 0]) > 0.05 * np.abs(y).max()


def test_gauss_ball_near_sensor_gradient():
    """Gradient of 1/2|y - d|^2 with the incoming term active (sensor 2.5 std from the
    centre) against central differences of the FP64 loss, for position, std and pressure."""
    wl = _near_gauss(synth.FS)
    d = oracle.forward(wl, balls=wl.balls * np.array([[1.0], [1.0], [1.0], [1.07], [0.9]]) +
                       np.array([[2e-5], [0.0], [0.0], [0.0], [0.0]]))
    y = oracle.forward(wl)
    gb, _ = oracle.adjoint(wl, y - d)
    balls = wl.balls.astype(np.float64)
    for a, e in ((0, 1e-9), (1, 1e-9), (3, 1e-9), (4, 1e-6)):
        bp, bm = balls.copy(), balls.copy()
        bp[a, 0] += e
        bm[a, 0] -= e
        fd = (_loss_at(wl, d, bp, None) - _loss_at(wl, d, bm, None)) / (2 * e)
        assert gb[a, 0] == pytest.approx(fd, rel=2e-5, abs=1e-9 * np.abs(gb).max()), a


# ---------------------------------------------------------------- invariances
def test_superposition_and_homogeneity():
    wl = tiny_scene(n_balls=8, n_sensors=6, seed=5)
    y = oracle.forward(wl)
    a = oracle.forward(with_(wl, balls=wl.balls[:, :3], ball_offset=np.array([0, 3])))
    b = oracle.forward(with_(wl, balls=wl.balls[:, 3:], ball_offset=np.array([0, 5])))
    assert rel_l2(a + b, y) < 1e-14
    scaled = wl.balls.astype(np.float64).copy()
    scaled[4] *= 2.5
    assert rel_l2(oracle.forward(wl, balls=scaled), 2.5 * y) < 1e-14


@pytest.mark.parametrize("kernel", [0, 1])
def test_rotation_invariance(kernel):
    """Rotating balls and sensors together by an orthogonal Q leaves every trace unchanged."""
    wl = tiny_scene(n_balls=5, n_sensors=4, kernel=kernel, seed=9)
    y = oracle.forward(wl)
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    balls = wl.balls.astype(np.float64).copy()
    balls[0:3] = Q @ balls[0:3]
    sens = Q @ wl.sensors.astype(np.float64)
    y2 = oracle.forward(with_(wl, balls=balls, sensors=sens))
    assert rel_l2(y2, y) < 1e-9


def test_centred_ball_same_trace_at_every_sensor():
    """A ball at the centre of the shell reaches every sensor at the same time."""
    wl = tiny_scene(n_balls=1, n_sensors=7)
    sens = synth.fibonacci_sphere(7, 1.0).astype(np.float64)
    sens = 0.060 * sens / np.linalg.norm(sens, axis=0)      # exact radius in float64
    wl = with_(wl, balls=np.array([[0.0], [0.0], [0.0], [0.25e-3], [0.9]]), sensors=sens)
    y = oracle.forward(wl)[0]
    for j in range(1, 7):
        assert rel_l2(y[j], y[0]) < 1e-9


@pytest.mark.parametrize("m", [1, 3, -2])
def test_radial_shift(m):
    """Moving a uniform ball by m*delta away from the sensor shifts its trace by m samples
    and scales it by r/(r + m delta) (time of flight and the 1/r law)."""
    delta = synth.C_SOUND / synth.FS
    R = 0.27e-3
    wl = single(0, R=R, P=0.8, r_samples=1500.3, t0=2e-6, T=2000, sensor_dir=(0.3, -0.5, 0.8))
    y = oracle.forward(wl)[0, 0]
    d = -(wl.sensors[:, 0] - wl.balls[0:3, 0])
    d = d / np.linalg.norm(d)
    r = 1500.3 * delta
    b2 = wl.balls.copy()
    b2[0:3, 0] += d * m * delta
    y2 = oracle.forward(wl, balls=b2)[0, 0]
    ref = np.zeros_like(y)
    if m > 0:
        ref[m:] = y[:-m]
    else:
        ref[:m] = y[-m:]
    assert rel_l2(y2, ref * r / (r + m * delta)) < 1e-9


# ---------------------------------------------------------------- deformation (Eq. 1-2)
def test_fourier_special_times():
    """At t = 1/4 the 2-harmonic series is b_1 - a_2; at t = 1/2 it is -a_1 + a_2; at t = 0,
    a_1 + a_2.  Additive position, multiplicative size and pressure (Eq. 1)."""
    wl = tiny_scene(n_balls=4, n_sensors=2, n_frames=3, basis=1, K=2)
    wl = with_(wl, frame_t=np.array([0.0, 0.25, 0.5], dtype=np.float32))
    D = wl.deform.astype(np.float64)
    base = wl.balls.astype(np.float64)
    H = {0: D[:, 0] + D[:, 2], 1: D[:, 1] - D[:, 2], 2: -D[:, 0] + D[:, 2]}
    for f in range(3):
        got = oracle.deformed(wl, f)
        exp = base.copy()
        exp[0:3] += H[f][0:3]
        exp[3:5] *= 1.0 + H[f][3:5]
        np.testing.assert_allclose(got, exp, rtol=1e-12, atol=1e-18)


def test_gauss_basis_special_values():
    """Eq. 2: one basis evaluated at its centre gives w; at centre +- sigma gives w e^{-1/2}.
    Multiplicative position (Eq. 1): mu(t) = mu (1 + H)."""
    wl = tiny_scene(n_balls=3, n_sensors=2, n_frames=3, basis=2, N=1, pos_mode=1)
    D = wl.deform.astype(np.float64).copy()
    D[:, 1] = 0.4      # theta
    D[:, 2] = 0.1      # sigma
    wl = with_(wl, deform=D, frame_t=np.array([0.4, 0.5, 0.3]))
    base = wl.balls.astype(np.float64)
    for f, fac in ((0, 1.0), (1, math.exp(-0.5)), (2, math.exp(-0.5))):
        got = oracle.deformed(wl, f)
        np.testing.assert_allclose(got, base * (1.0 + fac * D[:, 0]), rtol=1e-12)


def test_fourier_periodic_in_t():
    """Frames at t = 0 and t = 1 of a Fourier deformation produce identical signals."""
    wl = tiny_scene(n_balls=5, n_sensors=3, n_frames=2, basis=1)
    y = oracle.forward(wl)
    assert rel_l2(y[1], y[0]) < 1e-10


def test_zero_coefficients_reduce_to_static():
    for basis in (1, 2):
        wl = tiny_scene(n_balls=5, n_sensors=3, n_frames=4, basis=basis)
        D = wl.deform.astype(np.float64).copy()
        if basis == 1:
            D[:] = 0.0
        else:
            D[:, 0::3] = 0.0
        y = oracle.forward(wl, deform=D)
        ys = oracle.forward(with_(wl, basis=0, n_terms=0, deform=None, frame_t=np.zeros(1),
                                  frame_offset=np.array([0, 1])))
        for f in range(4):
            assert rel_l2(y[f], ys[0]) < 1e-14


def test_deformed_frames_equal_static_scenes():
    """Each frame of a deformed scene equals the static forward of that frame's attributes."""
    wl = tiny_scene(n_balls=6, n_sensors=3, n_frames=3, basis=1)
    y = oracle.forward(wl)
    for f in range(3):
        attrs = oracle.deformed(wl, f)
        ys = oracle.forward(with_(wl, basis=0, n_terms=0, deform=None, balls=attrs,
                                  frame_t=np.zeros(1), frame_offset=np.array([0, 1])))
        assert rel_l2(y[f], ys[0]) < 1e-13


# ---------------------------------------------------------------- loss and gradient
def test_loss_values():
    y = np.array([[1.0, 2.0, -1.0]])
    d = np.array([[0.5, 2.0, 1.0]])
    L, r = oracle.loss(y, d)
    assert L == 0.5 * (0.25 + 0 + 4.0)
    np.testing.assert_array_equal(r, [[0.5, 0.0, -2.0]])


def _loss_at(wl, d, balls, deform):
    y = oracle.forward(wl, balls=balls, deform=deform)
    return 0.5 * float(((y - d) ** 2).sum())


CASES = [
    dict(basis=0, kernel=0),
    dict(basis=0, kernel=1),
    dict(basis=1, kernel=0, n_frames=3),
    dict(basis=1, kernel=0, n_frames=3, pos_mode=1),
    dict(basis=2, kernel=0, n_frames=3),
    dict(basis=2, kernel=1, n_frames=2, pos_mode=1),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(f"{k}{v}" for k, v in c.items()))
def test_gradient_central_differences(case):
    """Every gradient entry of 1/2|y - d|^2 against central differences of the FP64 loss."""
    wl = tiny_scene(n_balls=3, n_sensors=3, seed=21, **case)
    balls = wl.balls.astype(np.float64)
    D = None if wl.deform is None else wl.deform.astype(np.float64)
    pert = synth.perturbed(wl.balls, 22)
    d = oracle.forward(wl, balls=pert)
    y = oracle.forward(wl)
    gb, gd = oracle.adjoint(wl, y - d)
    scale_b = np.array([1e-9, 1e-9, 1e-9, 1e-9, 1e-6])
    for a in range(5):
        for b in range(balls.shape[1]):
            e = scale_b[a] if a < 4 else 1e-6
            bp, bm = balls.copy(), balls.copy()
            bp[a, b] += e
            bm[a, b] -= e
            fd = (_loss_at(wl, d, bp, D) - _loss_at(wl, d, bm, D)) / (2 * e)
            assert gb[a, b] == pytest.approx(fd, rel=2e-5, abs=1e-9 * max(1.0, np.abs(gb[a]).max())), (a, b)
    if D is not None:
        M = D.shape[1]
        for a in range(5):
            for m in range(M):
                for b in range(balls.shape[1]):
                    mag = abs(D[a, m, b])
                    e = max(mag, 1e-4 if a >= 3 else 1e-7) * 1e-5
                    Dp, Dm = D.copy(), D.copy()
                    Dp[a, m, b] += e
                    Dm[a, m, b] -= e
                    fd = (_loss_at(wl, d, balls, Dp) - _loss_at(wl, d, balls, Dm)) / (2 * e)
                    tol = 1e-9 * max(1.0, np.abs(gd[a]).max())
                    assert gd[a, m, b] == pytest.approx(fd, rel=5e-5, abs=tol), (a, m, b)


def test_adjoint_dot_product():
    """<J v, w> = <v, J^T w> with J v from central differences of the forward map and
    J^T w from the oracle adjoint fed an arbitrary residual w."""
    wl = tiny_scene(n_balls=5, n_sensors=4, n_frames=3, basis=1, seed=31)
    rng = np.random.default_rng(3)
    balls = wl.balls.astype(np.float64)
    D = wl.deform.astype(np.float64)
    w = rng.normal(size=(3, 4, wl.n_samples))
    gb, gd = oracle.adjoint(wl, w)
    vb = rng.normal(size=balls.shape) * np.array([1, 1, 1, 0.1, 1e3])[:, None] * 1e-6
    vd = rng.normal(size=D.shape) * 1e-6
    vd[:3] *= 1.0
    vd[3:] *= 1e3
    eps = 1e-3
    yp = oracle.forward(wl, balls=balls + eps * vb, deform=D + eps * vd)
    ym = oracle.forward(wl, balls=balls - eps * vb, deform=D - eps * vd)
    lhs = float(((yp - ym) / (2 * eps) * w).sum())
    rhs = float((vb * gb).sum() + (vd * gd).sum())
    assert lhs == pytest.approx(rhs, rel=1e-5)


def test_gradient_identity_fourier_vs_per_frame():
    """dL/da_k^x = sum_f cos(2 pi k t_f) dL/dx_f: the deformed gradient equals the per-frame
    static gradients (at each frame's attributes) combined with the Fourier basis values."""
    wl = tiny_scene(n_balls=4, n_sensors=3, n_frames=4, basis=1, seed=41)
    rng = np.random.default_rng(5)
    res = rng.normal(size=(4, 3, wl.n_samples))
    gb, gd = oracle.adjoint(wl, res)
    acc_x = np.zeros((4,))
    acc_cos1 = np.zeros((4,))
    acc_sin2_R = np.zeros((4,))
    for f in range(4):
        attrs = oracle.deformed(wl, f)
        sw = with_(wl, basis=0, n_terms=0, deform=None, balls=attrs, frame_t=np.zeros(1),
                   frame_offset=np.array([0, 1]))
        g, _ = oracle.adjoint(sw, res[f:f + 1])
        t = float(wl.frame_t[f])
        acc_x += g[0]
        acc_cos1 += g[0] * math.cos(2 * math.pi * t)
        acc_sin2_R += g[3] * wl.balls[3].astype(np.float64) * math.sin(4 * math.pi * t)
    np.testing.assert_allclose(gb[0], acc_x, rtol=1e-10)
    np.testing.assert_allclose(gd[0, 0], acc_cos1, rtol=1e-10)
    np.testing.assert_allclose(gd[3, 3], acc_sin2_R, rtol=1e-10)


def test_multi_scene_batch_is_concatenation():
    """Two scenes in one batch give exactly the two single-scene results."""
    a = tiny_scene(n_balls=3, n_sensors=3, n_frames=2, basis=1, seed=51)
    b = tiny_scene(n_balls=4, n_sensors=3, n_frames=3, basis=1, seed=52)
    b = with_(b, sensors=a.sensors, n_samples=a.n_samples, t0=a.t0)
    both = with_(a, balls=np.concatenate([a.balls, b.balls], axis=1),
                 deform=np.concatenate([a.deform, b.deform], axis=2),
                 frame_t=np.concatenate([a.frame_t, b.frame_t]),
                 ball_offset=np.array([0, 3, 7]), frame_offset=np.array([0, 2, 5]))
    y = oracle.forward(both)
    assert rel_l2(y[:2], oracle.forward(a)) == 0.0
    assert rel_l2(y[2:], oracle.forward(b)) == 0.0
    rng = np.random.default_rng(1)
    res = rng.normal(size=y.shape)
    gb, gd = oracle.adjoint(both, res)
    ga, gda = oracle.adjoint(a, res[:2])
    gbb, gdb = oracle.adjoint(b, res[2:])
    np.testing.assert_array_equal(gb[:, :3], ga)
    np.testing.assert_array_equal(gb[:, 3:], gbb)
    np.testing.assert_array_equal(gd[:, :, 3:], gdb)


def test_invalid_geometry_is_reported():
    wl = single(0, R=0.3e-3)
    wl = with_(wl, sensors=np.array([[0.0001], [0.0], [0.0]]))
    with pytest.raises(oracle.OracleError):
        oracle.forward(wl)


def test_oracle_regression_fixture():
    """The oracle still reproduces the values its own generator script stored."""
    import os
    import sys
    here = os.path.join(os.path.dirname(__file__), "golden")
    sys.path.insert(0, here)
    import make_golden
    stored = {}
    with open(os.path.join(here, "oracle_regression.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, key, val = line.split()
            stored[(name, key)] = float(val)
    got = {(n, k): v for n, k, v in make_golden.rows()}
    assert set(got) == set(stored)
    for key, val in stored.items():
        assert got[key] == pytest.approx(val, rel=1e-12), key


def test_adam_first_step_is_signed_lr():
    """With zero moments, the first bias-corrected Adam step moves each parameter by
    lr * g/(|g| + eps): lr*sign(g) for |g| >> eps."""
    rng = np.random.default_rng(9)
    p = rng.normal(size=50)
    g = rng.normal(size=50) * 10.0
    newp, m, v = oracle.adam_step(p, g, np.zeros(50), np.zeros(50), lr=1e-3, step=1)
    np.testing.assert_allclose(newp, p - 1e-3 * np.sign(g), rtol=0, atol=1e-3 * 1e-8 / 1e-2 + 1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)
    # a constant gradient keeps the step at lr (bias correction cancels the moment decay)
    p2, m2, v2 = oracle.adam_step(newp, g, m, v, lr=1e-3, step=2)
    np.testing.assert_allclose(p2, newp - 1e-3 * np.sign(g), atol=1e-12)
