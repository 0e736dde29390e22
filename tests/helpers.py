"""Small shared test utilities: tiny seeded scenes and error norms (no method arithmetic)."""

import types

import numpy as np

from paper_2412_03898_amd import synth


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def tiny_scene(n_balls=6, n_sensors=5, n_samples=None, n_frames=1, basis=0, K=2, N=3,
               pos_mode=0, kernel=0, seed=11, shell=0.060, half=0.010):
    """A few balls in a cube, sensors on a hemisphere; optional deformation."""
    if kernel == 0:
        balls = synth.uniform_cube_balls(n_balls, half, (0.1e-3, 0.3e-3), (0.5, 1.0), seed)
        rmax = 0.3e-3
    else:
        balls = synth.uniform_cube_balls(n_balls, half, (0.05e-3, 0.15e-3), (0.5, 1.0), seed)
        rmax = 0.15e-3 * 12  # Gaussian window reach
    if pos_mode == 1:
        balls[0:3] += np.float32(0.004)   # keep multiplicative positions away from the origin
    deform = None
    if basis == 1:
        deform = synth.fourier_coeffs(n_balls, K, seed + 1)
    elif basis == 2:
        deform = synth.gauss_basis_coeffs(n_balls, N, seed + 1, mul_pos=(pos_mode == 1))
    reach_half = half + (0.004 if pos_mode == 1 else 0.0)
    k0 = synth.record_start(shell, reach_half, rmax * 1.1, 0.5e-3)
    need = synth.record_length_needed(shell, reach_half, rmax * 1.1, 0.5e-3, k0)
    if n_samples is None:
        n_samples = need
    assert n_samples >= need
    return types.SimpleNamespace(
        kernel=kernel, basis=basis, pos_mode=pos_mode,
        n_terms=(K if basis == 1 else (N if basis == 2 else 0)),
        c=synth.C_SOUND, fs=synth.FS, t0=k0 / synth.FS, n_samples=n_samples,
        sensors=synth.fibonacci_sphere(n_sensors, shell), balls=balls, deform=deform,
        frame_t=synth.frame_times(n_frames),
        ball_offset=np.array([0, n_balls], dtype=np.int64),
        frame_offset=np.array([0, n_frames], dtype=np.int64))


def with_(wl, **kw):
    d = dict(vars(wl))
    d.update(kw)
    return types.SimpleNamespace(**d)
