"""Pins of the oracle's voxel grid and maximum amplitude projections (CPU).

The grid holds the model's initial pressure p0(x) = sum_b P_b phi(|x - x_b|)
at voxel centres.  Checked against facts that do not restate the rasteriser:
lattice-point counts of spheres, the Gaussian's integral, shift and
superposition, MAP supports, and the deformation of Eq. 1.
"""

import numpy as np
import pytest

import oracle
from helpers import with_
from paper_2412_03898_amd import synth


def ball(x, y, z, R, P):
    return np.array([[x], [y], [z], [R], [P]], dtype=np.float64)


H = 0.25                                   # binary-exact pitch: exact distances at the centres
GRID = (9, 9, 9, -1.0, -1.0, -1.0, H)      # centres -1, -0.75, ..., 1


@pytest.mark.parametrize("r_over_h, count", [(0.99, 1), (1.0, 7), (1.5, 19), (2.0, 33), (2.5, 81)])
def test_uniform_sphere_lattice_count(r_over_h, count):
    """Closed ball of radius r h around a voxel centre contains the lattice points
    i^2 + j^2 + k^2 <= r^2: 1, 7, 19, 33, 81 for r = 0.99, 1, 1.5, 2, 2.5."""
    v = oracle.voxelize(0, ball(0.0, 0.0, 0.0, r_over_h * H, 2.0), GRID)
    assert int((v > 0).sum()) == count
    assert set(np.unique(v)) <= {0.0, 2.0}


@pytest.mark.parametrize("r_over_h, ties", [(0.99, 0), (1.0, 6), (1.5, 0), (2.0, 6), (2.5, 0)])
def test_tie_voxels_are_the_lattice_points_on_the_sphere(r_over_h, ties):
    """Tie voxels (inside test decided by rounding) of a ball centred on a voxel of the
    binary-exact grid are exactly the lattice points with i^2 + j^2 + k^2 = r^2, where
    d = R holds exactly: the 6 axis neighbours for r = 1 and r = 2, none for r = 0.99,
    1.5 or 2.5 (r^2 not a sum of three squares of integers, or not an integer)."""
    R = r_over_h * H
    mask, n = oracle.voxel_ties(ball(0.0, 0.0, 0.0, R, 1.0), GRID)
    i = np.arange(9) - 4
    K, J, I = np.meshgrid(i, i, i, indexing="ij")
    exact = (I * I + J * J + K * K) * H * H == R * R
    assert n == ties == int(exact.sum())
    np.testing.assert_array_equal(mask, exact)


def test_gaussian_mass():
    """sum of voxels x h^3 = P (2 pi)^(3/2) a^3 (Riemann sum of a Gaussian with a = 4 h,
    grid reaching past 8 a on every side)."""
    h, a, P = 0.05, 0.2, 1.5
    n = 81
    g = (n, n, n, -2.0, -2.0, -2.0, h)
    v = oracle.voxelize(1, ball(0.013, -0.007, 0.021, a, P), g)
    assert v.sum() * h ** 3 == pytest.approx(P * (2 * np.pi) ** 1.5 * a ** 3, rel=1e-9)


def test_superposition_and_shift():
    rng = np.random.default_rng(3)
    a = np.vstack([rng.uniform(-0.5, 0.5, (3, 20)), rng.uniform(0.1, 0.4, (1, 20)), rng.uniform(0.5, 1, (1, 20))])
    g = (25, 23, 21, -1.5, -1.4, -1.3, 0.125)
    for kernel in (0, 1):
        whole = oracle.voxelize(kernel, a, g)
        parts = oracle.voxelize(kernel, a[:, :7], g) + oracle.voxelize(kernel, a[:, 7:], g)
        np.testing.assert_allclose(whole, parts, rtol=1e-12, atol=1e-12)
        # moving every ball by one pitch along x moves the grid by one voxel
        b = a.copy()
        b[0] += 0.125
        shifted = oracle.voxelize(kernel, b, g)
        np.testing.assert_allclose(shifted[:, :, 1:], whole[:, :, :-1], rtol=1e-12, atol=1e-12)


def test_map_of_one_sphere():
    """XY map of a sphere of radius 1.5 h at a voxel centre: value P on the 9 pixels
    i^2 + j^2 <= 2.25 and 0 elsewhere; the same for YZ and XZ."""
    v = oracle.voxelize(0, ball(0.0, 0.0, 0.0, 1.5 * H, 3.0), GRID)
    for m in oracle.maps(v):
        assert int((m > 0).sum()) == 9 and m.max() == 3.0


def test_map_is_axis_maximum():
    rng = np.random.default_rng(4)
    v = rng.normal(size=(5, 6, 7))
    xy, yz, xz = oracle.maps(v)
    assert xy.shape == (6, 7) and yz.shape == (5, 6) and xz.shape == (5, 7)
    for k in range(5):
        for j in range(6):
            for i in range(7):
                assert xy[j, i] >= v[k, j, i] and yz[k, j] >= v[k, j, i] and xz[k, i] >= v[k, j, i]
    assert np.all(np.any(v == xy[None], axis=0))


def test_invalid_balls_contribute_nothing():
    a = np.hstack([ball(0, 0, 0, 0.3, 1.0), ball(np.nan, 0, 0, 0.3, 1.0), ball(0, 0, 0, -0.3, 1.0),
                   ball(0, 0, 0, 0.3, -1.0)])
    np.testing.assert_array_equal(oracle.voxelize(0, a, GRID), oracle.voxelize(0, a[:, :1], GRID))


def test_deformed_scene_shift():
    """Fourier deformation with the cos(2 pi t) coefficient of x equal to one pitch
    (additive position, Eq. 1): at t = 0 the grid is the static grid shifted by one
    voxel; at t = 1/4 (cos = 0) it is the static grid."""
    wl = synth.workload_plain(n_balls=30, n_sensors=4)
    B = wl.balls.shape[1]
    h = 2.0 ** -11                         # exact in FP32, like the coefficient below
    g = (50, 48, 46, -0.012, -0.0115, -0.011, h)
    D = np.zeros((5, 2, B), dtype=np.float32)
    D[0, 0] = h
    w4 = with_(wl, basis=1, n_terms=1, pos_mode=0, deform=D)
    static = oracle.voxelize(0, wl.balls.astype(np.float64), g)
    at0 = oracle.voxelize_scene(w4, 0.0, g)
    np.testing.assert_allclose(at0[:, :, 1:], static[:, :, :-1], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle.voxelize_scene(w4, 0.25, g), static, rtol=1e-12, atol=1e-12)
