"""GPU parity of the voxel grid and the maximum amplitude projections
(slingbag_voxelize, slingbag_map) against the FP64 oracle.

Bars: relative L2 <= 1e-5 over the volume and over each projection; for the
uniform sphere the inside test is FP64 on both sides, so the set of voxels a
ball reaches is identical, except at tie voxels: centres so close to a ball's
surface that two FP64 evaluations of d^2 (the oracle's plain sum, the kernel's
fused multiply-adds) may decide differently (oracle.voxel_ties).  Those are
counted and reported (none are expected), and excluded from the set comparison.
"""

import sys

import numpy as np
import pytest

import oracle
from helpers import rel_l2, with_
from paper_2412_03898_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _say(msg):
    print(f"[gpu-voxel] {msg}", flush=True)
    sys.stdout.flush()


def gpu_voxelize(wl, t, grid, balls=None, strict=True):
    import torch
    from paper_2412_03898_amd import binding, ops
    w = wl if balls is None else with_(wl, balls=balls)
    pb, b, d, _, _ = ops.to_device(w)
    vol = ops.voxelize(pb, b, d, t, grid)
    maps = ops.map_projections(vol)
    torch.cuda.synchronize()
    try:
        flags = ops.check()
    except binding.SlingbagError:
        if strict:
            raise
        flags = None
    return vol.cpu().numpy(), [m.cpu().numpy() for m in maps], flags


def compare(wl, t, grid, balls=None):
    got, gmaps, flags = gpu_voxelize(wl, t, grid, balls)
    ref = oracle.voxelize_scene(wl, t, grid, balls=balls)
    rmaps = oracle.maps(ref)
    err = rel_l2(got, ref)
    merr = [rel_l2(g, r) for g, r in zip(gmaps, rmaps)]
    ties = 0
    if wl.kernel == 0:
        tie, ties = oracle.voxel_ties_scene(wl, t, grid, balls=balls)
        np.testing.assert_array_equal((got != 0)[~tie], (ref != 0)[~tie])
    _say(f"volume rel-L2 {err:.2e}, maps {['%.2e' % e for e in merr]}, nonzero {int((ref != 0).sum())}, "
         f"tie voxels {ties}")
    assert err <= TOL and max(merr) <= TOL
    return flags


def plain(kernel, n=400, seed=21):
    wl = synth.workload_plain(n_balls=n, n_sensors=4, seed=seed)
    return with_(wl, kernel=kernel)


GRID = (61, 57, 53, -0.0101, -0.0099, -0.0102, 0.35e-3)     # ragged sizes, 0.35 mm pitch


@pytest.mark.parametrize("kernel", [0, 1])
def test_static_scene(kernel):
    _say(f"static kernel={kernel}")
    assert compare(plain(kernel), 0.0, GRID) == 0


@pytest.mark.parametrize("pos_mode", [0, 1])
def test_fourier_scene(pos_mode):
    wl = synth.workload_vessel_4d(n_balls=600, n_frames=3, n_sensors=4, n_samples=64)
    wl = with_(wl, pos_mode=pos_mode)
    if pos_mode == 1:      # multiplicative position scales: keep them small
        D = wl.deform.copy()
        D[0:3] *= 10.0
        wl = with_(wl, deform=D)
    g = (80, 81, 79, -0.02, -0.0202, -0.0199, 0.5e-3)
    for t in (0.0, 0.37):
        _say(f"fourier pos_mode={pos_mode} t={t}")
        compare(wl, t, g)


def test_gauss_basis_scene():
    wl = synth.workload_vessel_4d(n_balls=300, n_frames=2, n_sensors=4, n_samples=64)
    B = wl.balls.shape[1]
    D = synth.gauss_basis_coeffs(B, 3, 5)
    wl = with_(wl, basis=2, n_terms=3, deform=D)
    _say("gaussian basis")
    compare(wl, 0.6, (80, 80, 80, -0.02, -0.02, -0.02, 0.5e-3))


def test_edges():
    """Balls outside the grid, straddling its faces, covering all of it, and invalid
    balls (skipped and flagged); a one-voxel-thick grid."""
    wl = plain(0, n=6)
    b = wl.balls.copy()
    b[:, 0] = [0.5, 0.0, 0.0, 1e-3, 1.0]             # far outside
    b[:, 1] = [-0.0101, 0.0, 0.0, 1e-3, 1.0]         # centre on the lower x face
    b[:, 2] = [0.0, 0.0, 0.0, 0.5, 0.7]              # covers the whole grid
    b[:, 3] = [np.nan, 0.0, 0.0, 1e-3, 1.0]          # invalid
    b[:, 4] = [0.001, 0.002, 0.003, -1e-3, 1.0]      # invalid size
    from paper_2412_03898_amd import binding
    with pytest.raises(binding.SlingbagError) as err:      # the invalid balls set SB_FLAG_NONFINITE
        gpu_voxelize(wl, 0.0, GRID, balls=b)
    assert err.value.status == binding.SB_ERR_DEVICE_FLAG
    got, _, _ = gpu_voxelize(wl, 0.0, GRID, balls=b, strict=False)
    keep = b[:, [0, 1, 2, 5]]
    ref = oracle.voxelize_scene(with_(wl, balls=keep), 0.0, GRID)
    assert rel_l2(got, ref) <= TOL
    thin = (40, 1, 33, -0.01, 0.0, -0.01, 0.4e-3)
    compare(with_(wl, balls=b[:, [1, 2, 5]]), 0.0, thin)


def test_empty_scene_gives_zero_volume():
    import torch
    from paper_2412_03898_amd import ops
    wl = plain(0, n=1)
    pb = ops.Problem(0, 0, 0, 0, 4, 64, wl.c, wl.fs, wl.t0, np.array([0, 0]), np.array([0, 1]))
    vol = torch.full((5, 6, 7), 3.0, device="cuda")
    balls = torch.zeros((5, 0), device="cuda")
    ops.voxelize(pb, balls, None, 0.0, (7, 6, 5, 0.0, 0.0, 0.0, 1e-3), out=vol)
    assert float(vol.abs().max()) == 0.0


def test_large_scene_full_size():
    """The 1M-ball 32-frame scene at t = 0.5 on a 40 mm cube of 0.1 mm voxels (400^3)."""
    wl = synth.workload_large_ir()
    g = (400, 400, 400, -0.01995, -0.01995, -0.01995, 0.1e-3)
    _say("1M balls, 400^3 voxels, t = 0.5")
    compare(wl, 0.5, g)
