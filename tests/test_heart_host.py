"""Host-side pieces of the pulsating-heart workload (Sec. 3.1): the phantom and the
4D starting point, checked with the FP64 oracle's deformation (Eq. 1-2)."""

import numpy as np

import oracle
from helpers import with_
from paper_2412_03898_amd import heart, synth


def test_phantom_layout():
    slabs, ell = synth.heart_phantom(n_sensors=64, n_frames=5, spacing=1e-3)
    assert slabs.kernel == 0 and ell.kernel == 1 and ell.pos_mode == 1 and ell.basis == 1
    assert slabs.n_frames == ell.n_frames == 5 and slabs.t0 == ell.t0 and slabs.n_samples == ell.n_samples
    # full sphere of 60 mm
    r = np.linalg.norm(slabs.sensors.astype(np.float64), axis=0)
    np.testing.assert_allclose(r, 0.060, rtol=1e-6)
    assert slabs.sensors[2].min() < -0.05 and slabs.sensors[2].max() > 0.05
    # three slabs, each thin along one axis
    x = slabs.balls[0:3]
    thin = [(np.abs(x[a]) <= 1.05e-3).mean() for a in range(3)]
    assert min(thin) > 0.3
    assert np.all(np.abs(x) <= 12.2e-3)        # 12 mm plus the seeded jitter


def test_ellipsoid_pulsates_and_slabs_stay():
    """Deformed by Eq. 1 (oracle): the ellipsoid scales by 1 + a sin(2 pi t) about the centre,
    its size and pressure follow; the slabs carry no deformation."""
    slabs, ell = synth.heart_phantom(n_sensors=16, n_frames=5, spacing=1e-3, size_amp=0.25, p_amp=0.4)
    assert slabs.deform is None
    t = ell.frame_t
    for f in range(5):
        d = oracle.deformed(ell, f)
        s = 1.0 + 0.25 * np.sin(2 * np.pi * float(t[f]))
        np.testing.assert_allclose(d[0:4], ell.balls[0:4].astype(np.float64) * s, rtol=1e-6, atol=1e-12)
        np.testing.assert_allclose(d[4], ell.balls[4] * (1.0 + 0.4 * np.sin(2 * np.pi * float(t[f]))), rtol=1e-6)


def test_gauss_basis_start_is_identity():
    """All Eq. 2 weights zero: the deformed cloud equals the base cloud at every time."""
    cloud = heart.init_cloud(4e-3, 2e-3, 0.3e-3, 0.02, 1)
    B = cloud.shape[1]
    D = heart.gauss_basis_start(B, 5)
    wl = synth.workload_plain(n_balls=B, n_sensors=4)
    wl = with_(wl, balls=cloud, deform=D, basis=2, n_terms=5, pos_mode=1,
               frame_t=np.array([0.0, 0.3, 1.0], np.float32), frame_offset=np.array([0, 3]))
    for f in range(3):
        np.testing.assert_allclose(oracle.deformed(wl, f), cloud.astype(np.float64), rtol=0, atol=0)
    assert D[:, 1::3].min() == 0.0 and D[:, 1::3].max() == 1.0 and np.all(D[:, 2::3] > 0)
