"""The two-stage reconstruction of the pulsating-heart phantom runs end to end on the
GPU (small version): both stages reduce their loss and the MAP correlations are finite."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_two_stage_small():
    from paper_2412_03898_amd import heart
    print("[gpu-heart] two-stage, 128 sensors, 5 frames", flush=True)
    sys.stdout.flush()
    rec = heart.two_stage(n_static=25, n_4d=25, n_sensors=128, n_frames=5, fit_half=8e-3, fit_spacing=1.6e-3,
                          phantom_spacing=1e-3, voxel=0.5e-3, lr_scale=10.0, log=lambda s: print(s, flush=True))
    a, b = rec["stage1_loss"]
    c, d = rec["stage2_loss_all_frames"]
    assert b < a and d < c
    for plane in ("xy", "yz", "xz"):
        assert np.all(np.isfinite(rec["map_corr"]["25"][plane]))
