"""GPU parity of the forward's other layouts: the forward cases of the parity suite, run
again with the uniform sphere's 64-sample column per wave and its 132-sample shared column,
and with the Gaussian ball's 256- and 128-sample columns per wave (the suite itself runs
the defaults: the 92-sample shared column and a lane per sample).  Unsorted balls (every 256-ball chunk spans the whole cube) make each
sensor's arrivals spread over several columns, so they take the multi-pass path;
sensors among the balls take the path without an integer scale."""

import pytest

from test_gpu_parity import (plain, test_4d_fourier_small, test_ball_longer_than_any_record_is_skipped_and_flagged,  # noqa: F401
                             test_clipped_record_is_dropped_and_flagged, test_heart_ellipsoid_full_size_sampled, test_forward_plain,
                             test_large_ir_scene_full_size_sampled, test_nonfinite_ball_is_skipped_and_flagged,
                             test_result_independent_of_order, test_sensor_inside_ball_raises_flag,
                             test_sensors_among_the_balls, test_single_ball_single_sensor,
                             test_uneven_batch_full_size_sampled, test_uneven_batch_with_empty_scene,
                             test_variants, test_vessel_4d_full_size_sampled, test_vessel_static_full_size_sampled,
                             test_window_lengths_two_to_forty)

pytestmark = pytest.mark.gpu


# (uniform-sphere column, Gaussian-ball column)
@pytest.fixture(autouse=True, params=[(64, 256), (1, 128)], ids=["wave64-gauss256", "shared132-gauss128"])
def shared_column(request):
    from paper_2412_03898_amd import binding
    keys = (binding.SB_TUNE_FWD_COLUMN, binding.SB_TUNE_FWD_GAUSS_COLUMN)
    saved = [binding.tune_get(k) for k in keys]
    for k, v in zip(keys, request.param):
        binding.tune(k, v)
    try:
        yield
    finally:
        for k, v in zip(keys, saved):
            binding.tune(k, v)
