"""Host-side logic of the IR loop (no GPU): the learning-rate schedule of Sec. 3.2."""

import pytest

from paper_2412_03898_amd import ir


def test_paper_learning_rates():
    # coordinates, peak pressure, size, deformation coefficients (Sec. 3.2)
    assert (ir.LR_POS, ir.LR_P, ir.LR_R, ir.LR_DEF) == (5e-7, 5e-4, 5e-7, 5e-6)
    assert (ir.DECAY_STEP, ir.DECAY_RATE) == (160, 0.1)


@pytest.mark.parametrize("it, factor", [(0, 1.0), (159, 1.0), (160, 0.1), (199, 0.1), (319, 0.1),
                                        (320, 0.01)])
def test_step_decay(it, factor):
    assert ir.step_decay(it) == pytest.approx(factor, rel=1e-12)
