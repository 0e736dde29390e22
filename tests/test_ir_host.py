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


def test_frame_sampler_epochs():
    """Each step draws distinct frames, each epoch (ceil(n/m) steps) visits every frame,
    and the draws are seeded and reproducible."""
    import math
    import numpy as np
    for n, m in ((7, 3), (8, 2), (5, 5), (6, 1)):
        s = ir.FrameSampler(n, m, seed=4)
        per_epoch = math.ceil(n / m)
        draws = [s.next() for _ in range(3 * per_epoch)]
        assert all(len(d) == m and len(set(d.tolist())) == m for d in draws)
        for e in range(3):
            seen = set(np.concatenate(draws[e * per_epoch:(e + 1) * per_epoch]).tolist())
            assert seen == set(range(n))
        t = ir.FrameSampler(n, m, seed=4)
        assert all(np.array_equal(d, t.next()) for d in draws)
    with pytest.raises(ValueError):
        ir.FrameSampler(4, 5)
