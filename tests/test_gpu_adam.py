"""GPU parity of the projected Adam step (slingbag_adam) against the oracle's FP64
textbook update, over several steps (bias corrections) and with bounds."""

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("lo, hi", [(-np.inf, np.inf), (0.0, np.inf), (-0.2, 0.3)])
def test_adam_matches_oracle(lo, hi):
    import torch
    from paper_2412_03898_amd import ops
    rng = np.random.default_rng(5)
    n = 100_003                                   # ragged against the launch grid
    p = rng.normal(0.0, 0.3, n).astype(np.float32)
    pt = torch.from_numpy(p).cuda()
    mt, vt = torch.zeros_like(pt), torch.zeros_like(pt)
    ref_p, ref_m, ref_v = p.astype(np.float64), np.zeros(n), np.zeros(n)
    lr = 1e-2
    lo32, hi32 = float(np.float32(lo)), float(np.float32(hi))     # the bounds as the ABI receives them
    for step in range(1, 6):
        g = rng.normal(0.0, 1.0, n).astype(np.float32) * (10.0 ** rng.uniform(-3, 1, n)).astype(np.float32)
        ops.adam_(pt, torch.from_numpy(g).cuda(), mt, vt, lr, step, lo=lo, hi=hi)
        # the C ABI takes the hyper-parameters in FP32: the oracle gets the same values
        ref_p, ref_m, ref_v = oracle.adam_step(ref_p, g, ref_m, ref_v, float(np.float32(lr)), step,
                                               beta1=float(np.float32(0.9)), beta2=float(np.float32(0.999)),
                                               eps=float(np.float32(1e-8)), lo=lo32, hi=hi32)
    got = pt.cpu().numpy().astype(np.float64)
    # FP32 state: each step moves p by at most lr (about); allow FP32 rounding of that
    assert np.max(np.abs(got - ref_p)) <= 1e-6 + 1e-5 * lr * 5
    assert np.all(got >= lo32) and np.all(got <= hi32)
    # moments in FP32: rounding relative to their magnitude (m cancels to ~0 for some entries)
    np.testing.assert_allclose(mt.cpu().numpy(), ref_m, rtol=1e-5, atol=1e-6 * np.abs(ref_m).max())
    np.testing.assert_allclose(vt.cpu().numpy(), ref_v, rtol=1e-5, atol=1e-6 * np.abs(ref_v).max())
