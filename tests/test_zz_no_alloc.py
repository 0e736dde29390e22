"""GPU test of slingbag_loss_noalloc (the loss for callers that cannot allocate
device memory) through the C ABI: two calls in a row, the second on a smaller
input, each bit-identical to slingbag_loss on the same input and within FP32
rounding of the oracle's FP64 loss.  In a fresh process the no-alloc call comes
before any other call of the library, so it cannot lean on per-device buffers
that an earlier call allocated."""

import numpy as np
import pytest

import oracle
from paper_2412_03898_amd import binding
from paper_2412_03898_amd.binding import Problem

pytestmark = pytest.mark.gpu


def _problem(F, S, T):
    return Problem(0, 0, 0, 0, S, T, 1500.0, 40e6, 0.0, np.array([0, 10]), np.array([0, F]))


def _ptr(t):
    return t.data_ptr()


@pytest.mark.parametrize("shapes", [((3, 70, 1001), (1, 33, 517))])
def test_loss_noalloc_matches_loss_on_two_calls(shapes):
    import torch
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(21)
    for F, S, T in shapes:
        pb = _problem(F, S, T)
        y_np = rng.normal(0.0, 1.0, (F, S, T)).astype(np.float32)
        d_np = (y_np + rng.normal(0.0, 0.3, (F, S, T))).astype(np.float32)
        y, d = torch.from_numpy(y_np).cuda(), torch.from_numpy(d_np).cuda()
        r_na = torch.full_like(y, np.nan)
        L_na = torch.full((), np.nan, dtype=torch.float64, device="cuda")
        print(f"loss_noalloc F={F} S={S} T={T}", flush=True)
        binding.loss_noalloc(pb, _ptr(y), _ptr(d), _ptr(r_na), _ptr(L_na), stream)
        torch.cuda.synchronize()
        r_ref = torch.full_like(y, np.nan)
        L_ref = torch.full((), np.nan, dtype=torch.float64, device="cuda")
        binding.loss(pb, _ptr(y), _ptr(d), _ptr(r_ref), _ptr(L_ref), stream)
        torch.cuda.synchronize()
        # same kernels, same fixed reduction order: bit-identical
        assert torch.equal(r_na, r_ref)
        assert L_na.item() == L_ref.item()
        # and the loss itself against the oracle's FP64 definition (the GPU rounds each
        # residual to FP32 before squaring: relative error of order 1e-8)
        L_or, r_or = oracle.loss(y_np, d_np)
        assert abs(L_na.item() - L_or) <= 1e-6 * L_or
        assert np.max(np.abs(r_na.cpu().numpy() - r_or)) <= 1e-6 * np.max(np.abs(r_or))


def test_loss_noalloc_rejects_bad_arguments():
    import torch
    pb = _problem(1, 4, 16)
    L = torch.zeros((), dtype=torch.float64, device="cuda")
    with pytest.raises(binding.SlingbagError) as e:
        binding.loss_noalloc(pb, None, None, None, _ptr(L), 0)
    assert e.value.status == binding.SB_ERR_INVALID_ARG
