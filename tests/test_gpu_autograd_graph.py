"""GPU: the torch.autograd wrapper and the captured-graph IR step, against the oracle."""

import numpy as np
import pytest

import oracle
from helpers import rel_l2, with_
from paper_2412_03898_amd import synth

pytestmark = pytest.mark.gpu


def _scene():
    return synth.apply_order(synth.workload_vessel_4d(n_balls=2500, n_sensors=70, n_frames=6))


def test_autograd_gradient_matches_oracle():
    import torch
    from paper_2412_03898_amd import ops
    from paper_2412_03898_amd.autograd import l2_loss, radiate
    wl = _scene()
    pb, balls, deform, ft, sens = ops.to_device(wl)
    d_np = oracle.forward(wl, balls=synth.perturbed(wl.balls, 3)).astype(np.float32)
    d = torch.from_numpy(d_np).cuda()
    b = balls.clone().requires_grad_(True)
    D = deform.clone().requires_grad_(True)
    L = l2_loss(pb, radiate(pb, b, D, ft, sens), d)
    L.backward()
    y_ref = oracle.forward(wl)
    L_ref, r_ref = oracle.loss(y_ref, d_np)
    gb_ref, gd_ref = oracle.adjoint(wl, r_ref)
    assert float(L.item()) == pytest.approx(L_ref, rel=2e-5)
    g = b.grad.cpu().numpy()
    assert rel_l2(g[0:3], gb_ref[0:3]) <= 1e-4
    assert rel_l2(g[3], gb_ref[3]) <= 1e-4
    assert rel_l2(g[4], gb_ref[4]) <= 1e-4
    gd = D.grad.cpu().numpy()
    for a in range(5):
        assert rel_l2(gd[a], gd_ref[a]) <= 1e-4, a


def test_autograd_matches_finite_differences_of_oracle_loss():
    """<grad, v> from the GPU autograd gradient against central differences of the FP64
    oracle loss, along random directions and for single deformation coefficients."""
    import torch
    from paper_2412_03898_amd import ops
    from paper_2412_03898_amd.autograd import l2_loss, radiate
    wl = _scene()
    pb, balls, deform, ft, sens = ops.to_device(wl)
    d_np = oracle.forward(wl, balls=synth.perturbed(wl.balls, 4)).astype(np.float32)
    d = torch.from_numpy(d_np).cuda()
    b = balls.clone().requires_grad_(True)
    D = deform.clone().requires_grad_(True)
    l2_loss(pb, radiate(pb, b, D, ft, sens), d).backward()
    gb = b.grad.cpu().numpy().astype(np.float64)
    gd = D.grad.cpu().numpy().astype(np.float64)
    B0 = wl.balls.astype(np.float64)
    D0 = wl.deform.astype(np.float64)

    def L(bb, dd):
        y = oracle.forward(wl, balls=bb, deform=dd)
        return 0.5 * float(((y - d_np) ** 2).sum())

    rng = np.random.default_rng(11)
    for trial in range(2):
        vb = rng.normal(size=B0.shape) * np.array([1e-6, 1e-6, 1e-6, 1e-6, 1e-3])[:, None]
        vd = rng.normal(size=D0.shape) * np.array([1e-6, 1e-6, 1e-6, 1e-3, 1e-3])[:, None, None]
        # steps of ~1e-12 m: small enough that no ball edge crosses a sample boundary inside
        # the difference (the loss has kinks there), large enough for FP64
        eps = 1e-6
        fd = (L(B0 + eps * vb, D0 + eps * vd) - L(B0 - eps * vb, D0 - eps * vd)) / (2 * eps)
        an = float((gb * vb).sum() + (gd * vd).sum())
        assert an == pytest.approx(fd, rel=1e-4), trial
    # single coefficients: the largest-gradient entries of the position and pressure groups
    for a in (0, 4):
        m, bi = np.unravel_index(np.argmax(np.abs(gd[a])), gd[a].shape)
        e = 1e-12 if a < 3 else 1e-9
        Dp, Dm = D0.copy(), D0.copy()
        Dp[a, m, bi] += e
        Dm[a, m, bi] -= e
        fd = (L(B0, Dp) - L(B0, Dm)) / (2 * e)
        assert gd[a, m, bi] == pytest.approx(fd, rel=1e-3), (a, m, bi)


def test_graph_replays_match_eager():
    """Replay the captured forward+loss+adjoint several times, with eager work (an in-place
    parameter update) and synchronisations between replays; every replay equals the eager
    sequence on the same inputs."""
    import torch
    from paper_2412_03898_amd import ops
    wl = _scene()
    pb, balls, deform, ft, sens = ops.to_device(wl)
    d = torch.from_numpy(oracle.forward(wl, balls=synth.perturbed(wl.balls, 5)).astype(np.float32)).cuda()
    g = ops.StepGraph(pb, balls, deform, ft, sens, d)
    try:
        for rep in range(4):
            balls[0].add_(2e-6)            # eager work between replays, in place
            deform[4].mul_(0.99)
            torch.cuda.synchronize()
            Lg, gbg, gdg = g.run()
            torch.cuda.synchronize()
            Lg, gbg, gdg, yg = float(Lg.item()), gbg.clone(), gdg.clone(), g.signals.clone()
            y = ops.forward(pb, balls, deform, ft, sens)
            L, r = ops.loss(pb, y, d)
            gb, gd = ops.adjoint(pb, balls, deform, ft, sens, r)
            torch.cuda.synchronize()
            assert Lg == pytest.approx(float(L.item()), rel=1e-6), rep
            assert rel_l2(yg.cpu().numpy(), y.cpu().numpy()) <= 1e-6, rep
            assert rel_l2(gbg.cpu().numpy(), gb.cpu().numpy()) <= 1e-5, rep
            assert rel_l2(gdg.cpu().numpy(), gd.cpu().numpy()) <= 1e-5, rep
        ops.check()
        # and the last replay against the oracle
        wl2 = with_(wl, balls=balls.cpu().numpy(), deform=deform.cpu().numpy())
        assert rel_l2(g.signals.cpu().numpy(), oracle.forward(wl2)) <= 1e-5
    finally:
        g.close()


def test_graph_replays_on_uneven_batch_match_oracle():
    """The captured step on an uneven batch of three scenes (300 balls x 2 frames, an empty
    scene with 3 frames, 1,000 balls x 1 frame; Fourier deformation): four replays with an
    eager in-place parameter update and synchronisations between them, each replay's
    signals, loss and gradient groups against the oracle of the current parameters."""
    import sys
    import torch
    from helpers import tiny_scene
    from paper_2412_03898_amd import ops
    a = tiny_scene(n_balls=300, n_sensors=70, n_frames=2, basis=1, seed=171)
    b = tiny_scene(n_balls=1000, n_sensors=70, n_frames=1, basis=1, seed=172)
    wl = with_(a, balls=np.concatenate([a.balls, b.balls], axis=1),
               deform=np.concatenate([a.deform, b.deform], axis=2),
               frame_t=np.concatenate([a.frame_t, np.array([0.3, 0.7, 0.9], np.float32), b.frame_t]),
               ball_offset=np.array([0, 300, 300, 1300]), frame_offset=np.array([0, 2, 5, 6]))
    d_np = oracle.forward(wl, balls=synth.perturbed(wl.balls, 173)).astype(np.float32)
    pb, balls, deform, ft, sens = ops.to_device(wl)
    d = torch.from_numpy(d_np).cuda()
    g = ops.StepGraph(pb, balls, deform, ft, sens, d)
    try:
        for rep in range(4):
            print(f"[gpu-graph] uneven batch replay {rep}", flush=True)
            balls[4].mul_(1.0 + 0.01 * rep)        # eager work between replays, in place
            deform[0].add_(1e-6)
            torch.cuda.synchronize()
            Lg, gbg, gdg = g.run()
            torch.cuda.synchronize()
            assert ops.check() == 0
            cur = with_(wl, balls=balls.cpu().numpy(), deform=deform.cpu().numpy())
            y_ref = oracle.forward(cur)
            L_ref, r_ref = oracle.loss(y_ref, d_np)
            gb_ref, gd_ref = oracle.adjoint(cur, r_ref)
            y = g.signals.cpu().numpy()
            assert np.abs(y[2:5]).max() == 0.0, rep
            assert rel_l2(y, y_ref) <= 1e-5, rep
            assert float(Lg.item()) == pytest.approx(L_ref, rel=2e-5), rep
            gb, gd = gbg.cpu().numpy(), gdg.cpu().numpy()
            groups = [(gb[0:3], gb_ref[0:3]), (gb[3], gb_ref[3]), (gb[4], gb_ref[4])]
            groups += [(gd[k], gd_ref[k]) for k in range(5)]
            errs = [rel_l2(x, r) for x, r in groups]
            print(f"[gpu-graph] replay {rep}: grad rel-L2 max {max(errs):.2e}", flush=True)
            sys.stdout.flush()
            assert max(errs) <= 1e-4, (rep, errs)
    finally:
        g.close()


def test_graph_replays_are_timed():
    """A plan created with timing on times its forward, loss and adjoint at every replay
    (event nodes retargeted to fresh pool events per replay): one launch of each per
    replay, durations close to those of the same kernels called directly, and the
    replayed results unchanged by the timing nodes."""
    import torch
    from paper_2412_03898_amd import binding, ops
    # large enough that each kernel runs for about a tenth of a millisecond
    wl = synth.apply_order(synth.workload_vessel_4d(n_balls=20000, n_sensors=256, n_frames=4))
    pb, balls, deform, ft, sens = ops.to_device(wl)
    d = torch.zeros((pb.n_frames, 256, wl.n_samples), dtype=torch.float32, device="cuda")
    binding.timing(True)
    try:
        binding.timing_read()
        g = ops.StepGraph(pb, balls, deform, ft, sens, d)
        try:
            reps = 5
            for _ in range(reps):
                g.run()
            torch.cuda.synchronize()
            tg = binding.timing_read()
            for k in ("forward", "loss", "adjoint"):
                assert tg[k][1] == reps and tg[k][0] > 0.0, (k, tg[k])
            y = ops.forward(pb, balls, deform, ft, sens)
            L, r = ops.loss(pb, y, d)
            gb, gd = ops.adjoint(pb, balls, deform, ft, sens, r)
            for _ in range(reps - 1):
                ops.forward(pb, balls, deform, ft, sens, out=y)
                ops.adjoint(pb, balls, deform, ft, sens, r, grad_balls=gb, grad_deform=gd)
            torch.cuda.synchronize()
            te = binding.timing_read()
            for k in ("forward", "adjoint"):
                mg, me = tg[k][0] / tg[k][1], te[k][0] / te[k][1]
                print(f"[gpu-graph] {k}: replayed {mg * 1e3:.1f} us, direct {me * 1e3:.1f} us", flush=True)
                assert 0.5 * me <= mg <= 2.0 * me, (k, mg, me)
            assert float(g.loss.item()) == pytest.approx(float(L.item()), rel=1e-6)
            assert rel_l2(g.grad_balls.cpu().numpy(), gb.cpu().numpy()) <= 1e-5
            # timing off: replays record nothing
            binding.timing(False)
            g.run()
            torch.cuda.synchronize()
            assert all(n == 0 for _, n in binding.timing_read().values())
        finally:
            g.close()
    finally:
        binding.timing(False)
        ops.check()


def test_plan_keeps_its_chain_rule_buffer():
    """A plan of a deformation with the two-phase chain rule (Eq. 2) captures its own
    chain-rule buffer: a later, larger adjoint call, which replaces the per-device buffer,
    leaves the plan's replays correct (against the oracle)."""
    import torch
    from helpers import tiny_scene
    from paper_2412_03898_amd import ops
    wl = tiny_scene(n_balls=400, n_sensors=70, n_frames=3, basis=2, N=5, pos_mode=1, seed=181)
    d_np = oracle.forward(wl, balls=synth.perturbed(wl.balls, 182)).astype(np.float32)
    pb, balls, deform, ft, sens = ops.to_device(wl)
    g = ops.StepGraph(pb, balls, deform, ft, sens, torch.from_numpy(d_np).cuda())
    try:
        g.run()
        torch.cuda.synchronize()
        # a larger two-phase problem grows (reallocates) the per-device buffer
        big = tiny_scene(n_balls=3000, n_sensors=70, n_frames=6, basis=2, N=5, pos_mode=1, seed=183)
        pb2, b2, d2, ft2, s2 = ops.to_device(big)
        y2 = ops.forward(pb2, b2, d2, ft2, s2)
        ops.adjoint(pb2, b2, d2, ft2, s2, y2)
        torch.cuda.synchronize()
        print("[gpu-graph] replay after the per-device chain-rule buffer grew", flush=True)
        Lg, gbg, gdg = g.run()
        torch.cuda.synchronize()
        assert ops.check() == 0
        y_ref = oracle.forward(wl)
        L_ref, r_ref = oracle.loss(y_ref, d_np)
        gb_ref, gd_ref = oracle.adjoint(wl, r_ref)
        assert float(Lg.item()) == pytest.approx(L_ref, rel=2e-5)
        gb, gd = gbg.cpu().numpy(), gdg.cpu().numpy()
        for x, r in ((gb[0:3], gb_ref[0:3]), (gb[3], gb_ref[3]), (gb[4], gb_ref[4])):
            assert rel_l2(x, r) <= 1e-4
        for kind in range(3):
            for rows in (slice(0, 3), slice(3, 4), slice(4, 5)):
                assert rel_l2(gd[rows, kind::3], gd_ref[rows, kind::3]) <= 1e-4, (kind, rows)
    finally:
        g.close()
