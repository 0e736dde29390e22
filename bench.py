#!/usr/bin/env python3
"""Benchmark of one iterative-reconstruction step of the point-cloud
photoacoustic operator on one MI355X.

A step is the whole hot path on one batch of synthetic input already resident
in HBM: forward (the radiator applied to every ball, sensor and frame), L2
loss, adjoint (gradient with respect to every ball attribute and deformation
coefficient) and the Adam update of every parameter group.  The default
workload is the single-frame vessel scene at scale: 200,000 balls along a
seeded branching vessel tree in a 40 mm cube, 1,024 sensors on a 100 mm
Fibonacci hemisphere, 4,096 samples at 40 MHz.

Prints ONE JSON line.  `value` is ball*sensor*frame pairs per second through
forward + adjoint (GPairs/s).  The roofline object reports the dominant kernel
in vector-ALU lane operations against the chip's lane-operation peak (the path has no dense contraction and its
DRAM traffic is small next to its arithmetic), counting the closed forms the
kernels evaluate, with the direct per-sample evaluation beside it; the cpu_baseline object times
the FP64 CPU oracle on the host cores over the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Vector-ALU peak in lane operations (an FMA counts once; packed FP32 is switched
# off at compile time): 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12      # 39.32 T lane-ops/s

# Learning rates of Sec. 3.2 (coordinates, peak pressure, size, deformation).
LR_POS, LR_P, LR_R, LR_DEF = 5e-7, 5e-4, 5e-7, 5e-6
# projection of the updates (as in the IR loop): peak pressure >= 0, size >= 1 um
LO = {"pos": -float("inf"), "R": 1e-6, "P": 0.0, "def": -float("inf")}


def workloads():
    from paper_2412_03898_amd import synth
    return {
        "vessel-single-frame": lambda: synth.workload_vessel_static(),
        "plain-single-frame": lambda: synth.workload_plain(),
        "vessel-4d": lambda: synth.workload_vessel_4d(),
    }


# Algorithmic lane operations per pair of the closed forms the uniform-sphere
# kernels evaluate (counted from the formulas, not from the compiled code):
#   geometry (both kernels): 40 -- FP64 distance with its refinement, window start,
#     fraction, 1/r, validity;
#   forward window: 42 -- five sample values of the window (sample 0, the ramp's first
#     value and step, the two end samples; shift, clamp, square, difference, scale and
#     round: 25), the seven second differences (10 integer operations), the seven tile
#     additions (7);
#   adjoint window: 36 -- boundary count (4), prefix differences T0 and T1 (4), the
#     closed-form sums S_t, S_w, S_r (13), the pair's contributions to dL/dr, dL/dR,
#     dL/dP and the direction (15).
# The flush (running sums, scale and one atomic per touched sample) and the residual
# row staging are not counted.
FWD_PAIR_OPS = 40 + 42
ADJ_PAIR_OPS = 40 + 36


def op_model(wl):
    """Lane operations of one forward and one adjoint launch.

    `forward` / `adjoint`: the closed forms the kernels evaluate (FWD_PAIR_OPS,
    ADJ_PAIR_OPS per pair) for the uniform sphere.  `direct_forward` /
    `direct_adjoint`: the direct evaluation of the method per sample -- 40 for the FP64
    pair geometry in each kernel, 8 per sample in the forward (clamp, square,
    difference, scale, accumulate) and 14 per sample in the adjoint (residual
    difference and the three weighted sums) over a window of W samples (W = floor(2
    R_f/delta) + 2); the closed forms execute fewer operations than this count, so it
    can exceed the peak.  The Gaussian ball has no closed form: both models are the
    direct one.
    """
    import numpy as np
    delta = wl.c / wl.fs
    S = wl.n_sensors
    bo, fo = wl.ball_offset, wl.frame_offset
    sumW = 0.0
    pairs = 0
    for i in range(len(bo) - 1):
        R = wl.balls[3, bo[i]:bo[i + 1]].astype(np.float64)
        for f in range(fo[i], fo[i + 1]):
            Rf = R
            if wl.basis == 1 and wl.deform is not None:
                t = float(wl.frame_t[f])
                D = wl.deform[3, :, bo[i]:bo[i + 1]].astype(np.float64)
                h = sum(D[2 * (k - 1)] * np.cos(2 * np.pi * k * t) + D[2 * (k - 1) + 1] * np.sin(2 * np.pi * k * t)
                        for k in range(1, wl.n_terms + 1))
                Rf = R * (1.0 + h)
            W = np.floor(2.0 * Rf / delta) + 2.0
            sumW += float(W.sum()) * S
            pairs += len(R) * S
    dfwd = 40.0 * pairs + 8.0 * sumW
    dadj = 40.0 * pairs + 14.0 * sumW
    closed = wl.kernel == 0
    return {"forward": FWD_PAIR_OPS * pairs if closed else dfwd,
            "adjoint": ADJ_PAIR_OPS * pairs if closed else dadj,
            "direct_forward": dfwd, "direct_adjoint": dadj,
            "pairs": pairs, "mean_window": sumW / max(pairs, 1)}


def _fourier_frames(wl, balls_np, deform_np):
    """Per-frame static scenes of a Fourier-deformed scene (Eq. 1 with the Fourier
    series; additive position), materialised in FP64 and stored as FP32: the input of
    the frame-by-frame comparison path."""
    import numpy as np
    out = []
    b = balls_np.astype(np.float64)
    D = deform_np.astype(np.float64)
    for f in range(wl.n_frames):
        t = float(wl.frame_t[f])
        h = sum(D[:, 2 * (k - 1)] * np.cos(2 * np.pi * k * t) + D[:, 2 * (k - 1) + 1] * np.sin(2 * np.pi * k * t)
                for k in range(1, wl.n_terms + 1))
        x = b.copy()
        x[0:3] += h[0:3]
        x[3:5] *= 1.0 + h[3:5]
        out.append(np.ascontiguousarray(x.astype(np.float32)))
    return out


def ir_4d_comparison(steps, warmup):
    """ms per IR iteration on the 4D vessel scene (50,000 balls, 16 frames, 512 sensors,
    2,048 samples): all frames batched in one forward and one adjoint launch (25 parameters
    per ball), against the frame-by-frame path (16 independent static scenes, one forward,
    loss, adjoint and Adam each per iteration), with the peak device memory of each."""
    import numpy as np
    import torch
    from paper_2412_03898_amd import ops, synth, tune
    from paper_2412_03898_amd.binding import Problem

    wl = synth.workload_vessel_4d()
    pb, balls, deform, ft, sens = ops.to_device(wl, "cuda:0")
    balls, deform, _ = ops.apply_order(pb, balls, deform)
    choice = tune.autotune(pb, balls, deform, ft, sens, cache=None)
    pert = torch.from_numpy(synth.perturbed(balls.cpu().numpy(), 1)).cuda()
    pert, pert_def, _ = ops.apply_order(pb, pert, deform)
    d = ops.forward(pb, pert, pert_def, ft, sens)
    del pert, pert_def

    def run(step_fn):
        for _ in range(warmup):
            step_fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            step_fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps * 1e3

    # batched 4D step
    torch.cuda.reset_peak_memory_stats()
    y = torch.empty_like(d)
    r = torch.empty_like(d)
    L = torch.empty((), dtype=torch.float64, device="cuda")
    gb = torch.empty_like(balls)
    gd = torch.empty_like(deform)
    groups = [(balls[0:3], gb[0:3], LR_POS, LO["pos"]), (balls[3], gb[3], LR_R, LO["R"]),
              (balls[4], gb[4], LR_P, LO["P"]), (deform, gd, LR_DEF, LO["def"])]
    state = [(torch.zeros_like(p), torch.zeros_like(p)) for p, _, _, _ in groups]
    it = [0]

    def batched():
        ops.forward(pb, balls, deform, ft, sens, out=y)
        ops.loss(pb, y, d, residual=r, loss_out=L)
        ops.adjoint(pb, balls, deform, ft, sens, r, grad_balls=gb, grad_deform=gd)
        it[0] += 1
        for (p, g, lr, lo), (m, v) in zip(groups, state):
            ops.adam_(p, g, m, v, lr, it[0], lo=lo)

    ms_batched = run(batched)
    mem_batched = torch.cuda.max_memory_allocated() / 2**20
    ops.check()
    del y, r, gb, gd, state

    # frame-by-frame path: each frame is its own static scene
    frames_np = _fourier_frames(wl, balls.cpu().numpy(), deform.cpu().numpy())
    B = wl.n_balls
    pf = Problem(wl.kernel, 0, 0, 0, wl.n_sensors, wl.n_samples, wl.c, wl.fs, wl.t0,
                 np.array([0, B]), np.array([0, 1]))
    t0 = torch.zeros(1, dtype=torch.float32, device="cuda")
    torch.cuda.reset_peak_memory_stats()
    fb = [torch.from_numpy(x).cuda() for x in frames_np]
    fy = torch.empty((1, wl.n_sensors, wl.n_samples), dtype=torch.float32, device="cuda")
    fr = torch.empty_like(fy)
    fL = torch.empty((), dtype=torch.float64, device="cuda")
    fg = [torch.empty_like(x) for x in fb]
    fstate = [[(torch.zeros_like(x[0:3]), torch.zeros_like(x[0:3])), (torch.zeros_like(x[3]), torch.zeros_like(x[3])),
               (torch.zeros_like(x[4]), torch.zeros_like(x[4]))] for x in fb]
    fit = [0]

    def per_frame():
        fit[0] += 1
        for f in range(wl.n_frames):
            ops.forward(pf, fb[f], None, t0, sens, out=fy)
            ops.loss(pf, fy, d[f:f + 1], residual=fr, loss_out=fL)
            ops.adjoint(pf, fb[f], None, t0, sens, fr, grad_balls=fg[f])
            x, g = fb[f], fg[f]
            for (p, gg, lr, lo), (m, v) in zip(((x[0:3], g[0:3], LR_POS, LO["pos"]), (x[3], g[3], LR_R, LO["R"]),
                                                (x[4], g[4], LR_P, LO["P"])), fstate[f]):
                ops.adam_(p, gg, m, v, lr, fit[0], lo=lo)

    ms_frames = run(per_frame)
    mem_frames = torch.cuda.max_memory_allocated() / 2**20
    ops.check()
    pairs = pb.pairs()
    return {"workload": wl.name, "balls": wl.n_balls, "frames": wl.n_frames, "sensors": wl.n_sensors,
            "samples": wl.n_samples, "tuning": list(choice),
            "batched_ms_per_iter": round(ms_batched, 3), "per_frame_ms_per_iter": round(ms_frames, 3),
            "speedup": round(ms_frames / ms_batched, 3),
            "batched_gpairs_s": round(pairs / ms_batched / 1e6, 3),
            "per_frame_gpairs_s": round(pairs / ms_frames / 1e6, 3),
            "peak_mem_mb_batched": round(mem_batched, 1), "peak_mem_mb_per_frame": round(mem_frames, 1)}


def uneven_batch_timing(steps, warmup):
    """GPairs/s of forward + adjoint on the uneven batch: 8 independent 4D vessel scenes
    (ball counts log-uniform in 1e4..4e5, 4, 8, 16 or 32 frames each, Fourier K = 2)
    sharing one 1,024-sensor hemisphere, 4,096 samples, in one forward and one adjoint
    launch per step (with loss and Adam)."""
    import torch
    from paper_2412_03898_amd import ops, synth, tune
    wl = synth.workload_uneven_batch()
    pb, balls, deform, ft, sens = ops.to_device(wl, "cuda:0")
    balls, deform, _ = ops.apply_order(pb, balls, deform)
    choice = tune.autotune(pb, balls, deform, ft, sens, cache=None)
    pert = torch.from_numpy(synth.perturbed(balls.cpu().numpy(), 1)).cuda()
    d = ops.forward(pb, pert, deform, ft, sens)
    del pert
    y, r = torch.empty_like(d), torch.empty_like(d)
    L = torch.empty((), dtype=torch.float64, device="cuda")
    gb, gd = torch.empty_like(balls), torch.empty_like(deform)
    groups = [(balls[0:3], gb[0:3], LR_POS, LO["pos"]), (balls[3], gb[3], LR_R, LO["R"]),
              (balls[4], gb[4], LR_P, LO["P"]), (deform, gd, LR_DEF, LO["def"])]
    state = [(torch.zeros_like(p), torch.zeros_like(p)) for p, _, _, _ in groups]
    it = [0]

    def step():
        ops.forward(pb, balls, deform, ft, sens, out=y)
        ops.loss(pb, y, d, residual=r, loss_out=L)
        ops.adjoint(pb, balls, deform, ft, sens, r, grad_balls=gb, grad_deform=gd)
        it[0] += 1
        for (p, g, lr, lo), (m, v) in zip(groups, state):
            ops.adam_(p, g, m, v, lr, it[0], lo=lo)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) / steps * 1e3
    flags = ops.check()
    pairs = pb.pairs()
    return {"workload": wl.name, "scenes": len(wl.ball_offset) - 1, "balls": wl.n_balls,
            "frames": wl.n_frames, "sensors": wl.n_sensors, "samples": wl.n_samples,
            "pairs_per_pass": pairs, "tuning": list(choice), "ms_per_step": round(ms, 3),
            "gpairs_s": round(pairs / (ms * 1e-3) / 1e9, 3), "device_flags": flags}


def voxel_map_timing(pb, balls, deform, reps=5):
    """Point cloud -> voxel grid -> maximum amplitude projections for the bench scene:
    a 40 mm cube of 0.1 mm voxels (400^3, 256 MB) at frame time 0; mean ms of
    slingbag_voxelize and of slingbag_map (all three projections)."""
    import torch
    from paper_2412_03898_amd import ops
    g = (400, 400, 400, -0.01995, -0.01995, -0.01995, 0.1e-3)
    vol = ops.voxelize(pb, balls, deform, 0.0, g)
    ops.map_projections(vol)
    ops.check()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for _ in range(reps):
        ops.voxelize(pb, balls, deform, 0.0, g, out=vol)
    e[1].record()
    for _ in range(reps):
        ops.map_projections(vol)
    e[2].record()
    torch.cuda.synchronize()
    ops.check()
    tv, tm = e[0].elapsed_time(e[1]) / reps, e[1].elapsed_time(e[2]) / reps
    nvox = 400 ** 3
    del vol
    return {"grid": [400, 400, 400], "pitch_mm": 0.1, "balls": int(balls.shape[1]),
            "voxelize_ms": round(tv, 3), "map_ms": round(tm, 3),
            "map_read_gb_s": round(3 * nvox * 4 / (tm * 1e-3) / 1e9, 1)}


def cpu_baseline(wl, d_np):
    """Time the FP64 oracle on the host: one forward, loss and adjoint of the same workload."""
    import numpy as np
    import oracle
    threads = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit():
        threads = min(threads, int(omp))
    t = time.perf_counter()
    y = oracle.forward(wl, n_threads=threads)
    _, r = oracle.loss(y, d_np)
    oracle.adjoint(wl, r, n_threads=threads)
    dt = time.perf_counter() - t
    pairs = wl.pairs()
    return {"value": pairs / dt / 1e9, "unit": "GPairs/s", "cores": threads, "kind": "oracle",
            "sample": f"full workload, one forward + loss + adjoint in FP64 ({pairs:.3e} pairs, "
                      f"{dt:.1f} s on {threads} threads)",
            "seconds": dt}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="vessel-single-frame", choices=sorted(workloads()))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-4d", action="store_true", help="skip the 4D batched vs per-frame comparison")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven 8-scene batch timing")
    ap.add_argument("--no-voxel", action="store_true", help="skip the voxel grid / MAP timing")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with a 1 GiB device-to-device copy (a known amount of HBM traffic for "
                         "scaling memory counters)")
    ap.add_argument("--no-graph", action="store_true", help="skip the captured-graph step timing")
    ap.add_argument("--tuning", default=None,
                    help="fix the kernel knobs as COLUMN,OCCUPANCY,ITEMS instead of autotuning")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2412_03898_amd import binding, ops, synth

    torch.cuda.set_device(0)
    wl = workloads()[args.workload]()
    pb, balls, deform, ft, sens = ops.to_device(wl, "cuda:0")
    # ball order (performance only): Morton order computed on the GPU, as an IR loop
    # does once and then every few iterations
    balls, deform, _ = ops.apply_order(pb, balls, deform)
    # kernel knobs for this shape (timed once, outside the measured steps)
    from paper_2412_03898_amd import tune
    if args.tuning:
        choice = tuple(int(v) for v in args.tuning.split(","))
        tune.apply(choice)
    else:
        choice = tune.autotune(pb, balls, deform, ft, sens, cache=None)
    torch.cuda.synchronize()
    # measured data: the operator applied to a perturbed copy of the scene
    pert = torch.from_numpy(synth.perturbed(balls.cpu().numpy(), 1)).cuda()
    pert, pert_def, _ = ops.apply_order(pb, pert, deform)
    d = ops.forward(pb, pert, pert_def, ft, sens)
    y = torch.empty_like(d)
    r = torch.empty_like(d)
    L = torch.empty((), dtype=torch.float64, device="cuda")
    gb = torch.empty_like(balls)
    gd = torch.empty_like(deform) if deform is not None else None
    groups = [(balls[0:3], gb[0:3], LR_POS, LO["pos"]), (balls[3], gb[3], LR_R, LO["R"]),
              (balls[4], gb[4], LR_P, LO["P"])]
    if deform is not None:
        groups.append((deform, gd, LR_DEF, LO["def"]))
    state = [(torch.zeros_like(p), torch.zeros_like(p)) for p, _, _, _ in groups]
    step_no = [0]

    def step():
        ops.forward(pb, balls, deform, ft, sens, out=y)
        ops.loss(pb, y, d, residual=r, loss_out=L)
        ops.adjoint(pb, balls, deform, ft, sens, r, grad_balls=gb, grad_deform=gd)
        step_no[0] += 1
        for (p, g, lr, lo), (m, v) in zip(groups, state):
            ops.adam_(p, g, m, v, lr, step_no[0], lo=lo)

    for _ in range(args.warmup):
        step()
    ops.check()
    torch.cuda.synchronize()
    binding.timing(True)
    binding.timing_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = binding.timing_read()
    binding.timing(False)
    flags = ops.check()

    # the same step replayed as a captured graph (forward + loss + adjoint) + Adam
    ms_graph = None
    graph = None if args.no_graph else ops.StepGraph(pb, balls, deform, ft, sens, d)
    if graph is not None:
        ggroups = [(balls[0:3], graph.grad_balls[0:3], LR_POS, LO["pos"]),
                   (balls[3], graph.grad_balls[3], LR_R, LO["R"]), (balls[4], graph.grad_balls[4], LR_P, LO["P"])]
        if deform is not None:
            ggroups.append((deform, graph.grad_deform, LR_DEF, LO["def"]))

        def gstep():
            graph.run()
            step_no[0] += 1
            for (p, g, lr, lo), (m, v) in zip(ggroups, state):
                ops.adam_(p, g, m, v, lr, step_no[0], lo=lo)

        for _ in range(args.warmup):
            gstep()
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(args.steps):
            gstep()
        torch.cuda.synchronize()
        ms_graph = (time.perf_counter() - tg) / args.steps * 1e3
        graph.close()
        ops.check()

    pairs = pb.pairs()
    ms_step = elapsed / args.steps * 1e3
    value = pairs * args.steps / elapsed / 1e9
    fm = op_model(wl)
    per_kernel = {k: (ms / n if n else None) for k, (ms, n) in kt.items()}
    dom = max(("forward", "adjoint"), key=lambda k: per_kernel[k] or 0.0)
    achieved = fm[dom] / (per_kernel[dom] * 1e-3) / 1e12
    achieved_direct = fm["direct_" + dom] / (per_kernel[dom] * 1e-3) / 1e12
    # HBM bytes per launch of the dominant kernel from the committed rocprofv3 FETCH_SIZE /
    # WRITE_SIZE record of this workload and instance (null once its sources change)
    from paper_2412_03898_amd import profsum
    instance = (f"forward_kernel<4, 256, {choice[0]}, 0>" if dom == "forward"
                else f"adjoint_uniform_kernel<{4 if wl.basis == 1 and wl.n_terms == 2 else 0}, {choice[1]}>")
    traffic = profsum.traffic_for(instance, wl.name)
    out = {
        "metric": "GPairs/s fwd+adjoint (ball\u00b7sensor\u00b7frame) and ms/IR iteration vs per-frame path",
        "value": round(value, 4),
        "unit": "GPairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "balls": wl.n_balls, "sensors": wl.n_sensors,
                   "samples": wl.n_samples, "frames": wl.n_frames, "fs_hz": wl.fs,
                   "c_m_s": wl.c, "kernel": "uniform-sphere", "step": "forward+loss+adjoint+adam",
                   "ball_order": "morton",
                   "tuning": {"forward_column": choice[0], "adjoint_occupancy": choice[1],
                              "adjoint_items": choice[2]}},
        "roofline": {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3),
                     "peak": round(ALU_PEAK_TOPS, 2), "unit": "Tops/s",
                     "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": traffic, "traffic_unit": "B/launch",
                     "ops_per_launch": fm[dom], "mean_window": round(fm["mean_window"], 3),
                     "direct_model": {"ops_per_launch": fm["direct_" + dom],
                                      "achieved": round(achieved_direct, 3),
                                      "frac": round(achieved_direct / ALU_PEAK_TOPS, 4)}},
        "kernel_ms": {k: (round(v, 4) if v is not None else None) for k, v in per_kernel.items()},
        "graph_ms_per_step": None if ms_graph is None else round(ms_graph, 4),
        "device_flags": flags,
    }
    if not args.no_4d:
        out["ir_4d"] = ir_4d_comparison(max(3, args.steps // 4), 2)
    if not args.no_batch:
        out["uneven_batch"] = uneven_batch_timing(3, 1)
    if not args.no_voxel:
        out["voxel_map"] = voxel_map_timing(pb, balls, deform)
    if not args.no_cpu_baseline:
        # the oracle's timing does not depend on the measured values: zeros stand in for them
        d_np = np.zeros((wl.n_frames, wl.n_sensors, wl.n_samples))
        cb = cpu_baseline(wl, d_np)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
    print(json.dumps(out), flush=True)
    if args.copy_calibration:
        src = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
