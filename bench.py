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
against the chip's vector-ALU peak (the path has no dense contraction and its
DRAM traffic is small next to its arithmetic); the cpu_baseline object times
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

# Vector-ALU peak without packed FP32 (packed FP32 is not generated in this
# build): 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP per FMA x 2.4 GHz.
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12      # 78.64

# Learning rates of Sec. 3.2 (coordinates, peak pressure, size, deformation).
LR_POS, LR_P, LR_R, LR_DEF = 5e-7, 5e-4, 5e-7, 5e-6


def workloads():
    from paper_2412_03898_amd import synth
    return {
        "vessel-single-frame": lambda: synth.workload_vessel_static(),
        "plain-single-frame": lambda: synth.workload_plain(),
        "vessel-4d": lambda: synth.workload_vessel_4d(),
    }


def flop_model(wl):
    """Algorithmic FLOPs of one forward and one adjoint launch (FMA = 2).

    Per (ball, sensor, frame) pair with a window of W samples (W = floor(2 R_f/delta) + 2
    for the uniform sphere): geometry 16 FLOP; forward 7 FLOP per sample; adjoint
    13 FLOP per window boundary (W + 1 of them) plus 20 to form the five
    per-pair derivatives.
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
    fwd = 16.0 * pairs + 7.0 * sumW
    adj = 16.0 * pairs + 13.0 * (sumW + pairs) + 20.0 * pairs
    return {"forward": fwd, "adjoint": adj, "pairs": pairs, "mean_window": sumW / max(pairs, 1)}


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
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the operator has no multi-GPU path in this build "
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
    choice = tune.autotune(pb, balls, deform, ft, sens, cache=None)
    torch.cuda.synchronize()
    # measured data: the operator applied to a perturbed copy of the scene
    pert = torch.from_numpy(synth.perturbed(balls.cpu().numpy(), 1)).cuda()
    d = ops.forward(pb, pert, deform, ft, sens)
    y = torch.empty_like(d)
    r = torch.empty_like(d)
    L = torch.empty((), dtype=torch.float64, device="cuda")
    gb = torch.empty_like(balls)
    gd = torch.empty_like(deform) if deform is not None else None
    groups = [(balls[0:3], gb[0:3], LR_POS), (balls[3], gb[3], LR_R), (balls[4], gb[4], LR_P)]
    if deform is not None:
        groups.append((deform, gd, LR_DEF))
    state = [(torch.zeros_like(p), torch.zeros_like(p)) for p, _, _ in groups]
    step_no = [0]

    def step():
        ops.forward(pb, balls, deform, ft, sens, out=y)
        ops.loss(pb, y, d, residual=r, loss_out=L)
        ops.adjoint(pb, balls, deform, ft, sens, r, grad_balls=gb, grad_deform=gd)
        step_no[0] += 1
        for (p, g, lr), (m, v) in zip(groups, state):
            ops.adam_(p, g, m, v, lr, step_no[0])

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

    pairs = pb.pairs()
    ms_step = elapsed / args.steps * 1e3
    value = pairs * args.steps / elapsed / 1e9
    fm = flop_model(wl)
    per_kernel = {k: (ms / n if n else None) for k, (ms, n) in kt.items()}
    dom = max(("forward", "adjoint"), key=lambda k: per_kernel[k] or 0.0)
    achieved = fm[dom] / (per_kernel[dom] * 1e-3) / 1e12
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
                     "peak": round(ALU_PEAK_TFLOPS, 2), "unit": "TFLOP/s",
                     "frac": round(achieved / ALU_PEAK_TFLOPS, 4), "traffic": None,
                     "flop_per_launch": fm[dom], "mean_window": round(fm["mean_window"], 3)},
        "kernel_ms": {k: (round(v, 4) if v is not None else None) for k, v in per_kernel.items()},
        "device_flags": flags,
    }
    if not args.no_cpu_baseline:
        # the oracle's timing does not depend on the measured values: zeros stand in for them
        d_np = np.zeros((wl.n_frames, wl.n_sensors, wl.n_samples))
        cb = cpu_baseline(wl, d_np)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
