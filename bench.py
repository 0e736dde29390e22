#!/usr/bin/env python3
"""Benchmark of one iterative-reconstruction (IR) step of the 4D point-cloud
photoacoustic operator on one MI355X.

A step is the whole hot path on one batch of synthetic input already resident
in HBM: forward (every ball radiated into every sensor's samples at every
frame, the per-ball deformation recomputed), L2 loss, adjoint (gradient with
respect to every ball attribute and deformation coefficient) and the Adam
update of every parameter group with the learning rates of Sec. 3.2.  Forward,
loss and adjoint replay as one captured HIP graph; Adam is four launches.

The default workload is the large 4D IR scene: 1,000,000 balls along a seeded
branching vessel tree in a 40 mm cube, a 2-harmonic Fourier deformation
(additive position), 32 frames with t in [0, 1], 2,048 sensors on a 120 mm
Fibonacci hemisphere, 4,096 samples at 40 MHz; the measured data is the
forward of the ground-truth scene and the start has perturbed base attributes
and zero coefficients.

Prints ONE JSON line.  `value` is ball*sensor*frame pairs per second through
forward + adjoint (GPairs/s); `ms_per_step` the IR iteration.  Beside it:
  per_frame     the same iteration frame by frame (every frame an independent
                static scene with its own attributes), ms per iteration and
                peak device memory of both paths;
  roofline      the dominant kernel against the vector-ALU peak, counting the
                direct per-pair evaluation (40 lane operations of FP64 pair
                geometry plus 8 per window sample in the forward, 14 in the
                adjoint), with the issued-instruction and HBM figures of the
                committed rocprofv3 records;
  cpu_baseline  the FP64 oracle on the host cores, 1 thread and all cores,
                on one frame x every 32nd sensor of the same scene, with the
                GPU's outputs on exactly those rows checked against it;
  extras        the single-frame vessel scene, the small 4D scene (batched vs
                frame by frame), the uneven 8-scene batch, the small 4D scene with
                N = 1, 4, 13, 65 Gaussian bases per attribute (Eq. 2), and the
                voxel grid.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Vector-ALU peak in lane operations (an FMA counts once; packed FP32 is switched
# off at compile time; FP64 vector operations issue at the same rate):
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12      # 39.32 T lane-ops/s
HBM_PEAK_GBS = 8000.0

# Learning rates of Sec. 3.2 (coordinates, peak pressure, size, deformation).
LR_POS, LR_P, LR_R, LR_DEF = 5e-7, 5e-4, 5e-7, 5e-6
# projection of the updates (as in the IR loop): peak pressure >= 0, size >= 1 um
LO = {"pos": -float("inf"), "R": 1e-6, "P": 0.0, "def": -float("inf")}

METRIC = "GPairs/s fwd+adjoint (ball·sensor·frame) and ms/IR iteration vs per-frame path"


def workloads():
    from paper_2412_03898_amd import synth
    return {
        "vessel-4d-large": synth.workload_large_ir,
        "vessel-single-frame": synth.workload_vessel_static,
        "vessel-4d": synth.workload_vessel_4d,
        "uneven-4d-batch": synth.workload_uneven_batch,
        "plain-single-frame": synth.workload_plain,
    }


# Closed-form counts, context only: lane operations per pair of the formulas the
# uniform-sphere kernels evaluate (geometry 40 in each kernel; forward window 42: five
# sample values, seven second differences, seven tile additions; adjoint window 36:
# boundary count, two prefix differences, the sums S_t, S_w, S_r and the pair's four
# contributions).  The flush and the residual staging are not counted.
FWD_CLOSED_OPS = 40 + 42
ADJ_CLOSED_OPS = 40 + 36


def deformed_sizes(wl, balls_np, deform_np, f):
    """Deformed size R_f of every ball of a single scene at frame f (FP64)."""
    import numpy as np
    R = balls_np[3].astype(np.float64)
    if wl.basis != 1 or deform_np is None:
        return R
    t = float(wl.frame_t[f])
    D = deform_np[3].astype(np.float64)
    h = sum(D[2 * (k - 1)] * np.cos(2 * np.pi * k * t) + D[2 * (k - 1) + 1] * np.sin(2 * np.pi * k * t)
            for k in range(1, wl.n_terms + 1))
    return R * (1.0 + h)


def op_model(wl, balls_np, deform_np):
    """Lane operations of one forward and one adjoint launch.

    `forward` / `adjoint`: the direct per-sample evaluation of the method, per pair 40
    lane operations of FP64 geometry plus 8 per window sample (forward: shift, two
    clamps, two squares, difference, scale, accumulate) or 14 (adjoint: residual
    difference and the three weighted sums), over W = floor(2 R_f / delta) + 2 samples
    per pair with R_f the deformed size of each ball at each frame.  The uniform-sphere
    kernels evaluate closed forms that need fewer operations (`closed_*`), so the
    direct count divided by the time can exceed the peak: it measures the work done
    against the direct method, not the issue rate.
    """
    import numpy as np
    delta = wl.c / wl.fs
    S = wl.n_sensors
    bo, fo = wl.ball_offset, wl.frame_offset
    sumW, pairs = 0.0, 0
    for i in range(len(bo) - 1):
        sl = slice(int(bo[i]), int(bo[i + 1]))
        for f in range(int(fo[i]), int(fo[i + 1])):
            sub_b = balls_np[:, sl]
            sub_d = None if deform_np is None else deform_np[:, :, sl]
            Rf = deformed_sizes(wl, sub_b, sub_d, f)
            h = Rf / delta if wl.kernel == 0 else 6.0 * Rf / delta
            sumW += float((np.floor(2.0 * h) + 2.0).sum()) * S
            pairs += sub_b.shape[1] * S
    fwd, adj = 40.0 * pairs + 8.0 * sumW, 40.0 * pairs + 14.0 * sumW
    closed = wl.kernel == 0
    return {"forward": fwd, "adjoint": adj,
            "closed_forward": FWD_CLOSED_OPS * pairs if closed else fwd,
            "closed_adjoint": ADJ_CLOSED_OPS * pairs if closed else adj,
            "pairs": pairs, "mean_window": sumW / max(pairs, 1)}


class IRStep:
    """One IR step on device tensors: the captured forward + loss + adjoint graph
    (residual written over the signals) and one Adam launch per parameter group."""

    def __init__(self, pb, balls, deform, ft, sens, measured):
        from paper_2412_03898_amd import ops
        self.ops = ops
        self.graph = ops.StepGraph(pb, balls, deform, ft, sens, measured, in_place=True)
        gb, gd = self.graph.grad_balls, self.graph.grad_deform
        self.groups = [(balls[0:3], gb[0:3], LR_POS, LO["pos"]), (balls[3], gb[3], LR_R, LO["R"]),
                       (balls[4], gb[4], LR_P, LO["P"])]
        if deform is not None:
            self.groups.append((deform, gd, LR_DEF, LO["def"]))
        import torch
        self.state = [(torch.zeros_like(p), torch.zeros_like(p)) for p, _, _, _ in self.groups]
        self.n = 0

    def __call__(self):
        self.graph.run()
        self.n += 1
        for (p, g, lr, lo), (m, v) in zip(self.groups, self.state):
            self.ops.adam_(p, g, m, v, lr, self.n, lo=lo)

    def close(self):
        self.graph.close()


def timed_steps(step, steps, warmup):
    """(seconds for `steps` steps after `warmup` untimed ones, {kind: (total_ms, launches)})
    with the library's HIP-event timing of every launch inside the timed region."""
    import torch
    from paper_2412_03898_amd import binding, ops
    for _ in range(warmup):
        step()
    ops.check()
    torch.cuda.synchronize()
    binding.timing_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return elapsed, binding.timing_read()


def setup_scene(wl, tuning=None):
    """Device tensors of a single-scene or batch workload in Morton order, the kernel knobs
    (autotuned on the start unless given), the measured data and the start of the
    reconstruction.

    4D scenes: measured = forward of the ground-truth scene; start = the ground truth
    with perturbed base attributes and zero deformation coefficients.  Static scenes:
    measured = forward of a perturbed copy; start = the scene itself."""
    import torch
    from paper_2412_03898_amd import binding, ops, synth, tune
    pb, balls, deform, ft, sens = ops.to_device(wl, "cuda:0")
    balls, deform, _ = ops.apply_order(pb, balls, deform)
    if deform is not None:
        measured = ops.forward(pb, balls, deform, ft, sens)
        start = torch.from_numpy(synth.perturbed(balls.cpu().numpy(), 10)).cuda()
        gt = (balls.cpu().numpy(), deform.cpu().numpy())
        del balls
        balls = start
        if wl.basis == 2:
            # Eq. 2 from H = 0: every weight zero, the centres and widths kept
            deform = deform.clone()
            deform[:, 0::3] = 0.0
        else:
            deform = torch.zeros_like(deform)
    else:
        pert = torch.from_numpy(synth.perturbed(balls.cpu().numpy(), 1)).cuda()
        measured = ops.forward(pb, pert, None, ft, sens)
        gt = (pert.cpu().numpy(), None)
        del pert
    # kernel knobs for the state that is timed (the start), not for the ground truth
    if tuning:
        choice = tuple(int(v) for v in tuning)
        tune.apply(choice)
    else:
        choice = tune.autotune(pb, balls, deform, ft, sens, cache=None)
    ops.check()
    torch.cuda.synchronize()
    binding.timing_read()
    return pb, balls, deform, ft, sens, measured, choice, gt


def rel_l2(a, b):
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def oracle_leg(wl, pb, balls, deform, ft, sens, gt, s_step, frames, all_threads):
    """The FP64 oracle on a bounded sample of the workload: the frames `frames` and every
    s_step-th sensor, with the current (start) parameters.  It computes the sample's
    measured rows itself (forward of the ground truth), then one forward + loss +
    adjoint, timed with all threads and with one.  On the GPU, the full forward's rows
    of the sample are compared with the oracle's, and the full adjoint with the
    oracle's FP32-rounded residual on those rows (zero elsewhere) with the oracle's
    gradient of the sample (per group: positions, size, pressure, each coefficient
    attribute)."""
    import numpy as np
    import torch
    import oracle
    from paper_2412_03898_amd import ops
    f_idx = np.asarray(frames, dtype=np.int64)
    s_idx = np.arange(0, wl.n_sensors, s_step)
    import dataclasses
    sub = dataclasses.replace(wl, sensors=wl.sensors[:, s_idx].copy(), frame_t=wl.frame_t[f_idx].copy(),
                              frame_offset=np.array([0, len(f_idx)], dtype=np.int64),
                              balls=balls.cpu().numpy(),
                              deform=None if deform is None else deform.cpu().numpy())
    # the sample's measured rows, from the oracle (never from the GPU)
    d_sub = oracle.forward(sub, balls=gt[0], deform=gt[1], n_threads=all_threads)

    def one(threads):
        t = time.perf_counter()
        y = oracle.forward(sub, n_threads=threads)
        L, r = oracle.loss(y, d_sub)
        g = oracle.adjoint(sub, r, n_threads=threads)
        return time.perf_counter() - t, y, L, r, g

    t_all, y_ref, L_ref, r_ref, g_ref = one(all_threads)
    t_one = one(1)[0]
    pairs_sub = wl.n_balls * len(s_idx) * len(f_idx)
    # GPU rows of the same sample
    y = ops.forward(pb, balls, deform, ft, sens)
    fi = torch.from_numpy(f_idx).cuda()[:, None]
    si = torch.from_numpy(s_idx).cuda()[None, :]
    e_sig = rel_l2(y[fi, si].cpu().numpy(), y_ref)
    y.zero_()
    y[fi, si] = torch.from_numpy(r_ref.astype(np.float32)).cuda()
    gb, gd = ops.adjoint(pb, balls, deform, ft, sens, y)
    ops.check()
    gb, gd = gb.cpu().numpy(), None if gd is None else gd.cpu().numpy()
    del y
    torch.cuda.empty_cache()
    groups = [("xyz", gb[0:3], g_ref[0][0:3]), ("R", gb[3], g_ref[0][3]), ("P", gb[4], g_ref[0][4])]
    if gd is not None:
        groups += [(f"coef_{'xyzRP'[a]}", gd[a], g_ref[1][a]) for a in range(5)]
    e_grad = {k: rel_l2(a, b) for k, a, b in groups}
    parity = {"signal_rel_l2": e_sig, "signal_tol": 1e-5, "grad_rel_l2": e_grad, "grad_tol": 1e-4,
              "ok": bool(e_sig <= 1e-5 and max(e_grad.values()) <= 1e-4)}
    full_pairs = pb.pairs()
    return {
        "value": round(pairs_sub / t_all / 1e9, 6), "unit": "GPairs/s", "cores": all_threads, "kind": "oracle",
        "sample": (f"{len(f_idx)} frame(s) x every {s_step}th sensor ({len(s_idx)} sensors) x all "
                   f"{wl.n_balls} balls: {pairs_sub:.3e} pairs, one forward + loss + adjoint in FP64"),
        "cpu_model": cpu_model(),
        "seconds_all_cores": round(t_all, 3), "seconds_1_thread": round(t_one, 3),
        "gpairs_s_1_thread": round(pairs_sub / t_one / 1e9, 6),
        "extrapolated_full_iteration_s": {"all_cores": round(t_all * full_pairs / pairs_sub, 1),
                                          "1_thread": round(t_one * full_pairs / pairs_sub, 1)},
        "parity_on_sample": parity,
    }


def sq_and_traffic(instance, workload):
    """Committed rocprofv3 records of (kernel instance, workload): HBM bytes per launch
    and issued VALU instructions per launch (each None when missing or when the
    kernel's sources changed since the counters were taken)."""
    from paper_2412_03898_amd import profsum
    return profsum.traffic_for(instance, workload), profsum.sq_for(instance, workload)


def kernel_instance(kind, wl, choice):
    from paper_2412_03898_amd import binding
    if kind == "forward":
        if choice[0] == binding.SB_FWD_COLUMN_SHARED:
            return "forward_shared_kernel<33, 3>"
        if choice[0] == binding.SB_FWD_COLUMN_SHARED_SHORT:
            return "forward_shared_kernel<23, 4>"
        return f"forward_kernel<4, 256, {choice[0]}, 0>"
    mreg = 4 if wl.basis == 1 and wl.n_terms == 2 else 0
    return f"adjoint_uniform_kernel<{mreg}, {choice[1]}>"


def roofline(wl, balls_np, deform_np, kt, choice):
    fm = op_model(wl, balls_np, deform_np)
    per = {k: (ms / n if n else None) for k, (ms, n) in kt.items()}
    dom = max(("forward", "adjoint"), key=lambda k: per[k] or 0.0)
    sec = per[dom] * 1e-3
    achieved = fm[dom] / sec / 1e12
    traffic, sq = sq_and_traffic(kernel_instance(dom, wl, choice), wl.name)
    out = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TOPS, 2),
           "unit": "T lane-ops/s", "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": traffic,
           "traffic_unit": "B/launch", "kernel_ms": round(per[dom], 3),
           "ops_per_launch": fm[dom], "pairs_per_launch": fm["pairs"], "mean_window": round(fm["mean_window"], 3),
           "note": ("direct per-pair model (40 + 8 W forward, 40 + 14 W adjoint lane-ops); the kernels "
                    "evaluate closed forms with fewer operations, so frac can exceed 1"),
           "closed_form": {"ops_per_launch": fm["closed_" + dom],
                           "frac": round(fm["closed_" + dom] / sec / 1e12 / ALU_PEAK_TOPS, 4)}}
    if sq is not None:
        out["issued_valu_frac"] = round(sq * 64 / sec / 1e12 / ALU_PEAK_TOPS, 4)
    if traffic is not None:
        gbs = traffic / sec / 1e9
        out["hbm"] = {"achieved_gb_s": round(gbs, 1), "peak_gb_s": HBM_PEAK_GBS,
                      "frac": round(gbs / HBM_PEAK_GBS, 4)}
    # the other kernel of the pass, for context
    other = "adjoint" if dom == "forward" else "forward"
    if per[other]:
        osec = per[other] * 1e-3
        t2, q2 = sq_and_traffic(kernel_instance(other, wl, choice), wl.name)
        out["other_kernel"] = {
            "kernel": other, "kernel_ms": round(per[other], 3),
            "frac": round(fm[other] / osec / 1e12 / ALU_PEAK_TOPS, 4),
            "issued_valu_frac": None if q2 is None else round(q2 * 64 / osec / 1e12 / ALU_PEAK_TOPS, 4),
            "traffic": t2,
            "hbm_frac": None if t2 is None else round(t2 / osec / 1e9 / HBM_PEAK_GBS, 4)}
    return out, per


def per_frame_comparison(wl, balls, deform, sens, measured, iters):
    """The frame-by-frame path on the same start (materialised per-frame attributes)."""
    import torch
    from paper_2412_03898_amd import ir, ops
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    frames = ir.materialise_frames(wl, balls.cpu().numpy(), None if deform is None else deform.cpu().numpy())
    path = ir.PerFramePath(wl, sens, measured, frames)
    del frames
    ms = path.time_ms(iters, warmup=1)
    ops.check()
    mem = torch.cuda.max_memory_allocated() / 2**20
    del path
    torch.cuda.empty_cache()
    return ms, mem


def scene_step(wl, steps, warmup, tuning=None, compare_per_frame=False):
    """One workload's IR step through the captured graph (+ Adam): GPairs/s, ms per step,
    per-kernel ms; optionally beside the frame-by-frame path."""
    import torch
    from paper_2412_03898_amd import binding, ops
    pb, balls, deform, ft, sens, measured, choice, _ = setup_scene(wl, tuning)
    binding.timing(True)
    step = IRStep(pb, balls, deform, ft, sens, measured)
    torch.cuda.reset_peak_memory_stats()
    elapsed, kt = timed_steps(step, steps, warmup)
    mem = torch.cuda.max_memory_allocated() / 2**20
    binding.timing(False)
    step.close()
    flags = ops.check()
    pairs = pb.pairs()
    ms = elapsed / steps * 1e3
    rec = {"workload": wl.name, "scenes": len(wl.ball_offset) - 1, "balls": wl.n_balls,
           "frames": wl.n_frames, "sensors": wl.n_sensors, "samples": wl.n_samples,
           "tuning": list(choice), "ms_per_step": round(ms, 3),
           "gpairs_s": round(pairs * steps / elapsed / 1e9, 3),
           "kernel_ms": {k: (round(t / n, 4) if n else None) for k, (t, n) in kt.items()},
           "peak_mem_mb": round(mem, 1), "device_flags": flags}
    if compare_per_frame and len(wl.ball_offset) == 2 and wl.n_frames > 1:
        ms_f, mem_f = per_frame_comparison(wl, balls, deform, sens, measured, max(3, steps // 2))
        rec["per_frame_ms_per_iter"] = round(ms_f, 3)
        rec["per_frame_peak_mem_mb"] = round(mem_f, 1)
        rec["speedup_vs_per_frame"] = round(ms_f / ms, 3)
    del step, balls, deform, measured
    torch.cuda.empty_cache()
    return rec


def basis_sweep(counts=(1, 4, 13, 65), steps=6, warmup=1):
    """ms per IR iteration of the small 4D scene (50,000 balls, 16 frames, 512 sensors,
    2,048 samples) with the Gaussian-basis deformation of Eq. 2 (additive position) at N
    bases per attribute, against the 2-harmonic Fourier series of the same scene."""
    import dataclasses
    from paper_2412_03898_amd import synth
    base = synth.workload_vessel_4d()
    out = {}
    for n in counts:
        wl = dataclasses.replace(base, basis=2, n_terms=n,
                                 deform=synth.gauss_basis_coeffs(base.n_balls, n, 5))
        r = scene_step(wl, steps, warmup)
        out[str(n)] = {"ms_per_step": r["ms_per_step"], "kernel_ms": r["kernel_ms"], "tuning": r["tuning"],
                       "coefficients_per_ball": 15 * n}
    return out


def voxel_map_timing(reps=5):
    """Point cloud -> voxel grid -> maximum amplitude projections: the single-frame vessel
    scene (200,000 balls) on a 40 mm cube of 0.1 mm voxels (400^3, 256 MB); mean ms of
    slingbag_voxelize and of slingbag_map (all three projections)."""
    import torch
    from paper_2412_03898_amd import ops, synth
    wl = synth.workload_vessel_static()
    pb, balls, deform, _, _ = ops.to_device(wl, "cuda:0")
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


def host_threads():
    n = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit():
        n = min(n, int(omp))
    return n


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="vessel-4d-large", choices=sorted(workloads()))
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (timing and the parity check of its sample)")
    ap.add_argument("--no-per-frame", action="store_true", help="skip the frame-by-frame path")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads (single frame, small 4D, uneven batch, voxel grid)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with a 1 GiB device-to-device copy (a known amount of HBM traffic for "
                         "scaling memory counters)")
    ap.add_argument("--tuning", default=None,
                    help="fix the kernel knobs as COLUMN,OCCUPANCY,ITEMS instead of autotuning")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2412_03898_amd import binding, ops

    torch.cuda.set_device(0)
    wl = workloads()[args.workload]()
    tuning = args.tuning.split(",") if args.tuning else None
    pb, balls, deform, ft, sens, measured, choice, gt = setup_scene(wl, tuning)
    threads = host_threads()
    start_np = (balls.cpu().numpy(), None if deform is None else deform.cpu().numpy())
    cb = None
    if not args.no_cpu_baseline:
        cb = oracle_leg(wl, pb, balls, deform, ft, sens, gt,
                        s_step=32 if wl.n_frames > 1 else 8, frames=[0], all_threads=threads)
    del gt
    torch.cuda.empty_cache()

    # ---- the timed IR steps (captured forward + loss + adjoint, then Adam)
    binding.timing(True)
    step = IRStep(pb, balls, deform, ft, sens, measured)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    free0, total = torch.cuda.mem_get_info()
    elapsed, kt = timed_steps(step, args.steps, args.warmup)
    peak_torch = torch.cuda.max_memory_allocated() / 2**20
    binding.timing(False)
    step.close()
    flags = ops.check()
    del step
    torch.cuda.empty_cache()

    pairs = pb.pairs()
    ms_step = elapsed / args.steps * 1e3
    value = pairs * args.steps / elapsed / 1e9
    roof, per_kernel = roofline(wl, start_np[0], start_np[1], kt, choice)
    out = {
        "metric": METRIC,
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
                   "c_m_s": wl.c, "kernel": "uniform-sphere",
                   "deformation": ("fourier-2-harmonics-additive" if wl.basis == 1 else "static"),
                   "step": "graph(forward+loss+adjoint)+adam", "ball_order": "morton",
                   "tuning": {"forward_column": choice[0], "adjoint_occupancy": choice[1],
                              "adjoint_items": choice[2]}},
        "ms_per_ir_iteration": round(ms_step, 3),
        "peak_mem_mb": round(peak_torch, 1),
        "roofline": roof,
        "kernel_ms": {k: (round(v, 4) if v is not None else None) for k, v in per_kernel.items()},
        "device_flags": flags,
    }
    if not args.no_per_frame and wl.n_frames > 1:
        iters = max(2, min(5, args.steps // 4))
        ms_f, mem_f = per_frame_comparison(wl, balls, deform, sens, measured, iters)
        out["per_frame"] = {"ms_per_iter": round(ms_f, 3), "iterations_timed": iters,
                            "peak_mem_mb": round(mem_f, 1),
                            "batched_speedup": round(ms_f / ms_step, 3),
                            "gpairs_s": round(pairs / (ms_f * 1e-3) / 1e9, 3)}
    del balls, deform, measured
    torch.cuda.empty_cache()
    if cb is not None:
        out["cpu_baseline"] = cb
    if not args.no_extras:
        from paper_2412_03898_amd import synth
        ex = {}
        if args.workload != "vessel-single-frame":
            ex["single_frame"] = scene_step(synth.workload_vessel_static(), 20, 3)
        if args.workload != "vessel-4d":
            ex["small_4d"] = scene_step(synth.workload_vessel_4d(), 12, 2, compare_per_frame=True)
        ex["uneven_batch"] = scene_step(synth.workload_uneven_batch(), 4, 1)
        ex["gauss_basis_sweep_small_4d"] = basis_sweep()
        ex["voxel_map"] = voxel_map_timing()
        out["extras"] = ex
    print(json.dumps(out), flush=True)
    if args.copy_calibration:
        src = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
