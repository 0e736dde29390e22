"""Torch-facing wrappers: device tensors in, device tensors out.

PyTorch supplies device memory and the current stream only; the arithmetic
runs in libslingbag's HIP kernels through the C ABI (binding.py).  Tensors
must be contiguous float32 on the current GPU with the layouts of
include/slingbag.h.
"""

from __future__ import annotations

import torch

from . import binding
from .binding import Problem

__all__ = ["Problem", "forward", "loss", "adjoint", "adam_", "order", "permute", "apply_order",
           "check", "to_device"]


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t, name, shape=None, dtype=torch.float32):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr() if t.numel() > 0 else None


def _shapes(pb: Problem):
    B, F = pb.n_balls, pb.n_frames
    S, T, M = pb.cfg.n_sensors, pb.cfg.n_samples, pb.n_coef
    return B, F, S, T, M


def forward(pb: Problem, balls, deform, frame_t, sensors, out=None):
    """Signals [F][S][T] of the batch (slingbag_forward)."""
    B, F, S, T, M = _shapes(pb)
    if out is None:
        out = torch.empty((F, S, T), dtype=torch.float32, device=balls.device)
    binding.forward(pb, _ptr(balls, "balls", (5, B)), _ptr(deform, "deform", (5, M, B) if M else None),
                    _ptr(frame_t, "frame_t", (F,)), _ptr(sensors, "sensors", (3, S)),
                    _ptr(out, "signals", (F, S, T)), _stream())
    return out


def loss(pb: Problem, signals, measured, residual=None, loss_out=None):
    """(loss, residual): residual = signals - measured, loss = 1/2 sum residual^2 (device f64)."""
    B, F, S, T, M = _shapes(pb)
    if residual is None:
        residual = torch.empty_like(signals)
    if loss_out is None:
        loss_out = torch.empty((), dtype=torch.float64, device=signals.device)
    binding.loss(pb, _ptr(signals, "signals", (F, S, T)), _ptr(measured, "measured", (F, S, T)),
                 _ptr(residual, "residual", (F, S, T)), _ptr(loss_out, "loss", (), torch.float64),
                 _stream())
    return loss_out, residual


def adjoint(pb: Problem, balls, deform, frame_t, sensors, residual, grad_balls=None, grad_deform=None):
    """(grad_balls [5][B], grad_deform [5][M][B] or None) given residual = dL/dsignals."""
    B, F, S, T, M = _shapes(pb)
    if grad_balls is None:
        grad_balls = torch.empty((5, B), dtype=torch.float32, device=balls.device)
    if M and grad_deform is None:
        grad_deform = torch.empty((5, M, B), dtype=torch.float32, device=balls.device)
    binding.adjoint(pb, _ptr(balls, "balls", (5, B)), _ptr(deform, "deform", (5, M, B) if M else None),
                    _ptr(frame_t, "frame_t", (F,)), _ptr(sensors, "sensors", (3, S)),
                    _ptr(residual, "residual", (F, S, T)), _ptr(grad_balls, "grad_balls", (5, B)),
                    _ptr(grad_deform, "grad_deform", (5, M, B)) if M else None, _stream())
    return grad_balls, (grad_deform if M else None)


def adam_(param, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, lo=-float("inf"), hi=float("inf")):
    """In-place Adam step on one parameter group, projected onto [lo, hi] (slingbag_adam);
    tensors of equal size."""
    n = param.numel()
    for t, name in ((grad, "grad"), (m, "m"), (v, "v")):
        if t.numel() != n:
            raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    binding.adam(_ptr(param, "param"), _ptr(grad, "grad"), _ptr(m, "m"), _ptr(v, "v"), n,
                 float(lr), float(beta1), float(beta2), float(eps), int(step), _stream(), float(lo), float(hi))
    return param


class StepGraph:
    """forward + loss + adjoint captured once as a HIP graph (slingbag_plan_*), replayed per step.

    Binds the given tensors: update their contents in place between runs (e.g. the
    optimiser step), never reallocate them.  Needs a non-default stream (capture).
    With in_place=True the residual overwrites the signals in one buffer (the loss
    allows the alias), which saves one [F][S][T] array; `signals` then holds the
    residual after each run.
    """

    def __init__(self, pb: Problem, balls, deform, frame_t, sensors, measured, stream=None,
                 in_place: bool = False):
        B, F, S, T, M = _shapes(pb)
        dev = balls.device
        self.pb = pb
        self.tensors = (balls, deform, frame_t, sensors, measured)
        self.signals = torch.empty((F, S, T), dtype=torch.float32, device=dev)
        self.residual = self.signals if in_place else torch.empty_like(self.signals)
        self.loss = torch.empty((), dtype=torch.float64, device=dev)
        self.grad_balls = torch.empty((5, B), dtype=torch.float32, device=dev)
        self.grad_deform = torch.empty((5, M, B), dtype=torch.float32, device=dev) if M else None
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.stream.wait_stream(torch.cuda.current_stream())
        self.handle = binding.plan_create(
            pb, _ptr(balls, "balls", (5, B)), _ptr(deform, "deform", (5, M, B) if M else None),
            _ptr(frame_t, "frame_t", (F,)), _ptr(sensors, "sensors", (3, S)),
            _ptr(measured, "measured", (F, S, T)), _ptr(self.signals, "signals"),
            _ptr(self.residual, "residual"), _ptr(self.loss, "loss", (), torch.float64),
            _ptr(self.grad_balls, "grad_balls"),
            _ptr(self.grad_deform, "grad_deform") if M else None, self.stream.cuda_stream)

    def run(self):
        """Replay on the current stream; returns (loss, grad_balls, grad_deform)."""
        binding.plan_run(self.handle, torch.cuda.current_stream().cuda_stream)
        return self.loss, self.grad_balls, self.grad_deform

    def close(self):
        if self.handle:
            binding.plan_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def order(pb: Problem, balls):
    """Morton permutation of every scene's balls (slingbag_order): int32 [B] on the GPU."""
    B = pb.n_balls
    perm = torch.empty((B,), dtype=torch.int32, device=balls.device)
    binding.order(pb, _ptr(balls, "balls", (5, B)), _ptr(perm, "perm", (B,), torch.int32), _stream())
    return perm


def permute(src, perm, out=None):
    """out[..., i] = src[..., perm[i]] over the last axis (slingbag_permute)."""
    n = src.shape[-1]
    rows = src.numel() // max(n, 1)
    if out is None:
        out = torch.empty_like(src)
    binding.permute(_ptr(src, "src"), _ptr(out, "out"), rows, n,
                    _ptr(perm, "perm", (n,), torch.int32), _stream())
    return out


def apply_order(pb: Problem, balls, deform=None):
    """Sort balls (and their deformation coefficients) along the Morton curve on the GPU.
    Returns (balls, deform, perm); results of every operator are unchanged up to
    this permutation of the per-ball arrays."""
    perm = order(pb, balls)
    nb = permute(balls, perm)
    nd = permute(deform, perm) if deform is not None else None
    return nb, nd, perm


def voxelize(pb: Problem, balls, deform, t: float, grid, out=None):
    """Voxel grid [nz][ny][nx] of the initial pressure of one scene's balls deformed at frame
    time t (slingbag_voxelize).  grid = (nx, ny, nz, x0, y0, z0, h), voxel (i, j, k) centred
    at (x0 + i h, y0 + j h, z0 + k h)."""
    nx, ny, nz = (int(v) for v in grid[:3])
    g = binding.make_grid(nx, ny, nz, *grid[3:])
    B = balls.shape[1]
    M = pb.n_coef
    if out is None:
        out = torch.empty((nz, ny, nx), dtype=torch.float32, device=balls.device)
    binding.voxelize(pb.cfg.kernel, pb.cfg.basis, pb.cfg.pos_mode, pb.cfg.n_terms, g, B,
                     _ptr(balls, "balls", (5, B)), _ptr(deform, "deform", (5, M, B) if M else None),
                     float(t), _ptr(out, "volume", (nz, ny, nx)), _stream())
    return out


def map_projections(volume):
    """Maximum amplitude projections of a volume [nz][ny][nx] (slingbag_map):
    (xy [ny][nx], yz [nz][ny], xz [nz][nx])."""
    nz, ny, nx = volume.shape
    g = binding.make_grid(nx, ny, nz, 0.0, 0.0, 0.0, 1.0)
    xy = torch.empty((ny, nx), dtype=torch.float32, device=volume.device)
    yz = torch.empty((nz, ny), dtype=torch.float32, device=volume.device)
    xz = torch.empty((nz, nx), dtype=torch.float32, device=volume.device)
    binding.map_projections(g, _ptr(volume, "volume"), _ptr(xy, "xy"), _ptr(yz, "yz"), _ptr(xz, "xz"), _stream())
    return xy, yz, xz


def check() -> int:
    """Synchronise the current stream and return the device flag bits (raises on errors)."""
    return binding.check(_stream())


def to_device(wl, device="cuda"):
    """Move a synthetic workload's arrays to the GPU: (Problem, balls, deform, frame_t, sensors)."""
    pb = Problem.from_workload(wl)
    dev = torch.device(device)
    balls = torch.from_numpy(wl.balls).to(dev).contiguous()
    deform = torch.from_numpy(wl.deform).to(dev).contiguous() if wl.deform is not None else None
    frame_t = torch.from_numpy(wl.frame_t).to(dev).contiguous()
    sensors = torch.from_numpy(wl.sensors).to(dev).contiguous()
    return pb, balls, deform, frame_t, sensors
