"""Autotuning of the kernel knobs for a problem shape, with a JSON cache.

slingbag_autotune (C ABI) times the candidates on the caller's own problem and
keeps the fastest; this module wraps it for torch tensors and remembers the
choice per shape bucket (kernel, basis, terms, sensors, samples, ball count and
frame count rounded to powers of two) in a JSON file, so a later process with
a similar shape sets the knobs without timing again.
"""

from __future__ import annotations

import json
import math
import os

import torch

from . import binding
from .binding import Problem

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "slingbag", "autotune.json")


def shape_key(pb: Problem) -> str:
    c = pb.cfg
    b = max(pb.n_balls, 1)
    f = max(pb.n_frames, 1)
    return (f"k{c.kernel}-b{c.basis}-n{c.n_terms}-s{c.n_sensors}-t{c.n_samples}-"
            f"B{int(round(math.log2(b)))}-F{int(round(math.log2(f)))}-sc{len(pb.ball_offset) - 1}")


def apply(choice, kernel: int = 0):
    """Set the knobs of a choice; the column goes to the knob of `kernel` (0 uniform
    sphere, 1 Gaussian ball)."""
    col, occ, items = choice
    binding.tune(binding.SB_TUNE_FWD_GAUSS_COLUMN if kernel == 1 else binding.SB_TUNE_FWD_COLUMN, col)
    binding.tune(binding.SB_TUNE_ADJ_OCCUPANCY, occ)
    binding.tune(binding.SB_TUNE_ADJ_ITEMS, items)


def autotune(pb: Problem, balls, deform, frame_t, sensors, cache: str | None = DEFAULT_CACHE,
             force: bool = False):
    """Set the fastest knobs for this problem; returns (column, occupancy, items)."""
    key = shape_key(pb)
    table = {}
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
    if not force and key in table:
        choice = tuple(int(v) for v in table[key])
        apply(choice, pb.cfg.kernel)
        return choice
    B, F = pb.n_balls, pb.n_frames
    S, T, M = pb.cfg.n_sensors, pb.cfg.n_samples, pb.n_coef
    dev = balls.device
    sig = torch.empty((F, S, T), dtype=torch.float32, device=dev)
    gb = torch.empty((5, B), dtype=torch.float32, device=dev)
    gd = torch.empty((5, M, B), dtype=torch.float32, device=dev) if M else None
    stream = torch.cuda.current_stream().cuda_stream
    choice = binding.autotune(pb, balls.data_ptr(), deform.data_ptr() if deform is not None else None,
                              frame_t.data_ptr(), sensors.data_ptr(), sig.data_ptr(), gb.data_ptr(),
                              gd.data_ptr() if gd is not None else None, stream)
    if cache:
        table[key] = list(choice)
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        except OSError:
            pass
    return choice
