"""ctypes binding of libslingbag.so (include/slingbag.h), argument marshalling only.

The functions here take raw device addresses (ints) and host offset arrays and
call the C entry points of the same names; every step of the operator runs in
the library's HIP kernels.  Loading fails loudly when the library is missing:
there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
import re

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libslingbag.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "slingbag.h")

# status codes and enums, mirrored from include/slingbag.h
SB_OK = 0
SB_ERR_INVALID_ARG = -1
SB_ERR_SHAPE = -2
SB_ERR_NONFINITE = -3
SB_ERR_GEOMETRY = -4
SB_ERR_HIP = -5
SB_ERR_DEVICE_FLAG = -6
SB_ERR_UNSUPPORTED = -7
SB_FLAG_GEOMETRY, SB_FLAG_NONFINITE, SB_FLAG_CLIPPED = 1, 2, 4
SB_MAX_SCENES = 32


class SlingbagError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"slingbag status {status}: {message}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("basis", ctypes.c_int32),
                ("pos_mode", ctypes.c_int32), ("n_terms", ctypes.c_int32),
                ("n_sensors", ctypes.c_int32), ("n_samples", ctypes.c_int32),
                ("c", ctypes.c_double), ("fs", ctypes.c_double), ("t0", ctypes.c_double)]


class Batch(ctypes.Structure):
    _fields_ = [("n_scenes", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("ball_offset", ctypes.POINTER(ctypes.c_int64)),
                ("frame_offset", ctypes.POINTER(ctypes.c_int64))]


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("z0", ctypes.c_double), ("h", ctypes.c_double)]


_lib = None

_VP = ctypes.c_void_p
_SIGS = {
    "slingbag_forward": [ctypes.POINTER(Config), ctypes.POINTER(Batch), _VP, _VP, _VP, _VP, _VP, _VP],
    "slingbag_loss": [ctypes.POINTER(Config), ctypes.POINTER(Batch), _VP, _VP, _VP, _VP, _VP],
    "slingbag_loss_noalloc": [ctypes.POINTER(Config), ctypes.POINTER(Batch), _VP, _VP, _VP, _VP, _VP],
    "slingbag_adjoint": [ctypes.POINTER(Config), ctypes.POINTER(Batch), _VP, _VP, _VP, _VP, _VP,
                         _VP, _VP, _VP],
    "slingbag_check": [_VP, ctypes.POINTER(ctypes.c_uint32)],
    "slingbag_adam": [_VP, _VP, _VP, _VP, ctypes.c_int64, ctypes.c_float, ctypes.c_float,
                      ctypes.c_float, ctypes.c_float, ctypes.c_int32, ctypes.c_float, ctypes.c_float, _VP],
    "slingbag_order": [ctypes.POINTER(Batch), _VP, _VP, _VP],
    "slingbag_permute": [_VP, _VP, ctypes.c_int64, ctypes.c_int64, _VP, _VP],
    "slingbag_plan_create": [ctypes.POINTER(Config), ctypes.POINTER(Batch), _VP, _VP, _VP, _VP, _VP, _VP,
                             _VP, _VP, _VP, _VP, _VP, ctypes.POINTER(ctypes.c_void_p)],
    "slingbag_plan_run": [_VP, _VP],
    "slingbag_plan_destroy": [_VP],
    "slingbag_tune": [ctypes.c_int, ctypes.c_int],
    "slingbag_autotune": [ctypes.POINTER(Config), ctypes.POINTER(Batch), _VP, _VP, _VP, _VP, _VP, _VP,
                          _VP, ctypes.POINTER(ctypes.c_int32), _VP],
    "slingbag_tune_get": [ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
    "slingbag_timing": [ctypes.c_int],
    "slingbag_timing_read": [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)],
    "slingbag_voxelize": [ctypes.POINTER(Config), ctypes.POINTER(Grid), ctypes.c_int64, _VP, _VP, ctypes.c_float,
                          _VP, _VP],
    "slingbag_map": [ctypes.POINTER(Grid), _VP, _VP, _VP, _VP, _VP],
    "slingbag_last_error": [],
    "slingbag_version": [],
}


def header_functions() -> list[str]:
    """Names of the functions declared in include/slingbag.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(slingbag_\w+)\s*\(", text)))


def load():
    """Load libslingbag.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2412_03898_amd.build`"
                           " (the operator has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name == "slingbag_last_error" else ctypes.c_int
    _lib = lib
    return lib


def last_error() -> str:
    return load().slingbag_last_error().decode()


def _check(status: int):
    if status != SB_OK:
        raise SlingbagError(status, last_error())


class Problem:
    """Static description of a batch: physics config plus host offset arrays.

    Holds the ctypes structures so that repeated calls marshal nothing new.
    """

    def __init__(self, kernel, basis, pos_mode, n_terms, n_sensors, n_samples, c, fs, t0,
                 ball_offset, frame_offset):
        self.cfg = Config(int(kernel), int(basis), int(pos_mode), int(n_terms), int(n_sensors),
                          int(n_samples), float(c), float(fs), float(t0))
        self.ball_offset = np.ascontiguousarray(np.asarray(ball_offset, dtype=np.int64))
        self.frame_offset = np.ascontiguousarray(np.asarray(frame_offset, dtype=np.int64))
        n = len(self.ball_offset) - 1
        if n < 1 or len(self.frame_offset) != n + 1:
            raise ValueError("ball_offset and frame_offset must both have n_scenes+1 entries")
        self.batch = Batch(n, 0, self.ball_offset.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                           self.frame_offset.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))

    @classmethod
    def from_workload(cls, wl):
        return cls(wl.kernel, wl.basis, wl.pos_mode, wl.n_terms, wl.sensors.shape[1], wl.n_samples,
                   wl.c, wl.fs, wl.t0, wl.ball_offset, wl.frame_offset)

    @property
    def n_balls(self) -> int:
        return int(self.ball_offset[-1])

    @property
    def n_frames(self) -> int:
        return int(self.frame_offset[-1])

    @property
    def n_coef(self) -> int:
        b, n = self.cfg.basis, self.cfg.n_terms
        return 0 if b == 0 else (2 * n if b == 1 else 3 * n)

    def pairs(self) -> int:
        bo, fo = self.ball_offset, self.frame_offset
        return int(((bo[1:] - bo[:-1]) * (fo[1:] - fo[:-1])).sum()) * int(self.cfg.n_sensors)


def forward(pb: Problem, balls: int, deform: int, frame_t: int, sensors: int, signals: int,
            stream: int = 0):
    _check(load().slingbag_forward(ctypes.byref(pb.cfg), ctypes.byref(pb.batch), balls, deform,
                                   frame_t, sensors, signals, stream))


def loss(pb: Problem, signals: int, measured: int, residual: int, loss_out: int, stream: int = 0):
    _check(load().slingbag_loss(ctypes.byref(pb.cfg), ctypes.byref(pb.batch), signals, measured,
                                residual, loss_out, stream))


def loss_noalloc(pb: Problem, signals: int, measured: int, residual: int, loss_out: int, stream: int = 0):
    _check(load().slingbag_loss_noalloc(ctypes.byref(pb.cfg), ctypes.byref(pb.batch), signals, measured,
                                        residual, loss_out, stream))


def adjoint(pb: Problem, balls: int, deform: int, frame_t: int, sensors: int, residual: int,
            grad_balls: int, grad_deform: int, stream: int = 0):
    _check(load().slingbag_adjoint(ctypes.byref(pb.cfg), ctypes.byref(pb.batch), balls, deform,
                                   frame_t, sensors, residual, grad_balls, grad_deform, stream))


def adam(param: int, grad: int, m: int, v: int, n: int, lr: float, beta1: float, beta2: float,
         eps: float, step: int, stream: int = 0, lo: float = -float("inf"), hi: float = float("inf")):
    _check(load().slingbag_adam(param, grad, m, v, n, lr, beta1, beta2, eps, step, lo, hi, stream))


def plan_create(pb: Problem, balls: int, deform: int, frame_t: int, sensors: int, measured: int,
                signals: int, residual: int, loss_out: int, grad_balls: int, grad_deform: int,
                stream: int) -> int:
    h = ctypes.c_void_p(0)
    _check(load().slingbag_plan_create(ctypes.byref(pb.cfg), ctypes.byref(pb.batch), balls, deform, frame_t,
                                       sensors, measured, signals, residual, loss_out, grad_balls,
                                       grad_deform, stream, ctypes.byref(h)))
    return int(h.value)


def plan_run(plan: int, stream: int):
    _check(load().slingbag_plan_run(plan, stream))


def plan_destroy(plan: int):
    _check(load().slingbag_plan_destroy(plan))


def order(pb: Problem, balls: int, perm: int, stream: int = 0):
    _check(load().slingbag_order(ctypes.byref(pb.batch), balls, perm, stream))


def permute(src: int, dst: int, rows: int, n: int, perm: int, stream: int = 0):
    _check(load().slingbag_permute(src, dst, rows, n, perm, stream))


def make_grid(nx: int, ny: int, nz: int, x0: float, y0: float, z0: float, h: float) -> Grid:
    return Grid(int(nx), int(ny), int(nz), 0, float(x0), float(y0), float(z0), float(h))


def voxelize(kernel: int, basis: int, pos_mode: int, n_terms: int, grid: Grid, n_balls: int, balls: int,
             deform: int, t: float, volume: int, stream: int = 0):
    cfg = Config(int(kernel), int(basis), int(pos_mode), int(n_terms), 1, 1, 1.0, 1.0, 0.0)
    _check(load().slingbag_voxelize(ctypes.byref(cfg), ctypes.byref(grid), int(n_balls), balls, deform,
                                    float(t), volume, stream))


def map_projections(grid: Grid, volume: int, xy: int, yz: int, xz: int, stream: int = 0):
    _check(load().slingbag_map(ctypes.byref(grid), volume, xy, yz, xz, stream))


def check(stream: int = 0) -> int:
    """Wait for the stream; return the device flag bits (raises on geometry/non-finite flags)."""
    flags = ctypes.c_uint32(0)
    st = load().slingbag_check(stream, ctypes.byref(flags))
    if st != SB_OK:
        raise SlingbagError(st, last_error())
    return int(flags.value)


SB_TUNE_FWD_COLUMN, SB_TUNE_ADJ_OCCUPANCY, SB_TUNE_ADJ_ITEMS, SB_TUNE_FWD_GAUSS_COLUMN = 1, 2, 3, 4
# SB_TUNE_FWD_COLUMN values besides 64 and 128: one column per sensor shared by a block's
# waves, 132 samples (three blocks per compute unit) or 92 (four)
SB_FWD_COLUMN_SHARED, SB_FWD_COLUMN_SHARED_SHORT = 1, 2
# SB_TUNE_FWD_GAUSS_COLUMN value besides 128 and 256: a lane per sample, a row per wave
SB_FWD_GAUSS_LANE = 1


def tune(key: int, value: int):
    _check(load().slingbag_tune(int(key), int(value)))


def autotune(pb: Problem, balls: int, deform: int, frame_t: int, sensors: int, signals: int,
             grad_balls: int, grad_deform: int, stream: int = 0) -> tuple:
    c = (ctypes.c_int32 * 3)()
    _check(load().slingbag_autotune(ctypes.byref(pb.cfg), ctypes.byref(pb.batch), balls, deform, frame_t,
                                    sensors, signals, grad_balls, grad_deform, c, stream))
    return int(c[0]), int(c[1]), int(c[2])


def tune_get(key: int) -> int:
    v = ctypes.c_int(0)
    _check(load().slingbag_tune_get(int(key), ctypes.byref(v)))
    return int(v.value)


def timing(enable: bool):
    _check(load().slingbag_timing(1 if enable else 0))


TIMING_KINDS = ("forward", "adjoint", "loss", "adam")


def timing_read() -> dict:
    """{kind: (total_ms, launches)} of the main kernels since the last read."""
    ms = (ctypes.c_double * 4)()
    n = (ctypes.c_int64 * 4)()
    _check(load().slingbag_timing_read(ms, n))
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(TIMING_KINDS)}


def version() -> int:
    return int(load().slingbag_version())
