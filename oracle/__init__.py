"""FP64 CPU oracle for the point-cloud photoacoustic operator (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the HIP library; it loads its own
C implementation (``sb_oracle.c``) built with gcc, and a brute-force Poisson
spherical-means quadrature (``brute.py``) used to pin the closed forms.

Every array argument is promoted to float64 before the call, so FP32 inputs
are represented exactly.  The problem description is read from any object
with the attributes kernel, basis, pos_mode, n_terms, c, fs, t0, n_samples,
sensors [3][S], balls [5][B], deform [5][M][B] or None, frame_t [F],
ball_offset and frame_offset ([n_scenes+1] prefix sums).

Parity status: forward, loss and gradient are pinned by the tests in
tests/test_oracle_pins.py (worked single-ball values, the zero-sum,
superposition, rotation and radial-shift invariants, brute-force quadrature of
Poisson's formula, finite differences, Fourier/Gaussian-basis special values).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sb_oracle.c")
_LIB = os.path.join(_HERE, "libsb_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc -O3 -fopenmp, no fast-math) into libsb_oracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Problem(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("basis", ctypes.c_int32),
                ("pos_mode", ctypes.c_int32), ("n_terms", ctypes.c_int32),
                ("n_sensors", ctypes.c_int32), ("n_samples", ctypes.c_int32),
                ("n_threads", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("c", ctypes.c_double), ("fs", ctypes.c_double), ("t0", ctypes.c_double),
                ("gauss_window", ctypes.c_double)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d = P(ctypes.c_double)
        i64 = P(ctypes.c_int64)
        lib.sbo_forward.argtypes = [P(Problem), ctypes.c_int, i64, i64, d, d, d, d, d]
        lib.sbo_forward.restype = ctypes.c_int
        lib.sbo_adjoint.argtypes = [P(Problem), ctypes.c_int, i64, i64, d, d, d, d, d, d, d]
        lib.sbo_adjoint.restype = ctypes.c_int
        lib.sbo_loss.argtypes = [d, d, ctypes.c_int64, d]
        lib.sbo_loss.restype = ctypes.c_double
        lib.sbo_deformed.argtypes = [P(Problem), ctypes.c_int, i64, i64, d, d, d, ctypes.c_int64, d]
        lib.sbo_deformed.restype = ctypes.c_int
        lib.sbo_voxelize.argtypes = [ctypes.c_int, ctypes.c_int64, d, d, d, d, d, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_int32, d]
        lib.sbo_voxelize.restype = ctypes.c_int
        lib.sbo_voxel_ties.argtypes = [ctypes.c_int64, d, d, d, d, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       P(ctypes.c_ubyte)]
        lib.sbo_voxel_ties.restype = ctypes.c_int64
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _problem(wl, n_threads=0, gauss_window=10.0):
    pb = Problem()
    pb.kernel, pb.basis, pb.pos_mode = int(wl.kernel), int(wl.basis), int(wl.pos_mode)
    pb.n_terms = int(wl.n_terms)
    pb.n_sensors = int(np.asarray(wl.sensors).shape[1])
    pb.n_samples = int(wl.n_samples)
    pb.n_threads = int(n_threads)
    pb.c, pb.fs, pb.t0 = float(wl.c), float(wl.fs), float(wl.t0)
    pb.gauss_window = float(gauss_window)
    return pb


def _offsets(wl):
    bo = np.ascontiguousarray(np.asarray(wl.ball_offset, dtype=np.int64))
    fo = np.ascontiguousarray(np.asarray(wl.frame_offset, dtype=np.int64))
    return bo, fo


def _check(st, what):
    if st != 0:
        raise OracleError(f"{what} failed with status {st}")


def n_coef(wl) -> int:
    if wl.basis == 0:
        return 0
    return 2 * wl.n_terms if wl.basis == 1 else 3 * wl.n_terms


def forward(wl, balls=None, deform=None, n_threads=0, gauss_window=10.0) -> np.ndarray:
    """Signals [F][S][T] (float64).  balls/deform override wl.balls/wl.deform."""
    lib = _load()
    balls = _f64(wl.balls if balls is None else balls)
    deform = wl.deform if deform is None else deform
    dfm = _f64(deform) if deform is not None else np.zeros(1)
    bo, fo = _offsets(wl)
    F = int(fo[-1])
    S = int(np.asarray(wl.sensors).shape[1])
    out = np.zeros((F, S, int(wl.n_samples)), dtype=np.float64)
    pb = _problem(wl, n_threads, gauss_window)
    st = lib.sbo_forward(ctypes.byref(pb), len(bo) - 1,
                         bo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                         fo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                         _ptr(balls), _ptr(dfm), _ptr(_f64(wl.frame_t)), _ptr(_f64(wl.sensors)),
                         _ptr(out))
    _check(st, "oracle forward")
    return out


def loss(y, d):
    """(L, residual) with residual = y - d and L = 1/2 sum residual^2 (float64)."""
    lib = _load()
    y = _f64(y)
    d = _f64(d)
    r = np.empty_like(y)
    L = lib.sbo_loss(_ptr(y), _ptr(d), y.size, _ptr(r))
    return float(L), r


def adjoint(wl, residual, balls=None, deform=None, n_threads=0, gauss_window=10.0):
    """(grad_balls [5][B], grad_deform [5][M][B] or None) of 1/2|y - d|^2 given residual = y - d."""
    lib = _load()
    balls = _f64(wl.balls if balls is None else balls)
    deform = wl.deform if deform is None else deform
    dfm = _f64(deform) if deform is not None else np.zeros(1)
    bo, fo = _offsets(wl)
    B = int(bo[-1])
    M = n_coef(wl)
    gb = np.zeros((5, B), dtype=np.float64)
    gd = np.zeros((5, max(M, 1), B), dtype=np.float64)
    pb = _problem(wl, n_threads, gauss_window)
    st = lib.sbo_adjoint(ctypes.byref(pb), len(bo) - 1,
                         bo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                         fo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                         _ptr(balls), _ptr(dfm), _ptr(_f64(wl.frame_t)), _ptr(_f64(wl.sensors)),
                         _ptr(_f64(residual)), _ptr(gb), _ptr(gd))
    _check(st, "oracle adjoint")
    return gb, (gd if M > 0 else None)


def deformed(wl, frame: int, balls=None, deform=None) -> np.ndarray:
    """Deformed attributes [5][B] at global frame index `frame` (Eq. 1)."""
    lib = _load()
    balls = _f64(wl.balls if balls is None else balls)
    deform = wl.deform if deform is None else deform
    dfm = _f64(deform) if deform is not None else np.zeros(1)
    bo, fo = _offsets(wl)
    out = np.full((5, int(bo[-1])), np.nan)
    pb = _problem(wl)
    st = lib.sbo_deformed(ctypes.byref(pb), len(bo) - 1,
                          bo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                          fo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                          _ptr(balls), _ptr(dfm), _ptr(_f64(wl.frame_t)), int(frame), _ptr(out))
    _check(st, "oracle deformed")
    return out


def adam_step(param, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, lo=-np.inf, hi=np.inf):
    """One bias-corrected Adam step in float64 (new param, m, v): the textbook update
    m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, p -= lr mhat / (sqrt(vhat) + eps),
    then the projection of p onto [lo, hi]."""
    p = np.asarray(param, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return np.clip(p - lr * mhat / (np.sqrt(vhat) + eps), lo, hi), m, v


def voxelize(kernel: int, attrs, grid, gauss_window: float = 10.0, n_threads: int = 0) -> np.ndarray:
    """Voxel grid [nz][ny][nx] of the initial pressure of balls with (deformed) attributes
    attrs [5][B] (x, y, z, R, P): sum of P phi(d) at voxel centres, phi = 1[d <= R]
    (uniform sphere) or exp(-d^2 / 2R^2) (Gaussian ball).  grid = (nx, ny, nz, x0, y0, z0, h)
    with voxel (i, j, k) centred at (x0 + i h, y0 + j h, z0 + k h)."""
    lib = _load()
    a = _f64(attrs)
    nx, ny, nz, x0, y0, z0, h = grid
    vol = np.empty((int(nz), int(ny), int(nx)))
    st = lib.sbo_voxelize(int(kernel), a.shape[1], _ptr(np.ascontiguousarray(a[0])), _ptr(np.ascontiguousarray(a[1])),
                          _ptr(np.ascontiguousarray(a[2])), _ptr(np.ascontiguousarray(a[3])),
                          _ptr(np.ascontiguousarray(a[4])), int(nx), int(ny), int(nz), float(x0), float(y0),
                          float(z0), float(h), float(gauss_window), int(n_threads), _ptr(vol))
    _check(st, "oracle voxelize")
    return vol


def voxel_ties(attrs, grid):
    """(mask [nz][ny][nx] bool, count): uniform-sphere voxels whose centre lies within the
    rounding of two FP64 evaluations of d^2 of some ball's surface (sbo_voxel_ties), where
    the inside test d <= R is decided by rounding rather than by the geometry."""
    lib = _load()
    a = _f64(attrs)
    nx, ny, nz, x0, y0, z0, h = grid
    mask = np.zeros((int(nz), int(ny), int(nx)), dtype=np.uint8)
    n = lib.sbo_voxel_ties(a.shape[1], _ptr(np.ascontiguousarray(a[0])), _ptr(np.ascontiguousarray(a[1])),
                           _ptr(np.ascontiguousarray(a[2])), _ptr(np.ascontiguousarray(a[3])), int(nx), int(ny),
                           int(nz), float(x0), float(y0), float(z0), float(h),
                           mask.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)))
    if n < 0:
        raise OracleError("oracle voxel ties: bad grid")
    return mask.astype(bool), int(n)


def voxel_ties_scene(wl, t: float, grid, balls=None, deform=None):
    """voxel_ties() of a single-scene workload's balls deformed by Eq. 1 at frame time t."""
    import types
    B = (wl.balls if balls is None else balls).shape[1]
    one = types.SimpleNamespace(**{**vars(wl), "frame_t": np.array([t], dtype=np.float32),
                                   "ball_offset": np.array([0, B]), "frame_offset": np.array([0, 1])})
    return voxel_ties(deformed(one, 0, balls=balls, deform=deform), grid)


def voxelize_scene(wl, t: float, grid, balls=None, deform=None, **kw) -> np.ndarray:
    """voxelize() of a single-scene workload's balls deformed by Eq. 1 at frame time t."""
    import types
    B = (wl.balls if balls is None else balls).shape[1]
    one = types.SimpleNamespace(**{**vars(wl), "frame_t": np.array([t], dtype=np.float32),
                                   "ball_offset": np.array([0, B]), "frame_offset": np.array([0, 1])})
    attrs = deformed(one, 0, balls=balls, deform=deform)
    return voxelize(wl.kernel, attrs, grid, **kw)


def maps(vol):
    """Maximum amplitude projections of vol [nz][ny][nx]: (xy [ny][nx] = max over z,
    yz [nz][ny] = max over x, xz [nz][nx] = max over y)."""
    v = np.asarray(vol)
    return v.max(axis=0), v.max(axis=2), v.max(axis=1)
