"""Seeded synthetic inputs for the point-cloud photoacoustic operator.

This module only draws inputs: sensor layouts, ball clouds, deformation
coefficients, frame times and the record start.  It holds none of the
operator's arithmetic (no pressure traces, no deformation evaluation, no
gradients), so both the FP64 oracle tests and the GPU path can take their
inputs from here without sharing any of the method's code.

All arrays are float32, SI units (metres, seconds), structure-of-arrays:
  balls   [5][B]        rows x, y, z, R, P (R = radius, or std for Gaussian balls)
  deform  [5][M][B]     per attribute (x, y, z, R, P), M coefficients per attribute
  sensors [3][S]        rows x, y, z
  frame_t [F]           normalised frame times in [0, 1]

The workloads follow the paper's experiments (Sec. 3.1 and 3.2: Fibonacci
sphere arrays, a cube-shaped source region, 17 frames, vascular networks) at
the scene sizes given for each named workload below; the rat-liver vessel data
of Sec. 3.2 is not available, so a seeded random branching vessel tree stands
in for it.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C_SOUND = 1500.0          # m/s
FS = 40.0e6               # Hz

ATTR_X, ATTR_Y, ATTR_Z, ATTR_R, ATTR_P = range(5)


# ---------------------------------------------------------------- sensors
def fibonacci_sphere(n: int, radius: float, hemisphere: bool = True) -> np.ndarray:
    """Fibonacci-spiral points on a sphere (Sec. 3.1/3.2 use this layout).

    hemisphere=True keeps z >= 0: z_i = 1 - (i + 1/2)/n; the full sphere uses
    z_i = 1 - 2(i + 1/2)/n.  Azimuth phi_i = i * pi * (3 - sqrt 5).
    Returns float32 [3][n].
    """
    i = np.arange(n, dtype=np.float64)
    if hemisphere:
        z = 1.0 - (i + 0.5) / n
    else:
        z = 1.0 - 2.0 * (i + 0.5) / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    pts = np.stack([rho * np.cos(phi), rho * np.sin(phi), z]) * radius
    return np.ascontiguousarray(pts.astype(np.float32))


# ---------------------------------------------------------------- balls
def uniform_cube_balls(n: int, half: float, r_range, p_range, seed: int) -> np.ndarray:
    """n balls uniform in [-half, half]^3, R ~ U(r_range), P ~ U(p_range)."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-half, half, size=(3, n))
    R = rng.uniform(r_range[0], r_range[1], size=n)
    P = rng.uniform(p_range[0], p_range[1], size=n)
    return np.ascontiguousarray(np.vstack([pos, R[None], P[None]]).astype(np.float32))


def _perpendicular_basis(d: np.ndarray):
    a = np.array([1.0, 0.0, 0.0]) if abs(d[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(d, a)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(d, e1)
    return e1, e2


def vessel_tree_segments(seed: int, depth: int = 6, half: float = 0.020,
                         root_len: float = 12e-3, shrink: float = 0.8,
                         tube_r=(1.0e-3, 0.2e-3), angle_deg=(20.0, 45.0)):
    """Binary branching tree of straight tube segments inside [-half, half]^3.

    depth levels (depth 6 -> 63 segments).  Level l has length
    root_len * shrink**l and tube radius tube_r[0] * (tube_r[1]/tube_r[0])**(l/(depth-1)).
    Each child leaves its parent's end at an angle U(angle_deg) about a random
    azimuth; the two children of a node sit on opposite azimuths.  Segment
    ends are clamped into the cube (a margin of the tube radius is kept).
    Returns a list of (start[3], end[3], tube_radius).
    """
    rng = np.random.default_rng(seed)
    segs = []
    lim = half - tube_r[0]
    start = np.array([0.0, 0.0, -0.75 * half])
    d0 = np.array([0.0, 0.0, 1.0])
    stack = [(start, d0, 0)]
    while stack:
        s, d, lev = stack.pop()
        length = root_len * shrink ** lev
        frac = lev / max(depth - 1, 1)
        rad = tube_r[0] * (tube_r[1] / tube_r[0]) ** frac
        e = np.clip(s + d * length, -lim, lim)
        segs.append((s.copy(), e.copy(), rad))
        if lev + 1 < depth:
            e1, e2 = _perpendicular_basis(d)
            az = rng.uniform(0.0, 2.0 * math.pi)
            for side in (0.0, math.pi):
                ang = math.radians(rng.uniform(*angle_deg))
                w = math.cos(az + side) * e1 + math.sin(az + side) * e2
                nd = math.cos(ang) * d + math.sin(ang) * w
                nd /= np.linalg.norm(nd)
                stack.append((e, nd, lev + 1))
    return segs


def vessel_tree_balls(n: int, seed: int, depth: int = 6, half: float = 0.020,
                      r_range=(0.1e-3, 0.4e-3), p_range=(0.3, 1.0),
                      tube_r=(1.0e-3, 0.2e-3)) -> np.ndarray:
    """n balls inside the tubes of a seeded vessel tree (Sec. 3.2 stand-in).

    Balls are allotted to segments in proportion to tube volume, uniform
    along the axis and uniform over the cross-section disc.  Centres are
    clamped so every ball stays inside the cube.  Returns float32 [5][n].
    """
    segs = vessel_tree_segments(seed, depth=depth, half=half, tube_r=tube_r)
    rng = np.random.default_rng(seed + 7919)
    vol = np.array([math.pi * r * r * np.linalg.norm(e - s) for s, e, r in segs])
    counts = rng.multinomial(n, vol / vol.sum())
    parts = []
    for (s, e, r), m in zip(segs, counts):
        if m == 0:
            continue
        axis = e - s
        ln = np.linalg.norm(axis)
        d = axis / ln if ln > 0 else np.array([0.0, 0.0, 1.0])
        e1, e2 = _perpendicular_basis(d)
        tt = rng.uniform(0.0, 1.0, size=m)
        rr = r * np.sqrt(rng.uniform(0.0, 1.0, size=m))
        ps = rng.uniform(0.0, 2.0 * math.pi, size=m)
        pts = (s[:, None] + axis[:, None] * tt[None]
               + e1[:, None] * (rr * np.cos(ps))[None]
               + e2[:, None] * (rr * np.sin(ps))[None])
        parts.append(pts)
    pos = np.concatenate(parts, axis=1)
    perm = rng.permutation(n)          # no spatial order in the returned cloud
    pos = pos[:, perm]
    R = rng.uniform(r_range[0], r_range[1], size=n)
    P = rng.uniform(p_range[0], p_range[1], size=n)
    lim = half - r_range[1]
    pos = np.clip(pos, -lim, lim)
    return np.ascontiguousarray(np.vstack([pos, R[None], P[None]]).astype(np.float32))


def perturbed(balls: np.ndarray, seed: int, pos_sd: float = 0.05e-3,
              r_rel: float = 0.05, p_rel: float = 0.1) -> np.ndarray:
    """Copy of a ball cloud with seeded perturbations (position N(0, pos_sd),
    R*(1 + N(0, r_rel)), P*(1 + N(0, p_rel))).  Used to build 'measured' data."""
    rng = np.random.default_rng(seed)
    out = balls.astype(np.float64).copy()
    n = balls.shape[1]
    out[0:3] += rng.normal(0.0, pos_sd, size=(3, n))
    out[3] *= 1.0 + rng.normal(0.0, r_rel, size=n)
    out[4] *= 1.0 + rng.normal(0.0, p_rel, size=n)
    out[3] = np.maximum(out[3], 0.25 * balls[3])
    return np.ascontiguousarray(out.astype(np.float32))


# ---------------------------------------------------------------- deformation coefficients
def fourier_coeffs(n: int, K: int, seed: int, pos_amp: float = 0.5e-3,
                   r_amp: float = 0.1, p_amp: float = 0.2, sd: float = 0.3) -> np.ndarray:
    """Coefficients of a K-harmonic Fourier deformation, layout [5][2K][n].

    Within one attribute, coefficient 2(k-1) multiplies cos(2 pi k t) and
    2(k-1)+1 multiplies sin(2 pi k t).  Each is drawn N(0, sd) * amp; when the
    sum of absolute values of an attribute exceeds amp it is rescaled to amp,
    so the deformation of that attribute stays within +-amp for every t.
    """
    rng = np.random.default_rng(seed)
    amps = np.array([pos_amp, pos_amp, pos_amp, r_amp, p_amp])
    c = rng.normal(0.0, sd, size=(5, 2 * K, n)) * amps[:, None, None]
    s = np.abs(c).sum(axis=1, keepdims=True)
    scale = np.where(s > amps[:, None, None], amps[:, None, None] / np.maximum(s, 1e-300), 1.0)
    c = c * scale
    return np.ascontiguousarray(c.astype(np.float32))


def gauss_basis_coeffs(n: int, N: int, seed: int, pos_amp: float = 0.5e-3,
                       r_amp: float = 0.1, p_amp: float = 0.2,
                       sigma_range=(0.08, 0.3), mul_pos: bool = False) -> np.ndarray:
    """Parameters of N Gaussian basis functions per attribute (Eq. 2), layout
    [5][3N][n]: within an attribute, entry 3n is the weight omega_n, 3n+1 the
    centre theta_n, 3n+2 the width sigma_n.  Weights are scaled so that
    sum |omega_n| <= amp; with mul_pos the position amplitude is relative
    (Eq. 1 multiplies mu by 1 + H)."""
    rng = np.random.default_rng(seed)
    pa = 0.02 if mul_pos else pos_amp
    amps = np.array([pa, pa, pa, r_amp, p_amp])
    out = np.empty((5, 3 * N, n), dtype=np.float64)
    w = rng.normal(0.0, 0.3, size=(5, N, n)) * amps[:, None, None]
    s = np.abs(w).sum(axis=1, keepdims=True)
    w = w * np.where(s > amps[:, None, None], amps[:, None, None] / np.maximum(s, 1e-300), 1.0)
    out[:, 0::3, :] = w
    out[:, 1::3, :] = rng.uniform(0.0, 1.0, size=(5, N, n))
    out[:, 2::3, :] = rng.uniform(sigma_range[0], sigma_range[1], size=(5, N, n))
    return np.ascontiguousarray(out.astype(np.float32))


def frame_times(F: int) -> np.ndarray:
    """Normalised frame times t_f = f/(F-1) in [0, 1]; a single frame sits at t = 0."""
    if F == 1:
        return np.zeros(1, dtype=np.float32)
    return (np.arange(F, dtype=np.float64) / (F - 1)).astype(np.float32)


# ---------------------------------------------------------------- record window
def record_start(shell_radius: float, half: float, r_max: float, pos_amp: float,
                 c: float = C_SOUND, fs: float = FS, margin: int = 8) -> int:
    """First recorded sample index k0 (t0 = k0/fs) so that the earliest
    arrival from anywhere in the cube is still inside the record:
    k0 = floor((R_shell - half*sqrt3 - 1.1 R_max - A_pos)/delta) - margin."""
    delta = c / fs
    return int(math.floor((shell_radius - half * math.sqrt(3.0) - 1.1 * r_max - pos_amp) / delta)) - margin


def record_length_needed(shell_radius: float, half: float, r_max: float, pos_amp: float,
                         k0: int, c: float = C_SOUND, fs: float = FS, margin: int = 8) -> int:
    delta = c / fs
    return int(math.ceil((shell_radius + half * math.sqrt(3.0) + 1.1 * r_max + pos_amp) / delta)) + margin - k0


# ---------------------------------------------------------------- workloads
@dataclass
class Workload:
    """One synthetic problem instance (host float32 arrays)."""
    name: str
    kernel: int                # 0 uniform sphere, 1 Gaussian ball
    basis: int                 # 0 static, 1 Fourier, 2 Gaussian basis (Eq. 2)
    pos_mode: int              # 0 additive offset, 1 multiplicative (Eq. 1)
    n_terms: int
    c: float
    fs: float
    t0: float
    n_samples: int
    sensors: np.ndarray        # [3][S]
    balls: np.ndarray          # [5][B_total]
    deform: np.ndarray | None  # [5][M][B_total]
    frame_t: np.ndarray        # [F_total]
    ball_offset: np.ndarray    # int64 [n_scenes+1]
    frame_offset: np.ndarray   # int64 [n_scenes+1]
    extra: dict = field(default_factory=dict)

    @property
    def n_sensors(self) -> int:
        return int(self.sensors.shape[1])

    @property
    def n_balls(self) -> int:
        return int(self.balls.shape[1])

    @property
    def n_frames(self) -> int:
        return int(self.frame_t.shape[0])

    @property
    def n_coef(self) -> int:
        if self.basis == 0:
            return 0
        return 2 * self.n_terms if self.basis == 1 else 3 * self.n_terms

    def pairs(self) -> int:
        """ball*sensor*frame pairs of one pass."""
        bo, fo = self.ball_offset, self.frame_offset
        return int(sum((bo[i + 1] - bo[i]) * (fo[i + 1] - fo[i])
                       for i in range(len(bo) - 1)) * self.n_sensors)


def _single_scene(name, balls, sensors, n_samples, k0, deform=None, F=1, basis=0,
                  K=0, pos_mode=0, kernel=0, extra=None):
    B = balls.shape[1]
    return Workload(name=name, kernel=kernel, basis=basis, pos_mode=pos_mode, n_terms=K,
                    c=C_SOUND, fs=FS, t0=k0 / FS, n_samples=n_samples, sensors=sensors,
                    balls=balls, deform=deform, frame_t=frame_times(F),
                    ball_offset=np.array([0, B], dtype=np.int64),
                    frame_offset=np.array([0, F], dtype=np.int64), extra=extra or {})


def workload_plain(n_balls: int = 2000, n_sensors: int = 256, n_samples: int = 1024,
                   seed: int = 0) -> Workload:
    """Plain single frame: balls uniform in a 20 mm cube, R ~ U(0.1, 0.3) mm,
    P ~ U(0.5, 1), sensors on a 60 mm Fibonacci hemisphere, 40 MHz, 1500 m/s."""
    half = 0.010
    balls = uniform_cube_balls(n_balls, half, (0.1e-3, 0.3e-3), (0.5, 1.0), seed)
    sensors = fibonacci_sphere(n_sensors, 0.060)
    k0 = record_start(0.060, half, 0.3e-3, 0.0)
    return _single_scene("plain-single-frame", balls, sensors, n_samples, k0,
                         extra={"half": half, "shell": 0.060})


def workload_vessel_static(n_balls: int = 200_000, n_sensors: int = 1024,
                           n_samples: int = 4096, seed: int = 2,
                           shell: float = 0.100) -> Workload:
    """Single frame at scale: vessel-tree balls in a 40 mm cube, R ~ U(0.1, 0.4) mm,
    P ~ U(0.3, 1), sensors on a 100 mm hemisphere, 4096 samples."""
    half = 0.020
    balls = vessel_tree_balls(n_balls, seed, half=half)
    sensors = fibonacci_sphere(n_sensors, shell)
    k0 = record_start(shell, half, 0.4e-3, 0.0)
    return _single_scene("vessel-single-frame", balls, sensors, n_samples, k0,
                         extra={"half": half, "shell": shell})


def workload_vessel_4d(n_balls: int = 50_000, n_frames: int = 16, n_sensors: int = 512,
                       n_samples: int = 2048, seed: int = 4, coef_seed: int = 5,
                       shell: float = 0.100, K: int = 2) -> Workload:
    """4D scene: vessel-tree balls deformed by a K-harmonic Fourier series
    (position offset <= 0.5 mm, radius scale +-10 %, P scale +-20 %),
    frames at t in [0, 1]."""
    half = 0.020
    balls = vessel_tree_balls(n_balls, seed, half=half)
    deform = fourier_coeffs(n_balls, K, coef_seed)
    sensors = fibonacci_sphere(n_sensors, shell)
    k0 = record_start(shell, half, 0.4e-3 * 1.1, 0.5e-3)
    return _single_scene("vessel-4d", balls, sensors, n_samples, k0, deform=deform,
                         F=n_frames, basis=1, K=K, extra={"half": half, "shell": shell})


def workload_uneven_batch(n_scenes: int = 8, n_sensors: int = 1024, n_samples: int = 4096,
                          seed: int = 7, b_range=(10_000, 400_000),
                          frame_choices=(4, 8, 16, 32), K: int = 2) -> Workload:
    """Independent 4D scenes with log-uniform ball counts and frame counts
    drawn from frame_choices, sharing one 1024-sensor hemisphere."""
    rng = np.random.default_rng(seed)
    half, shell = 0.020, 0.100
    counts = np.round(np.exp(rng.uniform(math.log(b_range[0]), math.log(b_range[1]),
                                         size=n_scenes))).astype(np.int64)
    frames = rng.choice(np.array(frame_choices), size=n_scenes)
    balls, deform, ts = [], [], []
    for i in range(n_scenes):
        balls.append(vessel_tree_balls(int(counts[i]), 100 + i, half=half))
        deform.append(fourier_coeffs(int(counts[i]), K, 200 + i))
        ts.append(frame_times(int(frames[i])))
    k0 = record_start(shell, half, 0.4e-3 * 1.1, 0.5e-3)
    bo = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    fo = np.concatenate([[0], np.cumsum(frames)]).astype(np.int64)
    return Workload(name="uneven-4d-batch", kernel=0, basis=1, pos_mode=0, n_terms=K,
                    c=C_SOUND, fs=FS, t0=k0 / FS, n_samples=n_samples,
                    sensors=fibonacci_sphere(n_sensors, shell),
                    balls=np.ascontiguousarray(np.concatenate(balls, axis=1)),
                    deform=np.ascontiguousarray(np.concatenate(deform, axis=2)),
                    frame_t=np.concatenate(ts).astype(np.float32),
                    ball_offset=bo, frame_offset=fo, extra={"half": half, "shell": shell})


def workload_large_ir(n_balls: int = 1_000_000, n_frames: int = 32, n_sensors: int = 2048,
                      n_samples: int = 4096, seed: int = 8, coef_seed: int = 9,
                      K: int = 2) -> Workload:
    """Large 4D IR scene: vessel tree, Fourier deformation, 120 mm hemisphere."""
    half, shell = 0.020, 0.120
    balls = vessel_tree_balls(n_balls, seed, half=half)
    deform = fourier_coeffs(n_balls, K, coef_seed)
    sensors = fibonacci_sphere(n_sensors, shell)
    k0 = record_start(shell, half, 0.4e-3 * 1.1, 0.5e-3)
    return _single_scene("vessel-4d-large", balls, sensors, n_samples, k0, deform=deform,
                         F=n_frames, basis=1, K=K, extra={"half": half, "shell": shell})


def heart_phantom(n_sensors: int = 1024, n_frames: int = 17, spacing: float = 0.5e-3,
                  slab_half: float = 12e-3, slab_thick: float = 1e-3, axes=(6e-3, 4.5e-3, 3.5e-3),
                  size_amp: float = 0.25, p_amp: float = 0.4, seed: int = 30):
    """Pulsating-heart phantom in the manner of Sec. 3.1 (its dimensions are not given).

    Three mutually perpendicular slabs (|z|, |x|, |y| <= slab_thick, the other two
    coordinates within +-slab_half) of uniform pressure, filled with uniform spheres of
    radius 0.6 spacing on a regular grid, static; and a central Gaussian ellipsoid
    (semi-axes `axes`) made of Gaussian balls (std 0.6 spacing) on the same grid out to
    1.5 semi-axes, pressure exp(-q^2/2) at normalised radius q, pulsating over the
    frames: positions (about the centre) and sizes scale by 1 + size_amp sin(2 pi t),
    pressure by 1 + p_amp sin(2 pi t) (Eq. 1, multiplicative, one Fourier harmonic).
    1,024 sensors on the full 60 mm Fibonacci sphere, 17 frames, cube +-25.6 mm.

    Returns (slabs, ellipsoid): two single-scene workloads sharing sensors, frames and
    record window (uniform-sphere and Gaussian-ball kernels); the measured signals are
    the sum of their forwards.
    """
    rng = np.random.default_rng(seed)
    half_cube, shell = 25.6e-3, 0.060
    g = np.arange(-slab_half, slab_half + 1e-9, spacing)
    t = np.arange(-slab_thick, slab_thick + 1e-9, spacing)
    slabs = []
    for axis in range(3):                       # thin along axis
        A, Bg, Cg = np.meshgrid(t, g, g, indexing="ij")
        pts = np.zeros((3, A.size))
        pts[axis] = A.ravel()
        pts[(axis + 1) % 3] = Bg.ravel()
        pts[(axis + 2) % 3] = Cg.ravel()
        slabs.append(pts)
    sp = np.concatenate(slabs, axis=1)
    sp += rng.normal(0.0, 0.02 * spacing, size=sp.shape)      # break exact lattice ties
    n_s = sp.shape[1]
    slab_balls = np.vstack([sp, np.full((1, n_s), 0.6 * spacing), np.full((1, n_s), 0.5)])
    ax = np.asarray(axes)
    r = np.arange(-1.5 * ax.max(), 1.5 * ax.max() + 1e-9, spacing)
    X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
    q2 = (X / ax[0]) ** 2 + (Y / ax[1]) ** 2 + (Z / ax[2]) ** 2
    keep = q2 <= 1.5 ** 2
    ep = np.stack([X[keep], Y[keep], Z[keep]])
    n_e = ep.shape[1]
    ell_balls = np.vstack([ep, np.full((1, n_e), 0.6 * spacing), np.exp(-0.5 * q2[keep])[None]])
    D = np.zeros((5, 2, n_e))
    D[0:4, 1] = size_amp                         # sin(2 pi t) coefficient: x, y, z, R
    D[4, 1] = p_amp                              # and P
    sensors = fibonacci_sphere(n_sensors, shell, hemisphere=False)
    r_max = 1.1 * 6 * 0.6 * spacing * (1 + size_amp)
    k0 = record_start(shell, half_cube, r_max, 0.0)
    T = record_length_needed(shell, half_cube, r_max, 0.0, k0)
    T = int(math.ceil(T / 64.0) * 64)
    extra = {"half": half_cube, "shell": shell, "spacing": spacing}
    slabs_wl = _single_scene("heart-slabs", np.ascontiguousarray(slab_balls.astype(np.float32)), sensors, T, k0,
                             F=n_frames, kernel=0, extra=extra)
    ell_wl = _single_scene("heart-ellipsoid", np.ascontiguousarray(ell_balls.astype(np.float32)), sensors, T, k0,
                           deform=np.ascontiguousarray(D.astype(np.float32)), F=n_frames, basis=1, K=1,
                           pos_mode=1, kernel=1, extra=extra)
    return slabs_wl, ell_wl


def synthetic_residual(n_frames: int, n_sensors: int, n_samples: int, seed: int) -> np.ndarray:
    """Seeded N(0, 1e-3) residual [F][S][T] for adjoint-only checks."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, 1e-3, size=(n_frames, n_sensors, n_samples)).astype(np.float32)


def morton_order(balls: np.ndarray, bits: int = 19, quantum: float = 2.0 ** -18,
                 origin: float = -1.0) -> np.ndarray:
    """Permutation that sorts balls by the Morton (Z-order) code of their centres.

    The operator's result does not depend on ball order; a spatially coherent
    order only makes consecutive balls arrive at nearly the same sample at
    every sensor.  Centres are quantised on a fixed grid (cells of `quantum`
    metres from `origin`, `bits` bits per axis, clamped to the grid), the
    same grid for every scene, and the sort is stable.
    """
    pos = np.asarray(balls[0:3], dtype=np.float64)
    q = np.floor((pos - origin) / quantum)
    q = np.clip(q, 0, (1 << bits) - 1).astype(np.int64)
    code = np.zeros(pos.shape[1], dtype=np.int64)
    for bit in range(bits):
        for a in range(3):
            code |= ((q[a] >> bit) & 1) << (3 * bit + a)
    return np.argsort(code, kind="stable")


def apply_order(wl: "Workload", per_scene: bool = True) -> "Workload":
    """Copy of a workload with each scene's balls (and coefficients) in Morton order."""
    balls = wl.balls.copy()
    deform = None if wl.deform is None else wl.deform.copy()
    bo = wl.ball_offset
    for i in range(len(bo) - 1):
        a, b = int(bo[i]), int(bo[i + 1])
        if b - a < 2:
            continue
        perm = morton_order(wl.balls[:, a:b]) + a
        balls[:, a:b] = wl.balls[:, perm]
        if deform is not None:
            deform[:, :, a:b] = wl.deform[:, :, perm]
    out = Workload(**{k: getattr(wl, k) for k in wl.__dataclass_fields__})
    out.balls = np.ascontiguousarray(balls)
    out.deform = None if deform is None else np.ascontiguousarray(deform)
    return out
