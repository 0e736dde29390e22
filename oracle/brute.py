"""Brute-force quadrature of Poisson's spherical-means formula (test infrastructure).

Independent of the closed forms in sb_oracle.c: the pressure at a point
sensor x_s of the 3D wave equation with initial pressure p0 and zero initial
velocity is p(x_s, t) = d/dt [ t M(x_s, c t) ], where M(x_s, rho) is the mean of
p0 over the sphere of radius rho about x_s.  A sample is the average of p over
[t_k - dt/2, t_k + dt/2], i.e. v_k = [t M(x_s, ct)] between the interval ends,
divided by dt.  M is evaluated here by a midpoint rule over the sphere
(cos(theta) x azimuth), with the pole on the sensor-to-ball axis and the polar
range cut to the cone outside of which p0 vanishes (uniform ball) or is below
exp(-cut^2/2) of its peak (Gaussian ball).  Pure numpy, for tiny inputs only.
"""

from __future__ import annotations

import math

import numpy as np


def _basis(e):
    a = np.array([1.0, 0.0, 0.0]) if abs(e[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(e, a)
    e1 /= np.linalg.norm(e1)
    return e1, np.cross(e, e1)


def spherical_mean(xs, xb, R, P, kernel, rho, n_mu, n_phi, cut=12.0, chunk=200_000):
    """Mean of one ball's p0 over the sphere |x - xs| = rho (midpoint quadrature)."""
    xs = np.asarray(xs, dtype=np.float64)
    xb = np.asarray(xb, dtype=np.float64)
    d = xb - xs
    r = float(np.linalg.norm(d))
    e = d / r
    e1, e2 = _basis(e)
    reach = R if kernel == 0 else cut * R
    if reach >= r:
        mu_min = -1.0
    else:
        mu_min = math.sqrt(1.0 - (reach / r) ** 2)
    hmu = (1.0 - mu_min) / n_mu
    phi = (np.arange(n_phi) + 0.5) * (2.0 * math.pi / n_phi)
    cphi, sphi = np.cos(phi), np.sin(phi)
    total = 0.0
    for s in range(0, n_mu, chunk):
        mu = mu_min + (np.arange(s, min(n_mu, s + chunk)) + 0.5) * hmu
        st = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
        # points xs + rho * (mu e + st (cos phi e1 + sin phi e2)), shape [n_mu_chunk, n_phi, 3]
        dirs = (mu[:, None, None] * e[None, None, :]
                + st[:, None, None] * (cphi[None, :, None] * e1[None, None, :]
                                       + sphi[None, :, None] * e2[None, None, :]))
        pts = xs[None, None, :] + rho * dirs
        dist2 = ((pts - xb[None, None, :]) ** 2).sum(axis=-1)
        if kernel == 0:
            vals = np.where(dist2 <= R * R, P, 0.0)
        else:
            vals = P * np.exp(-dist2 / (2.0 * R * R))
        total += vals.sum()
    return total * hmu * (2.0 * math.pi / n_phi) / (4.0 * math.pi)


def forward_bruteforce(balls, sensors, c, fs, t0, n_samples, kernel, k_range=None,
                       n_mu=200_000, n_phi=2, cut=12.0):
    """Signals [S][T] of a static scene (balls [5][B], sensors [3][S]) by quadrature.

    Only samples in k_range=(k_lo, k_hi) (inclusive) are evaluated; the rest are 0.
    """
    balls = np.asarray(balls, dtype=np.float64)
    sensors = np.asarray(sensors, dtype=np.float64)
    S = sensors.shape[1]
    dt = 1.0 / fs
    k_lo, k_hi = (0, n_samples - 1) if k_range is None else k_range
    out = np.zeros((S, n_samples))
    ends = t0 + (np.arange(k_lo, k_hi + 2) - 0.5) * dt        # interval boundaries
    for j in range(S):
        xs = sensors[:, j]
        phi_vals = np.zeros(len(ends))
        for b in range(balls.shape[1]):
            xb, R, P = balls[0:3, b], balls[3, b], balls[4, b]
            r = float(np.linalg.norm(xb - xs))
            reach = R if kernel == 0 else cut * R
            for m, t in enumerate(ends):
                if abs(c * t - r) > reach:      # the sphere misses the support: M = 0
                    continue
                phi_vals[m] += t * spherical_mean(xs, xb, R, P, kernel, c * t, n_mu, n_phi, cut=cut)
        out[j, k_lo:k_hi + 1] = np.diff(phi_vals) / dt
    return out
