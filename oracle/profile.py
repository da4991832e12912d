"""Radial density profiles of a droplet, the representation the learned initialiser
predicts (FP64, NumPy, plain loops).

TEST INFRASTRUCTURE ONLY (oracle).

The paper starts a droplet from the tanh profile of Eq. (31) around a centre and
radius; the relaxed droplet is again radially symmetric.  A profile here is the
vector of log densities at the radii r_k = R + (k - 63.5) / 2, k = 0..127 (a
64-lattice-unit window centred on the initial interface radius R):

  * extract: log of the mean, over 256 equally spaced angles, of the density
    interpolated bilinearly (periodic lattice) at distance r_k from the centre;
  * to_rho0: density field whose value at a site is exp of the profile
    interpolated linearly at the site's minimum-image distance from the centre,
    with the end values held outside the window.
"""
from __future__ import annotations

import math

import numpy as np

N_SAMPLES = 128
N_ANGLES = 256


def radii(R):
    return R + (np.arange(N_SAMPLES, dtype=np.float64) - 63.5) * 0.5


def bilinear_periodic(rho, x, y):
    """Bilinear interpolation of rho[ny][nx] at the point (x, y), periodic in both directions."""
    ny, nx = rho.shape
    x0, y0 = math.floor(x), math.floor(y)
    fx, fy = x - x0, y - y0
    i0, j0 = x0 % nx, y0 % ny
    i1, j1 = (i0 + 1) % nx, (j0 + 1) % ny
    return ((1 - fx) * (1 - fy) * rho[j0, i0] + fx * (1 - fy) * rho[j0, i1]
            + (1 - fx) * fy * rho[j1, i0] + fx * fy * rho[j1, i1])


def extract(rho, cx, cy, R):
    """Profile (log densities at r_k) of the field rho around (cx, cy)."""
    rho = np.asarray(rho, dtype=np.float64)
    out = np.empty(N_SAMPLES)
    for k, r in enumerate(radii(R)):
        acc = 0.0
        for j in range(N_ANGLES):
            th = 2.0 * math.pi * j / N_ANGLES
            acc += bilinear_periodic(rho, cx + r * math.cos(th), cy + r * math.sin(th))
        out[k] = math.log(acc / N_ANGLES)
    return out


def to_rho0(logrho, R, cx, cy, nx, ny):
    """Density field [ny][nx] built from a profile."""
    logrho = np.asarray(logrho, dtype=np.float64)
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    dx = np.abs(x - cx)
    dy = np.abs(y - cy)
    dx = np.minimum(dx, nx - dx)
    dy = np.minimum(dy, ny - dy)
    d = np.sqrt(dx * dx + dy * dy)
    # np.interp is linear interpolation with the end values held outside
    return np.exp(np.interp(d, radii(R), logrho))
