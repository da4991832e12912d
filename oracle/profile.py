"""Radial density profiles of a droplet, the representation the learned initialiser
predicts (FP64, NumPy).

TEST INFRASTRUCTURE ONLY (oracle).

The paper starts a droplet from the tanh profile of Eq. (31) around a centre and
radius; the relaxed droplet is again radially symmetric.  A profile is the vector
L_k of log densities at the radii r_k = R + (k - 63.5) / 2, k = 0..127 (a
64-lattice-unit window centred on the initial interface radius R).

  * to_rho0: the density field of a profile: at a site of minimum-image distance
    d from the centre, exp of L linearly interpolated at d, with L_0 / L_127 held
    inside r_0 / beyond r_127.  In terms of the hat functions h_k of the r_k grid
    (with the end hats extended to constants), log rho0 = sum_k L_k h_k(d).
  * to_rho0_mass: the field of the profile shifted outwards by the distance
    delta (|delta| <= 8) at which the field's total mass equals a given mass,
    log rho0(d) = sum_k L_k h_k(d - delta); delta by bisection (the mass grows
    with delta for a profile that falls outwards).
  * extract: the profile whose to_rho0 field best fits a given field in least
    squares of log density over all sites, plus lam * sum_k (L_{k+1} - L_k)^2,
    a weak smoothness term that only matters where no site falls (r_k < 0, or
    very few sites near the centre); on a linear profile it acts only at the two
    end samples.
    Normal equations: (H^T H + lam D) L = H^T log rho, tridiagonal.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_banded

N_SAMPLES = 128
LAM = 1e-4


def radii(R):
    return R + (np.arange(N_SAMPLES, dtype=np.float64) - 63.5) * 0.5


def min_image_distance(nx, ny, cx, cy):
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    dx = np.abs(x - cx)
    dy = np.abs(y - cy)
    dx = np.minimum(dx, nx - dx)
    dy = np.minimum(dy, ny - dy)
    return np.sqrt(dx * dx + dy * dy)


def hat_coordinates(d, R):
    """Left sample index k and weight t of the right one: log rho0 = (1-t) L_k + t L_{k+1}."""
    s = np.clip((d - radii(R)[0]) / 0.5, 0.0, N_SAMPLES - 1.0)
    k = np.minimum(np.floor(s).astype(np.int64), N_SAMPLES - 2)
    return k, s - k


def to_rho0(logrho, R, cx, cy, nx, ny):
    """Density field [ny][nx] of a profile."""
    logrho = np.asarray(logrho, dtype=np.float64)
    k, t = hat_coordinates(min_image_distance(nx, ny, cx, cy), R)
    return np.exp((1.0 - t) * logrho[k] + t * logrho[k + 1])


def to_rho0_mass(logrho, R, cx, cy, nx, ny, mass, iters=60):
    """(field, delta): the profile's field shifted radially to carry the given total mass."""
    lo, hi = -8.0, 8.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if to_rho0(logrho, R + mid, cx, cy, nx, ny).sum() < mass:
            lo = mid
        else:
            hi = mid
    delta = 0.5 * (lo + hi)
    return to_rho0(logrho, R + delta, cx, cy, nx, ny), delta


def extract(rho, cx, cy, R, lam=LAM):
    """Least-squares profile of the field rho[ny][nx] around (cx, cy)."""
    rho = np.asarray(rho, dtype=np.float64)
    ny, nx = rho.shape
    k, t = hat_coordinates(min_image_distance(nx, ny, cx, cy), R)
    k, t, v = k.ravel(), t.ravel(), np.log(rho).ravel()
    n = N_SAMPLES
    diag = np.zeros(n)
    off = np.zeros(n - 1)  # A[k][k+1]
    rhs = np.zeros(n)
    np.add.at(diag, k, (1.0 - t) ** 2)
    np.add.at(diag, k + 1, t * t)
    np.add.at(off, k, (1.0 - t) * t)
    np.add.at(rhs, k, (1.0 - t) * v)
    np.add.at(rhs, k + 1, t * v)
    # smoothness: lam * sum (L_{k+1} - L_k)^2 adds lam * (graph Laplacian of the path)
    diag[:-1] += lam
    diag[1:] += lam
    off -= lam
    ab = np.zeros((3, n))
    ab[0, 1:] = off
    ab[1] = diag
    ab[2, :-1] = off
    return solve_banded((1, 1), ab, rhs)
