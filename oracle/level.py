"""Liquid level of a droplet profile: band levels, the level model and plateau
anchoring (FP64, NumPy).

TEST INFRASTRUCTURE ONLY (oracle).

Inside a relaxed droplet the density is uniform: the coexisting liquid density
(Sec. IV.A) shifted by the droplet's Laplace pressure (Sec. IV.B).  How far the
droplet's pressure jump starts from its relaxed value is set almost entirely by
that interior density, so the learned initialiser predicts it with a separate
FP64 linear model and pins the network's profile to it.

Profiles L_k (log density) sit at r_k = R + d_k, d_k = (k - 63.5) / 2, k = 0..127
(as in oracle.profile).

  * bands: inner = samples with d_k <= -min(12, R / 2) (never empty for
    0 <= R <= 63.5, where d_0 = -31.75 qualifies); outer = samples with d_k >= 12
    (k = 88..127).
  * levels(L, R) = (mean of L_k over the inner band, mean over the outer band).
  * anchor(L, R, lev): with rho_k = exp(L_k), rho_in = exp(inner level),
    rho_out = exp(outer level), rho* = exp(lev) and
    g = (rho* - rho_out) / (rho_in - rho_out):
    rho'_k = rho_out + (rho_k - rho_out) g, then rho'_k = rho* on the inner band;
    L'_k = log rho'_k.  The map is affine in density, so the interface shape is
    kept and the vapour end does not move; the inner band becomes exactly flat at
    the target.  L is returned unchanged when lev is not finite, when
    rho_in == rho_out, when g is not finite or when some rho'_k is not positive.
  * level model: least squares on the Chebyshev tensor basis
    T_i(z_a) T_j(z_t) T_k(z_u) T_l(z_v), i <= 2, j <= 6, k <= 3, l <= 1 (168
    terms, column ((i * 7 + j) * 4 + k) * 2 + l) of the features
    (a, T/T_c, u = 1/R, nu_g/nu_l); z = 2 (v - lo) / (hi - lo) - 1 clamped to
    [-1, 1], with lo, hi the range of that feature over the fit's rows (z = 0 when
    hi == lo).  Ridge term lam |c|^2, lam = 1e-12 trace(A^T A) / 168, i.e. the
    least-squares solution of the stacked system [A; sqrt(lam) I] c = [y; 0].
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import chebyshev

N_SAMPLES = 128
BAND = 12.0
DEG = (2, 6, 3, 1)
TERMS = int(np.prod([d + 1 for d in DEG]))
RIDGE = 1e-12

D = (np.arange(N_SAMPLES, dtype=np.float64) - 63.5) * 0.5


def bands(R):
    """Boolean masks (inner, outer) over the 128 samples of a profile around R."""
    return D <= -min(BAND, 0.5 * float(R)), D >= BAND


def levels(L, R):
    """(inner level, outer level) of one profile."""
    L = np.asarray(L, dtype=np.float64)
    inner, outer = bands(R)
    return float(np.mean(L[inner])), float(np.mean(L[outer]))


def anchor(L, R, lev):
    """The profile pinned to the inner level lev (see the module docstring)."""
    L = np.asarray(L, dtype=np.float64)
    if not np.isfinite(lev):
        return L.copy()
    inner, _ = bands(R)
    l_in, l_out = levels(L, R)
    r_in, r_out, r_t = np.exp(l_in), np.exp(l_out), np.exp(lev)
    if r_in == r_out:
        return L.copy()
    g = (r_t - r_out) / (r_in - r_out)
    if not np.isfinite(g):
        return L.copy()
    rho = r_out + (np.exp(L) - r_out) * g
    rho[inner] = r_t
    if not np.all(rho > 0.0):
        return L.copy()
    return np.log(rho)


def scaled(x, lo, hi):
    """Features mapped onto [-1, 1] (R replaced by 1/R; lo, hi are in that variable)."""
    v = np.array(x, dtype=np.float64, copy=True).reshape(-1, 4)
    v[:, 2] = 1.0 / v[:, 2]
    z = np.zeros_like(v)
    for f in range(4):
        if hi[f] > lo[f]:
            z[:, f] = np.clip(2.0 * (v[:, f] - lo[f]) / (hi[f] - lo[f]) - 1.0, -1.0, 1.0)
    return z


def design(x, lo, hi):
    """[n][168] basis matrix, column ((i * 7 + j) * 4 + k) * 2 + l."""
    z = scaled(x, lo, hi)
    V = [chebyshev.chebvander(z[:, f], DEG[f]) for f in range(4)]
    A = np.einsum("ni,nj,nk,nl->nijkl", *V)
    return A.reshape(len(z), TERMS)


def fit(x, y):
    """Level model (lo[4], hi[4], coef[168]) of targets y at features x."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 4)
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    v = x.copy()
    v[:, 2] = 1.0 / v[:, 2]
    lo, hi = v.min(0), v.max(0)
    A = design(x, lo, hi)
    lam = RIDGE * np.sum(A * A) / TERMS
    As = np.vstack([A, np.sqrt(lam) * np.eye(TERMS)])
    ys = np.concatenate([y, np.zeros(TERMS)])
    coef = np.linalg.lstsq(As, ys, rcond=None)[0]
    return lo, hi, coef


def evaluate(model, x):
    lo, hi, coef = model
    return design(x, lo, hi) @ coef
