"""Post-processing of density fields (FP64, NumPy).

TEST INFRASTRUCTURE ONLY (oracle).  Measures what the paper evaluates on its
runs: the Laplace pressure jump (Sec. IV.B and IV.C use Laplace's law to
evaluate the surface tension), the effective droplet radius, the interface
thickness (Sec. IV.B, Fig. 3) and the maximum spurious velocity (Table I).

Readings (the paper does not define these precisely):
  * pressure p = p_EOS(rho) per site (equal to Eq. (11) when psi follows Eq. (24));
  * p_in = mean over sites at distance d <= R0/2 from the droplet centre,
    p_out = mean over d >= R0 + 3W (W = 5, the tanh width of Eq. (31));
  * R_eff = sqrt((sum rho - rho_out N) / (pi (rho_in - rho_out)));
  * interface thickness = distance between the 10 % and 90 % crossings of
    (rho - rho_g)/(rho_l - rho_g), linearly interpolated;
  * droplet oscillation (Sec. IV.A, Fig. 2): the interface on the major axis is
    where the density on the horizontal line through the centre (linear in y
    between the two rows around it) first falls below a level, going outwards,
    linearly interpolated in x; the period is twice the mean spacing of the
    successive crossings of the signal's mean;
  * droplet splashing (Sec. IV.C): the spread radius is the half-width of the
    liquid around the impact point on the line half a lattice unit above the
    undisturbed film surface (linear in y between rows, mid-density crossings
    linearly interpolated in x, the mean of the two sides).
"""
from __future__ import annotations

import math

import numpy as np

from . import eos


def distance_field(nx, ny, cx, cy, periodic_y=True):
    """Distance of every site (x, y) to (cx, cy); minimum image in x, and in y if periodic."""
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    dx = np.abs(x - cx)
    dx = np.minimum(dx, nx - dx)
    dy = np.abs(y - cy)
    if periodic_y:
        dy = np.minimum(dy, ny - dy)
    return np.sqrt(dx * dx + dy * dy)


def region_means(field, d, r_min, r_max):
    """Mean of field over sites with r_min <= d < r_max, and the site count."""
    m = (d >= r_min) & (d < r_max)
    n = int(m.sum())
    return (float(field[m].mean()) if n else float("nan")), n


def laplace(rho, params, R0, W=5.0, cx=None, cy=None):
    """Pressure jump and effective radius of a centred droplet.

    Returns dict(p_in, p_out, dp, rho_in, rho_out, R_eff, theta, n_in, n_out) with
    theta = dp * R_eff (2-D Laplace law dp = theta / R) and n_in, n_out the site counts
    of the two regions."""
    ny, nx = rho.shape
    cx = (nx - 1) / 2.0 if cx is None else cx
    cy = (ny - 1) / 2.0 if cy is None else cy
    d = distance_field(nx, ny, cx, cy, periodic_y=(params.get("bc", 0) == 0))
    p = eos.p_eos(rho, params["a"], params["b"], params["R"], params["T"])
    p_in, n_in = region_means(p, d, 0.0, R0 / 2.0 + 1e-12)
    p_out, n_out = region_means(p, d, R0 + 3.0 * W, np.inf)
    rho_in, _ = region_means(rho, d, 0.0, R0 / 2.0 + 1e-12)
    rho_out, _ = region_means(rho, d, R0 + 3.0 * W, np.inf)
    R_eff = math.sqrt((rho.sum() - rho_out * rho.size) / (math.pi * (rho_in - rho_out)))
    dp = p_in - p_out
    return dict(p_in=p_in, p_out=p_out, dp=dp, rho_in=rho_in, rho_out=rho_out, R_eff=R_eff,
                theta=dp * R_eff, n_in=n_in, n_out=n_out)


def interface_width(profile, rho_l, rho_g, lo=0.1, hi=0.9):
    """Distance between the lo and hi crossings of the normalised profile along a
    monotone stretch (first crossing pair found scanning from the liquid side)."""
    phi = (np.asarray(profile, dtype=np.float64) - rho_g) / (rho_l - rho_g)
    i0 = int(np.argmax(phi))
    seg = phi[i0:]
    def crossing(level):
        k = np.nonzero(seg < level)[0]
        if k.size == 0:
            raise ValueError("profile does not cross the level")
        k = int(k[0])
        # linear interpolation between seg[k-1] >= level > seg[k]
        return (k - 1) + (seg[k - 1] - level) / (seg[k - 1] - seg[k])
    return crossing(lo) - crossing(hi)


def max_speed(ux, uy):
    return float(np.sqrt(ux * ux + uy * uy).max())


def linear_fit(x, y):
    """Least-squares y = s x + c; returns (s, c, r2)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    A = np.vstack([x, np.ones_like(x)]).T
    (s, c), *_ = np.linalg.lstsq(A, y, rcond=None)
    yhat = s * x + c
    r2 = 1.0 - ((y - yhat) ** 2).sum() / ((y - y.mean()) ** 2).sum()
    return float(s), float(c), float(r2)


def major_axis_radius(rho, cx, cy, level):
    """Distance from (cx, cy) along +x to the first crossing of `level` (see module notes)."""
    ny, nx = rho.shape
    j = int(np.floor(cy))
    fy = cy - j
    line = (1.0 - fy) * rho[j % ny] + fy * rho[(j + 1) % ny]
    i0 = int(np.floor(cx))
    xs = np.arange(i0, i0 + nx + 1, dtype=np.float64)
    vals = line[(np.arange(i0, i0 + nx + 1)) % nx]
    # the centre itself, then the lattice columns to its right
    v_c = vals[0] + (cx - i0) * (vals[1] - vals[0])
    xs = np.concatenate([[cx], xs[1:]])
    vals = np.concatenate([[v_c], vals[1:]])
    below = np.nonzero(vals < level)[0]
    if below.size == 0:
        raise ValueError("no crossing on the major axis")
    k = int(below[0])
    x = xs[k - 1] + (vals[k - 1] - level) / (vals[k - 1] - vals[k]) * (xs[k] - xs[k - 1])
    return float(x - cx)


def oscillation_period(t, r):
    """Twice the mean spacing of successive crossings (either direction) of r - mean(r)."""
    t = np.asarray(t, dtype=np.float64)
    v = np.asarray(r, dtype=np.float64) - float(np.mean(r))
    s = np.sign(v)
    idx = np.nonzero(s[:-1] * s[1:] < 0)[0]
    if idx.size < 3:
        raise ValueError("too few crossings")
    tc = t[idx] - v[idx] * (t[idx + 1] - t[idx]) / (v[idx + 1] - v[idx])
    return float(2.0 * np.mean(np.diff(tc)))


def spread_radius(rho, cx, y_line, level):
    """Half-width of the liquid (rho > level) around column cx on the line y = y_line."""
    ny, nx = rho.shape
    j = int(np.floor(y_line))
    fy = y_line - j
    line = (1.0 - fy) * rho[j] + fy * rho[j + 1]
    # walk outwards over the columns on each side, starting from the interpolated centre value
    i0 = int(np.floor(cx))
    v_c = line[i0 % nx] + (cx - i0) * (line[(i0 + 1) % nx] - line[i0 % nx])
    if v_c < level:
        return 0.0
    half = []
    for cols in (np.arange(i0 + 1, i0 + 1 + nx // 2), np.arange(int(np.ceil(cx)) - 1, int(np.ceil(cx)) - 1 - nx // 2, -1)):
        pos = np.concatenate([[cx], cols.astype(np.float64)])
        val = np.concatenate([[v_c], line[cols % nx]])
        k = np.nonzero(val < level)[0]
        if k.size == 0:
            half.append(nx / 2.0)
            continue
        k = int(k[0])
        x = pos[k - 1] + (val[k - 1] - level) / (val[k - 1] - val[k]) * (pos[k] - pos[k - 1])
        half.append(abs(x - cx))
    return 0.5 * (half[0] + half[1])
