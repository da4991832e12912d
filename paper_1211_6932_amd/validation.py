"""Validation runs of the paper's droplet tests on the GPU path.

  * surface tension from Laplace's law, dp = theta / R, fitted over stationary
    droplets of several radii (Sec. IV.B and IV.C evaluate the surface tension
    this way);
  * droplet oscillation (Sec. IV.A, Fig. 2): an elliptic droplet relaxes to a
    circle while oscillating in mode n = 2; the interface position along the major
    axis is fitted by a damped cosine c + A exp(-g t) cos(w t + phi), and the
    undamped period 2 pi / sqrt(w^2 + g^2) is compared with Lamb's inviscid
    two-dimensional result, Eq. (32); the damping rate with the viscous rate of the
    mode, 2 nu_l n (n - 1) / R0^2.

  * droplet splashing (Sec. IV.C, Fig. 9): the spread radius r of the liquid joining
    droplet and film, against the power law r / D = C sqrt(U t / D) (the paper:
    C ~ 1.3 for a planar droplet, no clear dependence on Re).

Lattice steps and reductions run in liblbmp.so; this module sequences them and
does the host arithmetic on the reduced values and on one lattice row per sample
(interface position by linear interpolation, level crossings for a first period
estimate, least-squares fits).

Readings: p_in is averaged over d < R0/2 and p_out over d >= R0 + 15 (three tanh
widths); the effective radius comes from the mass, R = sqrt((M - rho_out N) /
(pi (rho_in - rho_out))); the surface tension that enters Eq. (32) is Laplace's law
read at the oscillating droplet's own radius, theta = dp R for a stationary droplet of
radius R0 (the straight-line fit over several radii has a small intercept, so its
slope differs from dp R by a few per cent); the interface on the major axis is where the density
along the line through the centre crosses (rho_l + rho_g)/2 of the Maxwell
densities; rho_l in Eq. (32) is the oscillating droplet's inner density averaged
over the run.  Splash: the spread radius is the half-width of the liquid around
the impact point on the line half a lattice unit above the undisturbed film
surface (mean of the left and right mid-density crossings), and t counts from the
geometric contact time gap / U.
"""
from __future__ import annotations

import math

import numpy as np

from . import lbmp


def lamb_period(theta, rho_l, R0, n=2):
    """Eq. (32): T = 2 pi [n (n^2 - 1) theta / (rho_l R0^3)]^(-1/2)."""
    return 2.0 * math.pi / math.sqrt(n * (n * n - 1) * theta / (rho_l * R0 ** 3))


def effective_radius(mass, rho_in, rho_out, sites):
    return math.sqrt((mass - rho_out * sites) / (math.pi * (rho_in - rho_out)))


def laplace_regions(w):
    cx, cy, R = w.info["cx"], w.info["cy"], w.info["R0"]
    return (cx, cy, 0.0, 0.5 * R), (cx, cy, R + 15.0, math.inf)


def surface_tension(ws, steps=30000, window=10000, every=250, log=None):
    """Run stationary droplets `ws` together; average dp, rho_in, rho_out over the last
    `window` steps; fit dp = theta / R_eff + c.  Returns dict(theta, c, r2, points), each
    point with its own theta = dp R_eff."""
    import torch
    b = lbmp.Batch([w.params for w in ws], [torch.from_numpy(w.rho0.astype(np.float32)) for w in ws])
    rin, rout = zip(*[laplace_regions(w) for w in ws])
    b.step(steps - window)
    acc = []
    for k in range(window // every + 1):
        if k:
            b.step(every)
        acc.append(b.diagnostics_all(rin, rout))
    b.close()
    if any(d["unstable"] for d in acc[-1]):
        raise RuntimeError("a Laplace droplet went unstable")
    pts = []
    for i, w in enumerate(ws):
        dp = float(np.mean([a[i]["dp"] for a in acc]))
        r_in = float(np.mean([a[i]["rho_in"] for a in acc]))
        r_out = float(np.mean([a[i]["rho_out"] for a in acc]))
        R = effective_radius(acc[-1][i]["mass"], r_in, r_out, w.params["nx"] * w.params["ny"])
        pts.append(dict(R0=w.info["R0"], R_eff=R, dp=dp, rho_in=r_in, rho_out=r_out, theta=dp * R))
    x = np.array([1.0 / p["R_eff"] for p in pts])
    y = np.array([p["dp"] for p in pts])
    A = np.vstack([x, np.ones_like(x)]).T
    (theta, c), *_ = np.linalg.lstsq(A, y, rcond=None)
    r2 = 1.0 - ((y - A @ np.array([theta, c])) ** 2).sum() / ((y - y.mean()) ** 2).sum()
    if log:
        log(f"surface tension {theta:.5e} (intercept {c:.2e}, R^2 {r2:.5f})")
    return dict(theta=float(theta), c=float(c), r2=float(r2), points=pts)


def axis_extent(row, cx, rho_mid):
    """Distance from cx to the first point right of cx where the density along `row`
    (one lattice row through the centre, periodic) falls below rho_mid."""
    nx = row.shape[0]
    x = int(math.floor(cx)) + 1
    prev_x, prev_v = cx, float(np.interp(cx, np.arange(nx), row))
    for _ in range(nx):
        v = float(row[x % nx])
        if v < rho_mid:
            return (prev_x + (prev_v - rho_mid) / (prev_v - v) * (x - prev_x)) - cx
        prev_x, prev_v = x, v
        x += 1
    raise ValueError("no interface on the row")


def centre_row(rho, cy):
    """Density on the line y = cy (linear between the two rows around it)."""
    y0 = int(math.floor(cy))
    f = cy - y0
    return rho[y0] if f == 0.0 else (1.0 - f) * rho[y0] + f * rho[y0 + 1]


def period_from_crossings(t, x):
    """Mean period of x(t) from its upward crossings of its mean (linear interpolation)."""
    t = np.asarray(t, dtype=np.float64)
    v = np.asarray(x, dtype=np.float64) - np.mean(x)
    up = [t[i] - v[i] * (t[i + 1] - t[i]) / (v[i + 1] - v[i])
          for i in range(len(v) - 1) if v[i] < 0.0 <= v[i + 1]]
    if len(up) < 2:
        raise ValueError("fewer than two upward crossings")
    return (up[-1] - up[0]) / (len(up) - 1), up


def fit_damped_cosine(t, x, period_guess):
    """Least-squares fit of x(t) = c + A exp(-g t) cos(w t + phi).  Returns dict(period
    (damped, 2 pi / w), period0 (undamped, 2 pi / sqrt(w^2 + g^2)), decay (1 / g), rms)."""
    from scipy.optimize import curve_fit

    t = np.asarray(t, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)

    def model(tt, c, A, g, w, ph):
        return c + A * np.exp(-g * tt) * np.cos(w * tt + ph)

    t0 = t[0]
    c0 = float(np.mean(x))
    p0 = [c0, float(np.max(np.abs(x - c0))), 1.0 / (t[-1] - t0), 2.0 * math.pi / period_guess, 0.0]
    best = None
    for ph in (0.0, 0.5 * math.pi, math.pi, 1.5 * math.pi):
        p0[4] = ph
        try:
            p, _ = curve_fit(model, t - t0, x, p0=p0, maxfev=20000)
        except RuntimeError:
            continue
        rms = float(np.sqrt(np.mean((model(t - t0, *p) - x) ** 2)))
        if best is None or rms < best[1]:
            best = (p, rms)
    if best is None:
        raise ValueError("damped-cosine fit did not converge")
    (c, A, g, w, ph), rms = best
    w, g = abs(w), float(g)
    return dict(period=2.0 * math.pi / w, period0=2.0 * math.pi / math.sqrt(w * w + g * g),
                decay=(1.0 / g) if g > 0 else math.inf, rms=rms, mean=float(c))


def oscillation(w, steps=10400, every=10, skip=400, log=None):
    """Run the elliptic droplet; sample the interface position on the major axis every
    `every` steps and fit it from step `skip` on.  Returns dict(t, x, period, period0,
    decay, rho_l, ...)."""
    import torch
    s = lbmp.Sim(w.params, torch.from_numpy(w.rho0.astype(np.float32)))
    mid = 0.5 * (w.info["rho_l"] + w.info["rho_g"])
    rin, rout = laplace_regions(w)
    ts, xs, rls = [], [], []
    for k in range(steps // every + 1):
        if k:
            s.step(every)
        rho = s.moments()[0].cpu().numpy().astype(np.float64)
        ts.append(k * every)
        xs.append(axis_extent(centre_row(rho, w.info["cy"]), w.info["cx"], mid))
        if k % 50 == 0:
            rls.append(s.diagnostics(rin[0], rin[1], rin[3], rout[2])["rho_in"])
    s.check()
    s.close()
    ts, xs = np.array(ts), np.array(xs)
    keep = ts >= skip
    guess, _ = period_from_crossings(ts[keep], xs[keep])
    fit = fit_damped_cosine(ts[keep], xs[keep], guess)
    if log:
        log(f"{w.name}: damped period {fit['period']:.1f}, undamped {fit['period0']:.1f}, "
            f"decay {fit['decay']:.0f} steps (fit rms {fit['rms']:.1e})")
    return dict(t=ts, x=xs, rho_l=float(np.mean(rls)), crossing_period=float(guess), **fit)


def spread_half_width(row, cx, rho_mid):
    """Mean distance from cx to the mid-density crossings left and right of it on a
    periodic row whose density at cx is above rho_mid; 0 if it is not."""
    nx = row.shape[0]
    xs = np.arange(nx, dtype=np.float64)
    if float(np.interp(cx, xs, row)) < rho_mid:
        return 0.0
    ext = []
    for step in (1, -1):
        x_prev, v_prev = cx, float(np.interp(cx, xs, row))
        x = math.floor(cx) + 1 if step == 1 else math.ceil(cx) - 1
        while abs(x - cx) < nx / 2:
            v = float(row[x % nx])
            if v < rho_mid:
                ext.append(abs(x_prev + (v_prev - rho_mid) / (v_prev - v) * (x - x_prev) - cx))
                break
            x_prev, v_prev = x, v
            x += step
        else:
            ext.append(nx / 2.0)
    return 0.5 * (ext[0] + ext[1])


def splash_spread(w, t_end_star=2.0, every=10, log=None):
    """Run a splash workload; sample the spread radius every `every` steps up to
    t* = U t / D = t_end_star after contact.  Returns dict(t_star, r_over_D)."""
    import torch

    def f(a):
        return torch.from_numpy(np.asarray(a, dtype=np.float32))

    U, D, film = w.info["U"], 2.0 * w.info["R"], w.info["film"]
    t_contact = (w.info.get("gap", 5.0)) / U
    steps = int(math.ceil(t_contact + t_end_star * D / U))
    s = lbmp.Sim(w.params, f(w.rho0), f(w.ux0), f(w.uy0))
    mid = 0.5 * (w.info["rho_l"] + w.info["rho_g"])
    cx = w.params["nx"] / 2.0
    ts, rs = [], []
    for k in range(steps // every + 1):
        if k:
            s.step(every)
        rho = s.moments()[0].cpu().numpy().astype(np.float64)
        t = k * every - t_contact
        if t > 0:
            ts.append(U * t / D)
            rs.append(spread_half_width(centre_row(rho, film + 0.5), cx, mid) / D)
    s.check()
    s.close()
    if log:
        log(f"{w.name}: {len(ts)} samples to t* = {ts[-1]:.2f}, r/D at the end {rs[-1]:.3f}")
    return dict(t_star=np.array(ts), r_over_D=np.array(rs))


def power_law_coefficient(t_star, r_over_D, lo=0.1, hi=1.0):
    """Least-squares C of r / D = C sqrt(t*) over lo <= t* <= hi."""
    t = np.asarray(t_star)
    r = np.asarray(r_over_D)
    m = (t >= lo) & (t <= hi)
    q = np.sqrt(t[m])
    return float((q * r[m]).sum() / (q * q).sum())
