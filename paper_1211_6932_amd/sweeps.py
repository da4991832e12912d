"""Parameter sweeps of the paper's stationary-droplet tests on the batched GPU path.

  * coexistence curves (Sec. IV.A, Fig. 1): liquid and vapour densities of
    equilibrated droplets over T/T_c, original forcing (sigma = 0) against the
    improved one (Eq. (25)), and the lowest T/T_c each scheme survives;
  * spurious velocities (Sec. IV.B, Table I): the largest velocity of equilibrated
    droplets for a = 1, 0.5, 0.25;
  * lowest achievable liquid viscosity against the viscosity ratio nu_g / nu_l
    (Sec. IV.C, Fig. 4): splash runs over a grid of nu_l per ratio, the lowest nu_l
    above which every run of the grid survives.

Every droplet of a sweep advances in one batched launch (lb_batch_*); the
reductions (densities in the inner disc d < R0/2 and beyond d >= R0 + 15, the
maximum speed, the instability flag) come from lb_batch_diagnostics_all and are
averaged over the last `window` steps on the host.

Readings: the coexistence densities of a droplet run are its inner and outer
mean densities (the droplet's Laplace pressure shifts them slightly from a flat
interface's); a run "survives" if no site is flagged unstable (non-finite
density, b rho / 4 >= 1 or psi^2 <= 0) in `steps` steps; the spurious velocity is
the maximum speed over the lattice, averaged over the window.  The viscosity search
(Fig. 4) also applies a stricter criterion: a run fails once its maximum speed exceeds
the lattice speed of sound.
"""
from __future__ import annotations

import math

import numpy as np

from . import lbmp


def regions(w):
    cx, cy, R = w.info["cx"], w.info["cy"], w.info["R0"]
    return (cx, cy, 0.0, 0.5 * R), (cx, cy, R + 15.0, math.inf)


def droplet_sweep(ws, steps=40000, window=10000, every=500, log=None):
    """Equilibrate droplets `ws` together.  Returns one dict per droplet: rho_l, rho_g,
    ratio, max_u (window means), stable."""
    import torch
    b = lbmp.Batch([w.params for w in ws], [torch.from_numpy(w.rho0.astype(np.float32)) for w in ws])
    rin, rout = zip(*[regions(w) for w in ws])
    b.step(steps - window)
    recs = []
    for k in range(window // every + 1):
        if k:
            b.step(every)
        recs.append(b.diagnostics_all(rin, rout))
        if log and k == 0:
            log(f"sweep of {len(ws)} droplets reached step {steps - window}")
    b.close()
    out = []
    for i, w in enumerate(ws):
        stable = not any(r[i]["unstable"] for r in recs)
        if stable:
            rl = float(np.mean([r[i]["rho_in"] for r in recs]))
            rg = float(np.mean([r[i]["rho_out"] for r in recs]))
            mu = float(np.mean([r[i]["max_u"] for r in recs]))
        else:
            rl = rg = mu = float("nan")
        out.append(dict(t_over_tc=w.info["t_over_tc"], a=w.params["a"], sigma=w.params["sigma"],
                        tau_nu=w.info.get("tau_nu"), stable=stable, rho_l=rl, rho_g=rg,
                        ratio=rl / rg if stable else float("nan"), max_u=mu))
    return out


def lowest_stable(results):
    """Lowest T/T_c of a sweep such that every run at that T/T_c or above survived."""
    ts = sorted({r["t_over_tc"] for r in results}, reverse=True)
    low = None
    for t in ts:
        if all(r["stable"] for r in results if r["t_over_tc"] == t):
            low = t
        else:
            break
    return low


CS = 1.0 / math.sqrt(3.0)  # lattice speed of sound


def survival(ws, steps, every=100, u_limit=CS):
    """Advance runs `ws` (with initial velocities) together, checking every `every`
    steps.  Returns two lists: the step at which each run first flagged an unstable
    site (a non-finite density, b rho/4 >= 1 or psi^2 <= 0), and the step at which it
    first failed the stricter criterion, that or a maximum speed above `u_limit` (the
    speed of sound by default: the flow is then no longer a low-Mach-number flow the
    method models, whether or not the densities stay in range).  None = survived."""
    import torch

    def f(a):
        return None if a is None else torch.from_numpy(np.asarray(a, dtype=np.float32))

    has_u = all(w.ux0 is not None for w in ws)
    b = lbmp.Batch([w.params for w in ws], [f(w.rho0) for w in ws], [f(w.ux0) for w in ws] if has_u else None,
                   [f(w.uy0) for w in ws] if has_u else None)
    dummy = [(0.0, 0.0, 0.0, 1.0)] * len(ws)
    failed = [None] * len(ws)
    failed_u = [None] * len(ws)
    done = 0
    while done < steps:
        n = min(every, steps - done)
        b.step(n)
        done += n
        for i, d in enumerate(b.diagnostics_all(dummy, dummy)):
            if d["unstable"] and failed[i] is None:
                failed[i] = done
            if failed_u[i] is None and (d["unstable"] or not d["max_u"] <= u_limit):
                failed_u[i] = done
    b.close()
    return failed, failed_u


def lowest_stable_viscosity(nus, failed):
    """Lowest nu of the grid whose run survived (None if none did).  The surviving band
    need not reach the top of the grid: with nu_g / nu_l = 50 the largest liquid
    viscosities fail as well (the vapour relaxation rate 1/(3 nu_g + 1/2) gets small)."""
    alive = [nu for nu, fl in zip(nus, failed) if fl is None]
    return min(alive) if alive else None
