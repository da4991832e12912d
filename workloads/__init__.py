"""Seeded synthetic inputs for the D2Q9 pseudopotential runs.

This module is shared by the FP64 oracle tests and by the GPU path.  It holds
no arithmetic of the lattice Boltzmann step: it only builds initial density and
velocity fields and parameter sets.

Sources of the recipes (Li, Luo & Li):
  * Eq. (31), Sec. IV.A: tanh density profile of width W = 5 across the interface,
    between the coexistence densities rho_l and rho_g;
  * Sec. IV.A: b = 4, R = 1, G = -1, relaxation rates 1/tau_rho = 1/tau_j = 1,
    1/tau_e = 1/tau_zeta = 1/tau_q = 1.1; sigma = 0.11 for a = 0.5;
  * Sec. IV.B: sigma = 0.114 for a = 0.25;
  * Sec. IV.C: droplet splashing on a thin film: no-slip walls in y, periodic x,
    impact velocity (0, -U), 1/tau_e = 1/tau_zeta = 0.8, nu(rho) switched at rho_c.

Readings of points the paper leaves open:
  * T_c = 0.094 a (the rounded value the paper quotes for a = 1, 0.5, 0.25);
  * rho_l, rho_g of the initial profile are the Maxwell densities at T/T_c,
    interpolated from ``coexistence_table.json`` (written by
    ``python -m oracle.make_coexistence_table``);
  * the viscosity switch density is the printed rho_c = 0.5218 / b;
  * sigma = 0.11 for a = 1.0 (not stated in the paper);
  * droplet centre ((nx - 1)/2, (ny - 1)/2) so that the field is D4-symmetric;
  * splash: film interface at y = film, droplet centre (nx/2, film + R + gap),
    rho0 = max(film, drop), u0 = (0, -U) times the droplet's liquid fraction.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field

import numpy as np

TC_PER_A = 0.094
W_TANH = 5.0
_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "coexistence_table.json")
_table_cache = None

SIGMA_FOR_A = {0.25: 0.114, 0.5: 0.11, 1.0: 0.11}


def critical_temperature(a: float) -> float:
    return TC_PER_A * a


def rho_switch(b: float = 4.0) -> float:
    return 0.5218 / b


def coexistence(t_over_tc: float):
    """(rho_l, rho_g) of the Maxwell construction at T/T_c (b = 4), interpolated
    from the stored table: linear in rho_l, linear in log(rho_g)."""
    global _table_cache
    if _table_cache is None:
        with open(_TABLE) as fh:
            _table_cache = np.array(json.load(fh)["rows"], dtype=np.float64)
    t = _table_cache
    if not (t[0, 0] <= t_over_tc <= t[-1, 0]):
        raise ValueError(f"T/T_c = {t_over_tc} outside the stored table")
    rl = float(np.interp(t_over_tc, t[:, 0], t[:, 1]))
    rg = float(np.exp(np.interp(t_over_tc, t[:, 0], np.log(t[:, 2]))))
    return rl, rg


def tanh_profile(d, rho_l, rho_g, W=W_TANH):
    """Eq. (31) as a function of the signed distance d = r - r0 (liquid where d < 0)."""
    return 0.5 * (rho_l + rho_g) - 0.5 * (rho_l - rho_g) * np.tanh(2.0 * d / W)


def _grid(nx, ny):
    return np.arange(nx, dtype=np.float64)[None, :], np.arange(ny, dtype=np.float64)[:, None]


def _min_image(d, n):
    d = np.abs(d)
    return np.minimum(d, n - d)


def droplet_field(nx, ny, R0, rho_l, rho_g, W=W_TANH, cx=None, cy=None, periodic_y=True):
    """Circular droplet of radius R0 (Eq. 31), minimum-image distances on the torus."""
    cx = (nx - 1) / 2.0 if cx is None else cx
    cy = (ny - 1) / 2.0 if cy is None else cy
    x, y = _grid(nx, ny)
    dx = _min_image(x - cx, nx)
    dy = _min_image(y - cy, ny) if periodic_y else np.abs(y - cy)
    return tanh_profile(np.sqrt(dx * dx + dy * dy) - R0, rho_l, rho_g, W)


def ellipse_field(nx, ny, R0, aspect, rho_l, rho_g, W=W_TANH):
    """Elliptic droplet with semi-axes R0 sqrt(aspect) (x) and R0 / sqrt(aspect) (y),
    level set d = R0 (sqrt((x/A)^2 + (y/B)^2) - 1)."""
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    x, y = _grid(nx, ny)
    A, B = R0 * math.sqrt(aspect), R0 / math.sqrt(aspect)
    dx = _min_image(x - cx, nx)
    dy = _min_image(y - cy, ny)
    d = R0 * (np.sqrt((dx / A) ** 2 + (dy / B) ** 2) - 1.0)
    return tanh_profile(d, rho_l, rho_g, W)


def slab_field(nx, ny, thickness, rho_l, rho_g, W=W_TANH):
    """Liquid slab of the given thickness centred in y (two flat interfaces), uniform in x."""
    cy = (ny - 1) / 2.0
    _, y = _grid(nx, ny)
    d = np.abs(y - cy) - thickness / 2.0
    return np.broadcast_to(tanh_profile(d, rho_l, rho_g, W), (ny, nx)).copy()


def splash_field(nx, ny, R, film, U, rho_l, rho_g, gap, W=W_TANH):
    """Droplet of radius R above a liquid film of thickness `film` on the bottom wall.
    Returns rho0, ux0, uy0 (u0 = (0, -U) weighted by the droplet's liquid fraction)."""
    x, y = _grid(nx, ny)
    rho_film = tanh_profile(y - film + 0.0 * x, rho_l, rho_g, W)
    cx, cy = nx / 2.0, film + R + gap
    dx = _min_image(x - cx, nx)
    rho_drop = tanh_profile(np.sqrt(dx * dx + (y - cy) ** 2) - R, rho_l, rho_g, W)
    rho0 = np.maximum(rho_film, rho_drop)
    phi = (rho_drop - rho_g) / (rho_l - rho_g)
    ux0 = np.zeros_like(rho0)
    uy0 = -U * phi
    return rho0, ux0, uy0


@dataclass
class Workload:
    """One run: parameter dictionary (absolute T), initial fields and a name."""
    name: str
    params: dict
    rho0: np.ndarray
    ux0: np.ndarray | None = None
    uy0: np.ndarray | None = None
    info: dict = field(default_factory=dict)


def base_params(nx, ny, a=0.5, t_over_tc=0.6, bc=0, sigma=None, s_e=1.1, s_zeta=1.1, s_q=1.1,
                nu_l=0.1, nu_g=0.3, b=4.0):
    sigma = SIGMA_FOR_A.get(a, 0.11) if sigma is None else sigma
    return dict(nx=int(nx), ny=int(ny), bc=int(bc), a=float(a), b=float(b), R=1.0,
                T=float(t_over_tc * critical_temperature(a)), G=-1.0, sigma=float(sigma),
                s_rho=1.0, s_e=float(s_e), s_zeta=float(s_zeta), s_j=1.0, s_q=float(s_q),
                nu_l=float(nu_l), nu_g=float(nu_g), rho_switch=rho_switch(b))


def ss_params(nx, ny, G, eps, sigma=0.0, bc=0, nu=0.1, s_e=1.1, s_zeta=1.1, s_q=1.1):
    """Parameters of a run with the Sbragaglia-Shan pseudopotential of Eq. (23)
    (psi_form 1, parameter eps, coupling G); the Carnahan-Starling constants are
    unused and one viscosity holds in both phases."""
    return dict(nx=int(nx), ny=int(ny), bc=int(bc), a=0.0, b=4.0, R=1.0, T=1.0, G=float(G),
                sigma=float(sigma), s_rho=1.0, s_e=float(s_e), s_zeta=float(s_zeta), s_j=1.0,
                s_q=float(s_q), nu_l=float(nu), nu_g=float(nu), rho_switch=0.0, psi_form=1,
                psi_eps=float(eps))


def ss_slab(G, eps, rho_l, rho_g, sigma=0.0, nx=4, ny=200, thickness=None) -> Workload:
    """Flat liquid slab (periodic, uniform in x) with the Eq. (23) pseudopotential,
    started from a tanh profile between the given densities."""
    thickness = ny / 2.0 if thickness is None else thickness
    p = ss_params(nx, ny, G, eps, sigma)
    return Workload(f"ss_slab_{nx}x{ny}_eps{eps:g}_G{G:g}", p, slab_field(nx, ny, thickness, rho_l, rho_g),
                    info=dict(rho_l=rho_l, rho_g=rho_g, G=G, eps=eps, sigma=sigma))


def ss_droplet(n, R0, G, eps, rho_l, rho_g, sigma=0.0) -> Workload:
    """Stationary droplet with the Eq. (23) pseudopotential on an n x n periodic grid."""
    p = ss_params(n, n, G, eps, sigma)
    return Workload(f"ss_droplet_{n}x{n}_R{R0:g}_eps{eps:g}", p, droplet_field(n, n, R0, rho_l, rho_g),
                    info=dict(R0=R0, rho_l=rho_l, rho_g=rho_g, G=G, eps=eps, sigma=sigma))


def stationary_droplet(n=128, R0=25.0, a=0.5, t_over_tc=0.6, nu_l=0.1, nu_g=0.3, **kw) -> Workload:
    """Stationary droplet on an n x n periodic grid, tanh-initialised (Sec. IV.A recipe)."""
    p = base_params(n, n, a=a, t_over_tc=t_over_tc, nu_l=nu_l, nu_g=nu_g, **kw)
    rl, rg = coexistence(t_over_tc)
    rho0 = droplet_field(n, n, R0, rl, rg)
    return Workload(f"stationary_droplet_{n}x{n}_R{R0:g}", p, rho0,
                    info=dict(R0=R0, rho_l=rl, rho_g=rg, t_over_tc=t_over_tc))


def splash(scale=1, Re=200, nx=None, ny=None, U=0.05, t_over_tc=0.45, a=0.25, ratio=15.0) -> Workload:
    """Droplet splashing on a thin film (Sec. IV.C recipe at 2048 x 1024 per unit scale):
    R = 100 scale, film 20 scale, gap 5 scale, walls in y, periodic x.
    Re = U D / nu_l with D = 200 (the scale-1 diameter); nu_g = ratio * nu_l."""
    nx = 2048 * scale if nx is None else nx
    ny = 1024 * scale if ny is None else ny
    nu_l = U * 200.0 / Re
    p = base_params(nx, ny, a=a, t_over_tc=t_over_tc, bc=1, s_e=0.8, s_zeta=0.8, s_q=1.1,
                    nu_l=nu_l, nu_g=ratio * nu_l)
    rl, rg = coexistence(t_over_tc)
    R, film, gap = 100.0 * scale, 20.0 * scale, 5.0 * scale
    rho0, ux0, uy0 = splash_field(nx, ny, R, film, U, rl, rg, gap)
    return Workload(f"splash_{nx}x{ny}_Re{Re:g}", p, rho0, ux0, uy0,
                    info=dict(R=R, film=film, U=U, Re=Re, rho_l=rl, rho_g=rg, t_over_tc=t_over_tc))


def wall_film_droplet(nx=200, ny=150, U=0.02, t_over_tc=0.45, a=0.25) -> Workload:
    """Wall-bounded case without topology change: a liquid film of mean height 20 with
    a one-period sinusoidal surface (amplitude 3) on the lower wall, and a droplet of
    radius 25 centred at (nx/2, 95) moving towards it at (0, -U), well clear of the
    film, both walls and its periodic images.  Splash parameters (walls in y)."""
    p = splash(nx=nx, ny=ny).params
    p = dict(p, a=float(a), T=float(t_over_tc * critical_temperature(a)))
    rl, rg = coexistence(t_over_tc)
    x, y = _grid(nx, ny)
    film = tanh_profile(y - (20.0 + 3.0 * np.sin(2.0 * np.pi * x / nx)), rl, rg)
    drop = droplet_field(nx, ny, 25.0, rl, rg, cx=nx / 2.0, cy=95.0, periodic_y=False)
    rho0 = np.maximum(film, drop)
    phi = np.clip((drop - rg) / (rl - rg), 0.0, 1.0)
    ux0 = np.zeros_like(rho0)
    uy0 = -U * phi
    return Workload(f"wall_film_droplet_{nx}x{ny}", p, rho0, ux0, uy0,
                    info=dict(rho_l=rl, rho_g=rg, t_over_tc=t_over_tc, U=U))


def splash_crop(Re=200) -> Workload:
    """512 x 256 cut-down of the splash case (same R = 100, film 20, centre (256, 125))."""
    return splash(scale=1, Re=Re, nx=512, ny=256)


def batch_instances(n=512, seed=1211, side_lo=64, side_hi=512):
    """Sweep of independent droplets: square periodic grids with side ~ U{side_lo..side_hi},
    a ~ {0.25, 0.5, 1.0}, T/T_c ~ U[0.5, 0.85], R0 ~ U[0.1, 0.3] side, half of them
    elliptic (aspect 1.2, oscillating), nu_l = 0.1, nu_g = 0.3."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        side = int(rng.integers(side_lo, side_hi + 1))
        a = float(rng.choice([0.25, 0.5, 1.0]))
        tb = float(rng.uniform(0.5, 0.85))
        R0 = float(rng.uniform(0.1, 0.3) * side)
        ellipse = bool(rng.random() < 0.5)
        p = base_params(side, side, a=a, t_over_tc=tb)
        rl, rg = coexistence(tb)
        rho0 = ellipse_field(side, side, R0, 1.2, rl, rg) if ellipse else droplet_field(side, side, R0, rl, rg)
        out.append(Workload(f"inst{k}_{'ell' if ellipse else 'drop'}_{side}", p, rho0,
                            info=dict(R0=R0, rho_l=rl, rho_g=rg, t_over_tc=tb, ellipse=ellipse)))
    return out


def _droplet_case(side, a, tb, R0, ratio, nu_l=0.1):
    p = base_params(side, side, a=a, t_over_tc=tb, nu_l=nu_l, nu_g=ratio * nu_l)
    rl, rg = coexistence(tb)
    c = (side - 1) / 2.0
    rho0 = droplet_field(side, side, R0, rl, rg)
    return Workload(f"drop_{side}_a{a:g}_t{tb:.3f}_R{R0:.1f}_v{ratio:.2f}", p, rho0,
                    info=dict(R0=R0, rho_l=rl, rho_g=rg, t_over_tc=tb, ratio=ratio, cx=c, cy=c,
                              features=(a, tb, R0, ratio)))


def learned_train_instances(n=4096, seed=1212, side_lo=128, side_hi=512):
    """Training runs of the droplet initialiser: circular stationary droplets of the
    batched-sweep kind (square periodic side ~ U{side_lo..side_hi}, a ~ {0.25, 0.5, 1.0},
    T/T_c ~ U[0.5, 0.85], R0 ~ U[0.1, 0.3] side) with nu_g / nu_l ~ U[1, 15], nu_l = 0.1.
    side_lo = 128 keeps the sampled window (R0 +- 32) clear of the periodic images."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        side = int(rng.integers(side_lo, side_hi + 1))
        a = float(rng.choice([0.25, 0.5, 1.0]))
        tb = float(rng.uniform(0.5, 0.85))
        R0 = float(rng.uniform(0.1, 0.3) * side)
        ratio = float(rng.uniform(1.0, 15.0))
        out.append(_droplet_case(side, a, tb, R0, ratio))
    return out


def learned_eval_instances(n=256, seed=1213, side=256):
    """Held-out droplets for the initialiser: side x side periodic, R0 ~ U[0.1, 0.3] side,
    the other inputs drawn as for the training runs."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        a = float(rng.choice([0.25, 0.5, 1.0]))
        tb = float(rng.uniform(0.5, 0.85))
        R0 = float(rng.uniform(0.1, 0.3) * side)
        ratio = float(rng.uniform(1.0, 15.0))
        out.append(_droplet_case(side, a, tb, R0, ratio))
    return out


def oscillating_droplet(n=200, r_max=30.0, r_min=27.0, t_over_tc=0.5, a=0.5, nu_l=0.1, nu_g=0.3) -> Workload:
    """Droplet oscillation (Sec. IV.A, Fig. 2): n x n periodic, an ellipse with semi-axes
    r_max (x) and r_min (y) at the centre, tanh profile (Eq. 31) between the Maxwell
    densities; equilibrium radius R0 = sqrt(r_max r_min)."""
    p = base_params(n, n, a=a, t_over_tc=t_over_tc, nu_l=nu_l, nu_g=nu_g)
    rl, rg = coexistence(t_over_tc)
    R0 = math.sqrt(r_max * r_min)
    rho0 = ellipse_field(n, n, R0, r_max / r_min, rl, rg)
    c = (n - 1) / 2.0
    return Workload(f"oscillating_droplet_{n}_{r_max:g}x{r_min:g}_nu{nu_l:g}", p, rho0,
                    info=dict(R0=R0, r_max=r_max, r_min=r_min, rho_l=rl, rho_g=rg, t_over_tc=t_over_tc,
                              cx=c, cy=c))


def laplace_droplets(radii=(20.0, 25.0, 30.0, 35.0), n=200, t_over_tc=0.5, a=0.5, nu_l=0.1, nu_g=0.3):
    """Stationary droplets of several radii for a Laplace-law fit of the surface tension
    (Sec. IV.B/C evaluate it with Laplace's law)."""
    out = []
    for R in radii:
        w = stationary_droplet(n=n, R0=R, a=a, t_over_tc=t_over_tc, nu_l=nu_l, nu_g=nu_g)
        c = (n - 1) / 2.0
        w.info.update(cx=c, cy=c)
        out.append(w)
    return out


def coexistence_droplets(t_values, sigma=None, tau_nu=0.8, a=0.5, n=200, R0=50.0):
    """Stationary droplets of the coexistence-curve test (Sec. IV.A, Fig. 1): n x n periodic,
    radius R0 at the centre, tanh start (Eq. 31) between the Maxwell densities, one
    viscosity nu = (tau_nu - 1/2)/3 in both phases, s_e = s_zeta = s_q = 1.1; sigma = 0 is
    the original forcing scheme."""
    out = []
    nu = (tau_nu - 0.5) / 3.0
    for tb in t_values:
        kw = {} if sigma is None else {"sigma": float(sigma)}
        w = stationary_droplet(n=n, R0=R0, a=a, t_over_tc=float(tb), nu_l=nu, nu_g=nu, **kw)
        c = (n - 1) / 2.0
        w.info.update(cx=c, cy=c, sigma=w.params["sigma"], tau_nu=tau_nu, a=a)
        out.append(w)
    return out


def paper_splash(nu_l, ratio, U=0.125, nx=600, ny=250, R=50.0, gap=5.0, t_over_tc=0.5, a=0.25) -> Workload:
    """The paper's splash geometry (Sec. IV.C): 600 x 250, film one tenth of the height on
    the lower wall, droplet of radius 50 at (nx/2, film + R + gap) moving at (0, -U),
    walls in y, periodic x, a = 0.25, T = 0.5 T_c, 1/tau_e = 1/tau_zeta = 0.8,
    nu(rho) = nu_l above rho_c and ratio * nu_l below (the gap is not stated in the paper)."""
    p = base_params(nx, ny, a=a, t_over_tc=t_over_tc, bc=1, s_e=0.8, s_zeta=0.8, s_q=1.1,
                    nu_l=nu_l, nu_g=ratio * nu_l)
    rl, rg = coexistence(t_over_tc)
    film = ny / 10.0
    rho0, ux0, uy0 = splash_field(nx, ny, R, film, U, rl, rg, gap)
    return Workload(f"paper_splash_nu{nu_l:.4g}_ratio{ratio:g}", p, rho0, ux0, uy0,
                    info=dict(R=R, film=film, U=U, gap=gap, rho_l=rl, rho_g=rg, t_over_tc=t_over_tc, nu_l=nu_l,
                              ratio=ratio))
