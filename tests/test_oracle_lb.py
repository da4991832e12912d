"""Pins of the oracle's full time step (oracle/lbref.c) against invariants, textbook
special cases and the paper's own theory and printed results.  CPU only.

Readings used here (also listed in the design notes):
  * coexistence densities of a run = the densities in the middle of the liquid slab /
    far in the vapour of a flat-interface run (periodic 4 x 200 box, slab 100 thick);
  * interface thickness = W of the best fit of the Eq. (31) tanh profile;
  * Laplace pressure jump from post.laplace (p = p_EOS, inner / outer regions)."""
import functools
import math

import numpy as np
import pytest
from scipy.optimize import curve_fit

import workloads as W
from oracle import eos, post
from oracle import lbref as O

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def state(params, rho0, ux0=None, uy0=None):
    return O.State(O.Params(**params), rho0, ux0, uy0)


def momentum(f):
    return (f * EX[:, None, None]).sum(), (f * EY[:, None, None]).sum()


# ------------------------------------------------------------------ invariants

@pytest.mark.parametrize("bc", [0, 1])
def test_initial_moments_return_rho0_and_u0(bc):
    """Eq. (6): rho v = sum e f + F/2.  The initial state is built so that the
    velocity of the moments at t = 0 is the requested u0 (not u0 + F / (2 rho0))."""
    w = W.stationary_droplet(n=40, R0=11.0)
    p = dict(w.params, bc=bc)
    rng = np.random.default_rng(7)
    ux0 = 0.01 * rng.standard_normal(w.rho0.shape)
    uy0 = 0.01 * rng.standard_normal(w.rho0.shape)
    s = state(p, w.rho0, ux0, uy0)
    rho, ux, uy, Fx, Fy, _ = s.moments()
    assert np.abs(rho - w.rho0).max() < 1e-15
    assert np.abs(ux - ux0).max() < 1e-14 and np.abs(uy - uy0).max() < 1e-14
    # the force is far from zero across the interface, so the correction is not vacuous
    assert np.abs(Fx / (2 * rho)).max() > 1e-3
    # the distributions themselves are the equilibria at u_eq = u0 - F / (2 rho0)
    jx, jy = (s.f * EX[:, None, None]).sum(0), (s.f * EY[:, None, None]).sum(0)
    assert np.abs(jx - (w.rho0 * ux0 - Fx / 2)).max() < 1e-14
    assert np.abs(jy - (w.rho0 * uy0 - Fy / 2)).max() < 1e-14


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("rho", [0.4, 0.01])
def test_uniform_state_stays_at_equilibrium(bc, rho):
    p = W.base_params(24, 16, bc=bc)
    s = state(p, np.full((16, 24), rho))
    s.step(1000)
    r, ux, uy, Fx, Fy, _ = s.moments()
    assert np.abs(r - rho).max() <= 1e-15 * max(1.0, rho * 10)
    assert np.abs(ux).max() <= 1e-15 and np.abs(uy).max() <= 1e-15
    assert np.abs(Fx).max() == 0.0 and np.abs(Fy).max() == 0.0


@pytest.mark.parametrize("case", ["droplet", "splash_walls"])
def test_mass_is_conserved(case):
    if case == "droplet":
        w = W.stationary_droplet(n=48, R0=12)
        n = 3000
    else:
        w = W.splash(nx=64, ny=48, Re=200)
        n = 1500
    s = state(w.params, w.rho0, w.ux0, w.uy0)
    m0 = s.f.sum()
    s.step(n)
    assert abs(s.f.sum() - m0) / m0 <= 1e-12


def test_momentum_is_conserved_periodic():
    """Sum_x sum_a e_a f changes by sum_x F per step, and the pairwise stencil of Eq. (7)
    makes sum_x F vanish on a periodic lattice."""
    rng = np.random.default_rng(11)
    w = W.stationary_droplet(n=40, R0=9)
    rho0 = w.rho0 * (1 + 0.01 * rng.standard_normal(w.rho0.shape))
    ux0 = 0.01 * rng.standard_normal(rho0.shape)
    uy0 = 0.01 * rng.standard_normal(rho0.shape)
    s = state(w.params, rho0, ux0, uy0)
    _, _, _, Fx, Fy, _ = s.moments()
    assert abs(Fx.sum()) < 1e-14 and abs(Fy.sum()) < 1e-14
    p0 = momentum(s.f)
    s.step(500)
    p1 = momentum(s.f)
    scale = s.f.sum() * 0.01
    assert abs(p1[0] - p0[0]) <= 1e-12 * scale and abs(p1[1] - p0[1]) <= 1e-12 * scale


def test_translation_invariance_is_exact():
    w = W.stationary_droplet(n=36, R0=8)
    rng = np.random.default_rng(5)
    rho0 = w.rho0 * (1 + 0.02 * rng.random(w.rho0.shape))
    a = state(w.params, rho0).step(200).moments()[0]
    b = state(w.params, np.roll(rho0, (7, -11), axis=(0, 1))).step(200).moments()[0]
    assert np.array_equal(np.roll(a, (7, -11), axis=(0, 1)), b)


def test_centred_droplet_keeps_d4_symmetry():
    w = W.stationary_droplet(n=50, R0=11)
    r = state(w.params, w.rho0).step(1000).moments()[0]
    for sym in (r[:, ::-1], r[::-1, :], r.T):
        assert np.abs(r - sym).max() <= 1e-13


@pytest.mark.parametrize("shape,bc", [((4, 4), 0), ((3, 5), 0), ((5, 4), 1), ((6, 3), 1)])
def test_moment_form_equals_velocity_form_on_tiny_grids(shape, bc):
    """Eq. (4) path and the dense Eq. (1) path give the same trajectory."""
    ny, nx = shape
    rng = np.random.default_rng(ny * 10 + nx)
    p = W.base_params(nx, ny, bc=bc, t_over_tc=0.8)
    p.update(s_rho=0.9, s_j=1.3, s_q=1.2, s_e=0.7, s_zeta=1.4, nu_l=0.05, nu_g=0.2)
    rho0 = 0.05 + 0.3 * rng.random((ny, nx))
    ux0, uy0 = 0.02 * rng.standard_normal((2, ny, nx))
    a = state(p, rho0, ux0, uy0)
    b = state(p, rho0, ux0, uy0)
    a.step(30, O.FORM_MOMENT)
    b.step(30, O.FORM_VELOCITY)
    assert np.abs(a.f - b.f).max() <= 1e-13


@pytest.mark.parametrize("bc", [0, 1])
def test_collide_at_then_stream_equals_the_full_step(bc):
    """lbref_collide_at (the one-step reference of the GPU parity tests) evaluates
    psi, the Eq. (7) force, the Eq. (6) velocity and the Eq. (4) collision from each
    site's own 3 x 3 neighbourhood, with its own wall clamp.  Collided at every site and
    streamed (Eq. 5), it must reproduce lbref_step exactly, wall rows 0 and ny-1
    included.  A perturbed droplet with random velocities exercises every term."""
    nx, ny = 23, 17
    rl, rg = W.coexistence(0.6)
    p = W.base_params(nx, ny, bc=bc)
    rng = np.random.default_rng(3 + bc)
    rho0 = W.droplet_field(nx, ny, 6.0, rl, rg, periodic_y=(bc == 0)) * (1 + 0.02 * rng.random((ny, nx)))
    ux0, uy0 = 0.02 * rng.standard_normal((2, ny, nx))
    P = O.Params(**p)
    s = O.State(P, rho0, ux0, uy0).step(7)
    fstar = O.collide_at(P, s.f, np.arange(nx * ny)).T.reshape(9, ny, nx)
    streamed = O.stream(P, fstar)
    s.step(1)
    assert np.abs(streamed - s.f).max() <= 1e-15
    # the wall rows are where collide_at's clamp and the streaming's reflection act
    assert np.abs(s.f[:, [0, ny - 1], :]).min() > 0.0


# ------------------------------------------------------------------ transport: rates and walls

@pytest.mark.parametrize("rho,nu", [(0.4, 0.1), (0.01, 0.3)])
def test_shear_wave_decays_at_the_set_viscosity(rho, nu):
    """Eq. (10): nu = (1/s_nu - 1/2)/3, with nu switched by density (Sec. IV.C).
    u_x = U sin(k y) decays as exp(-nu k^2 t)."""
    nx, ny, U = 4, 64, 1e-3
    p = W.base_params(nx, ny, nu_l=0.1, nu_g=0.3)
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    s = state(p, np.full((ny, nx), rho), U * np.sin(2 * np.pi * y / ny), np.zeros((ny, nx)))
    ts, amps = [], []
    basis = np.sin(2 * np.pi * np.arange(ny) / ny)
    for _ in range(20):
        s.step(100)
        amps.append((s.moments()[1][:, 0] * basis).sum() * 2 / ny)
        ts.append(s.t)
    rate = -np.polyfit(ts[3:], np.log(amps[3:]), 1)[0]
    assert rate == pytest.approx(nu * (2 * np.pi / ny) ** 2, rel=3e-3)


def test_halfway_bounce_back_walls_sit_half_a_cell_out():
    """With walls at y = -1/2 and ny - 1/2 the no-slip mode U sin(pi (y + 1/2)/ny)
    decays as exp(-nu (pi/ny)^2 t)."""
    nx, ny, U = 4, 32, 1e-4
    p = W.base_params(nx, ny, bc=1, nu_l=0.1, nu_g=0.1)
    yc = (np.arange(ny) + 0.5)[:, None] * np.ones((1, nx))
    s = state(p, np.full((ny, nx), 0.4), U * np.sin(np.pi * yc / ny), np.zeros((ny, nx)))
    basis = np.sin(np.pi * (np.arange(ny) + 0.5) / ny)
    ts, amps = [], []
    for _ in range(30):
        s.step(100)
        amps.append((s.moments()[1][:, 0] * basis).sum() * 2 / ny)
        ts.append(s.t)
    rate = -np.polyfit(ts[5:], np.log(amps[5:]), 1)[0]
    assert rate == pytest.approx(0.1 * (np.pi / ny) ** 2, rel=3e-3)


def test_film_on_wall_stays_flat():
    """A flat liquid film on the bottom wall (walls in y) stays uniform in x and at rest."""
    nx, ny = 8, 60
    p = W.base_params(nx, ny, a=0.25, t_over_tc=0.6, bc=1)
    rl, rg = W.coexistence(0.6)
    rho0 = np.broadcast_to(W.tanh_profile(np.arange(ny)[:, None] - 20.0, rl, rg), (ny, nx)).copy()
    s = state(p, rho0)
    m0 = s.f.sum()
    s.step(3000)
    r, ux, uy, *_ = s.moments()
    assert np.abs(r - r[:, :1]).max() <= 1e-13
    assert np.abs(ux).max() <= 1e-13
    assert np.abs(uy).max() <= 5e-3  # spurious current at the interface only
    assert abs(s.f.sum() - m0) / m0 <= 1e-12


# ------------------------------------------------------------------ thermodynamics: Eqs. 21, 22, 29

def flat_interface(a, tb, sigma, steps=30000, nx=4, ny=200):
    p = W.base_params(nx, ny, a=a, t_over_tc=tb, sigma=sigma, nu_l=0.1, nu_g=0.1)
    rl, rg = W.coexistence(tb)
    s = state(p, W.slab_field(nx, ny, ny / 2, rl, rg))
    s.step(steps)
    r = s.moments()[0][:, 0]
    return r[ny // 2], r[0], p


@pytest.mark.parametrize("tb,sigma", [(0.85, 0.0), (0.85, 0.11), (0.8, 0.0), (0.8, 0.11)])
def test_flat_interface_matches_mechanical_stability_theory(tb, sigma):
    """Near T_c, where the interface is wide, the LB coexistence densities follow the
    mechanical-stability condition Eq. (21) with epsilon = -2(alpha + 24 G sigma)/beta
    (Eq. 29): this pins the force stencil, Eq. (24) and the improved term together."""
    rl, rg, p = flat_interface(0.5, tb, sigma)
    tl, tg = eos.mechanical_stability(p["T"], 0.5, eos.epsilon_of_sigma(sigma))
    assert rl == pytest.approx(tl, rel=1e-3)
    assert rg == pytest.approx(tg, rel=1e-2)


def test_improved_forcing_restores_maxwell_vapour_branch():
    """Sec. IV.A / Fig. 1: the original forcing (sigma = 0) misses the Maxwell vapour
    density badly; the improved one (sigma = 0.11) agrees closely."""
    rl0, rg0, p = flat_interface(0.5, 0.85, 0.0)
    rl1, rg1, _ = flat_interface(0.5, 0.85, 0.11)
    ml, mg = eos.maxwell(p["T"], 0.5)
    assert abs(rg0 / mg - 1) > 0.3
    assert rg1 == pytest.approx(mg, rel=0.03)
    assert rl1 == pytest.approx(ml, rel=1e-3)


@functools.lru_cache(maxsize=None)
def droplet_coexistence(tb, R0, steps, n=None):
    """Inner and outer mean densities of a stationary droplet (Sec. IV.A geometry:
    periodic n x n box, n = 4 R0 by default, tanh start, tau_nu = 0.8, a = 0.5)."""
    w = W.coexistence_droplets([tb], tau_nu=0.8, n=int(n or 4 * R0), R0=float(R0))[0]
    s = state(w.params, w.rho0).step(steps)
    lp = post.laplace(s.moments()[0], w.params, float(R0))
    return lp["rho_in"], lp["rho_out"]


@pytest.mark.slow
def test_table2_row_at_reduced_temperature_0_6_in_the_droplet_geometry(golden):
    """Table II, a = 0.5, sigma = 0.11, tau_nu = 0.8, T/Tc = 0.6, measured as the paper
    measures it (Sec. IV.A-B): a droplet of radius 50 in a 200 x 200 periodic box.  The
    inner and outer densities after 12,000 steps reproduce the printed 0.4077 / 0.00298
    (to 0.02 % and 0.1 %; they are converged to 1e-4 by then)."""
    row = golden["table2"]["rows"][0]
    rl, rg = droplet_coexistence(0.6, 50, 12000)
    assert rl == pytest.approx(row[1], rel=2e-3)
    assert rg == pytest.approx(row[2], rel=3e-2)


@pytest.mark.slow
def test_vapour_density_shifts_with_curvature():
    """Why a flat interface does not reproduce Table II's vapour density: the outer
    density of a droplet sits above the flat-interface value by an amount proportional
    to the curvature 1/R (the Laplace pressure of the droplet, Sec. IV.B).  With the
    flat slab as the R -> infinity limit, halving the radius doubles the shift, and the
    flat value itself lies clearly below the droplet's (by about 15 % at R = 50)."""
    rl_f, rg_f, _ = flat_interface(0.5, 0.6, 0.11)
    _, rg25 = droplet_coexistence(0.6, 25, 12000)
    _, rg50 = droplet_coexistence(0.6, 50, 12000)
    assert (rg25 - rg_f) / (rg50 - rg_f) == pytest.approx(2.0, rel=0.1)
    assert rg50 / rg_f - 1.0 > 0.1


def test_interface_width_scales_as_inverse_sqrt_a(golden):
    """Sec. IV.B / Fig. 3: widths for a = 0.25 and 0.5 are about 1.9 and 1.4 times the
    a = 1.0 width, flat interfaces at T/Tc = 0.7 and 0.6, with the width taken as the W
    of the best Eq. (31) tanh fit.  The 10-90 % width (post.interface_width) of the same
    interfaces lies 0-12 % above W ln 3 (its value for an exact tanh): linear
    interpolation across an interface only ~3 sites wide (a = 1) and the longer
    vapour-side tail inflate it, so its ratios come out lower and are only reported."""
    g = golden["interface_width_ratio"]

    def width(a, tb):
        nx, ny = 4, 200
        p = W.base_params(nx, ny, a=a, t_over_tc=tb, nu_l=0.1, nu_g=0.1)
        rl, rg = W.coexistence(tb)
        s = state(p, W.slab_field(nx, ny, ny / 2, rl, rg))
        s.step(20000)
        r = s.moments()[0][: ny // 2, 0]
        f = lambda y, yc, Wd, l, gg: 0.5 * (l + gg) + 0.5 * (l - gg) * np.tanh(2 * (y - yc) / Wd)
        popt, _ = curve_fit(f, np.arange(ny // 2, dtype=float), r, p0=[ny / 4, 4, r.max(), r.min()])
        # scanned from the liquid side
        return abs(popt[1]), post.interface_width(r[::-1], r.max(), r.min())

    for tb in (0.7, 0.6):
        w1, w05, w025 = width(1.0, tb), width(0.5, tb), width(0.25, tb)
        assert w05[0] / w1[0] == pytest.approx(g["a0.5_over_a1"], rel=0.1)
        assert w025[0] / w1[0] == pytest.approx(g["a0.25_over_a1"], rel=0.1)
        print(f"T/Tc={tb}: 10-90 width ratios {w05[1] / w1[1]:.3f} {w025[1] / w1[1]:.3f}")
        for w in (w1, w05, w025):
            assert 1.0 <= w[1] / (w[0] * math.log(3.0)) <= 1.12


@pytest.mark.slow
def test_laplace_law():
    """Pressure jump of equilibrated droplets against 1/R (2-D Laplace law, which the
    paper uses in Sec. IV.B and IV.C to evaluate the surface tension): 128 x 128
    periodic, R0 = 15 ... 35, T/Tc = 0.6, a = 0.5, 16,000 steps (the fit's intercept
    moves by 0.1 % of max Delta p between 16,000 and 40,000 steps).  The straight line in 1/R_eff
    has R^2 >= 0.9995; its intercept (3 % of the largest Delta p) is the second-order
    term of a finite-width interface, Delta p = theta/R (1 - 2 delta/R): fitting
    c + s/R + q/R^2 leaves no constant pressure offset (|c| <= 1 % of max Delta p)."""
    xs, ys = [], []
    for R0 in (15, 20, 25, 30, 35):
        w = W.stationary_droplet(n=128, R0=R0)
        s = state(w.params, w.rho0).step(16000)
        lp = post.laplace(s.moments()[0], w.params, R0)
        xs.append(1 / lp["R_eff"])
        ys.append(lp["dp"])
    slope, icpt, r2 = post.linear_fit(xs, ys)
    assert slope > 0 and r2 >= 0.9995
    x, y = np.array(xs), np.array(ys)
    A = np.vstack([np.ones_like(x), x, x * x]).T
    (c, s1, q), *_ = np.linalg.lstsq(A, y, rcond=None)
    assert s1 > 0 and q < 0
    assert abs(c) <= 0.01 * y.max()
    assert np.abs(A @ np.array([c, s1, q]) - y).max() <= 1e-3 * y.max()


def _disc_count(n_x, n_y, cx2, cy2, r2x4, periodic_y, strict):
    """Number of lattice sites (i, j) with |2 (i, j) - (cx2, cy2)|^2 < r2x4 (or <=), all in
    integers: cx2 = 2 cx, cy2 = 2 cy and r2x4 = 4 r^2; minimum image in x (and y)."""
    count = 0
    for j in range(n_y):
        dy = abs(2 * j - cy2)
        if periodic_y:
            dy = min(dy, 2 * n_y - dy)
        for i in range(n_x):
            dx = abs(2 * i - cx2)
            dx = min(dx, 2 * n_x - dx)
            q = dx * dx + dy * dy
            count += (q < r2x4) if strict else (q <= r2x4)
    return count


@pytest.mark.parametrize("bc,cx,cy", [(0, 63.5, 63.5), (0, 10.5, 120.0), (1, 70.0, 47.5)])
def test_laplace_post_processing_on_a_stepped_disc(bc, cx, cy):
    """post.laplace on a field whose answers are known exactly: density rho_a on a disc of
    radius 20, rho_b on the annulus 20 <= d < 33 and rho_c beyond.  Then p_in and p_out
    are p_EOS(rho_a) and p_EOS(rho_c) (evaluated by the C oracle, Eq. 30), the region
    sizes are integer lattice-point counts (d <= R0/2 = 15 and d >= R0 + 3W = 45 for
    R0 = 30, W = 5), and R_eff^2 pi (rho_a - rho_c) is the excess mass N_a (rho_a - rho_c)
    + N_ab (rho_b - rho_c).  The two off-centre cases wrap around the periodic edges (and
    the walls case does not wrap in y)."""
    nx, ny = 128, 96
    p = W.base_params(nx, ny, bc=bc)
    ra, rb, rc = 0.41, 0.2, 0.003
    d = post.distance_field(nx, ny, cx, cy, periodic_y=(bc == 0))
    rho = np.where(d < 20.0, ra, np.where(d < 33.0, rb, rc))
    got = post.laplace(rho, p, 30.0, cx=cx, cy=cy)
    cx2, cy2 = int(round(2 * cx)), int(round(2 * cy))
    per = bc == 0
    n_in = _disc_count(nx, ny, cx2, cy2, 4 * 15 ** 2, per, strict=False)
    n_out = nx * ny - _disc_count(nx, ny, cx2, cy2, 4 * 45 ** 2, per, strict=True)
    n_a = _disc_count(nx, ny, cx2, cy2, 4 * 20 ** 2, per, strict=True)
    n_ab = _disc_count(nx, ny, cx2, cy2, 4 * 33 ** 2, per, strict=True) - n_a
    P = O.Params(**p)
    assert got["n_in"] == n_in and got["n_out"] == n_out
    assert got["p_in"] == pytest.approx(O.p_eos(P, ra), rel=1e-14)
    assert got["p_out"] == pytest.approx(O.p_eos(P, rc), rel=1e-14)
    assert got["rho_in"] == pytest.approx(ra, rel=1e-14) and got["rho_out"] == pytest.approx(rc, rel=1e-14)
    r_eff = math.sqrt((n_a * (ra - rc) + n_ab * (rb - rc)) / (math.pi * (ra - rc)))
    assert got["R_eff"] == pytest.approx(r_eff, rel=1e-12)
    # the mass-based radius of the plain disc is close to its geometric radius (Gauss circle)
    assert math.sqrt(n_a / math.pi) == pytest.approx(20.0, abs=0.1)
    assert got["dp"] == pytest.approx(O.p_eos(P, ra) - O.p_eos(P, rc), rel=1e-13)


@pytest.mark.parametrize("width", [5.0, 12.0])
def test_ten_ninety_width_of_a_tanh_profile(width):
    """post.interface_width on the Eq. (31) profile: its 10 % and 90 % points lie at
    d = -+ (W/2) artanh(0.8), so the 10-90 width is W artanh(0.8) = W ln 3 (up to the
    linear interpolation between lattice samples)."""
    rl, rg = 0.4, 0.003
    d = np.arange(-60.0, 60.0)
    prof = W.tanh_profile(d + 0.37, rl, rg, W=width)
    got = post.interface_width(prof, rl, rg)
    # linear interpolation over unit spacing moves a crossing by at most |phi''/phi'| / 8,
    # which is 3.2 / W where tanh = +-0.8; the two crossings' errors can add
    assert abs(got - width * math.log(3.0)) <= 0.8 / width


# ------------------------------------------------------------------ Eq. (23) pseudopotential

def ss_flat_interface(eps, G, sigma, steps=20000):
    ml, mg = eos.maxwell_ss(G, eps)
    w = W.ss_slab(G, eps, ml, mg, sigma=sigma)
    s = state(w.params, w.rho0)
    s.step(steps)
    r = s.moments()[0][:, 0]
    return r[w.params["ny"] // 2], r[0], (ml, mg)


def test_eq23_psi_with_original_forcing_follows_maxwell():
    """Sec. III.A: with the Eq. (23) psi at eps = 0 and the original forcing (sigma = 0,
    nearest-neighbour epsilon = 0), the mechanical-stability coexistence is the Maxwell
    construction of p = rho/3 + G psi^2 / 2.  Flat interface at G = 1.1 G_c."""
    G = 1.1 * eos.critical_ss(0.0)[1]
    rl, rg, (ml, mg) = ss_flat_interface(0.0, G, 0.0)
    assert rl == pytest.approx(ml, rel=1e-5)
    assert rg == pytest.approx(mg, rel=1e-5)


@pytest.mark.parametrize("eps", [0.5, 1.0])
def test_eq23_psi_improved_forcing_sets_epsilon(eps):
    """Eq. (29) with alpha = 0, beta = 3: epsilon = -16 G sigma.  Choosing
    sigma = -eps / (16 G) for the Eq. (23) psi of parameter eps makes the LB coexistence
    follow the Maxwell construction of its pressure (G = 1.2 G_c)."""
    G = 1.2 * eos.critical_ss(eps)[1]
    rl, rg, (ml, mg) = ss_flat_interface(eps, G, -eps / (16.0 * G))
    assert rl == pytest.approx(ml, rel=1e-3)
    assert rg == pytest.approx(mg, rel=1e-2)


def test_eq23_psi_with_original_forcing_follows_eq21_not_maxwell():
    """The same psi (eps = 1) with sigma = 0 follows Eq. (21) at epsilon = 0 and misses
    the Maxwell vapour density by about a quarter."""
    G = 1.2 * eos.critical_ss(1.0)[1]
    rl, rg, (ml, mg) = ss_flat_interface(1.0, G, 0.0)
    tl, tg = eos.mechanical_stability_ss(G, 1.0, 0.0)
    assert rl == pytest.approx(tl, rel=1e-3)
    assert rg == pytest.approx(tg, rel=2e-3)
    assert abs(rg / mg - 1) > 0.2
