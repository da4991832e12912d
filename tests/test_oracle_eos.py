"""Pins of the oracle's thermodynamics (oracle/eos.py) against what the paper prints
and against closed forms.  CPU only."""
import math

import numpy as np
import pytest

from oracle import eos

TC_PER_A = 0.094  # the paper's rounded T_c for a = 1 (Sec. IV.A), 0.5 and 0.25 (Sec. IV.C)


def test_critical_constants_match_printed(golden):
    g = golden["critical_constants"]
    for a, b in [(1.0, 4.0), (0.5, 4.0), (0.25, 4.0), (1.0, 2.0)]:
        rho_c, T_c, p_c = eos.critical_point(a, b, 1.0)
        assert rho_c * b == pytest.approx(g["rho_c_times_b"], rel=1e-3)
        # a = 10.601 R T_c is printed for b = 4; it scales as b (a/b = 2.650 R T_c)
        assert a / T_c * 4.0 / b == pytest.approx(g["a_over_R_Tc"], rel=1e-3)
        assert p_c * b * b / a == pytest.approx(g["pc_b2_over_a"], rel=1e-3)
        # Sec. IV.A: a = 0.4963 R^2 T_c^2 / p_c and b = 0.18727 R T_c / p_c
        assert a == pytest.approx(0.4963 * T_c ** 2 / p_c, rel=1e-3)
        assert b == pytest.approx(0.18727 * T_c / p_c, rel=1e-3)
        # the critical point is an inflection with zero slope
        assert abs(eos.dp_drho(rho_c, a, b, 1.0, T_c)) < 1e-12
        assert abs(eos.d2p_drho2(rho_c, a, b, 1.0, T_c)) < 1e-9


def test_eos_matches_nondimensional_form_B3():
    """Eq. (30) against Eq. (33)/(B3) with the paper's rounded constants."""
    for a in (1.0, 0.5, 0.25):
        _, T_c, p_c = eos.critical_point(a)
        T = 0.6 * T_c
        rho = np.linspace(1e-4, 0.6, 200)
        p30 = eos.p_eos(rho, a, 4.0, 1.0, T)
        pB3 = eos.p_eos_nondim_B3(rho, a, 4.0, 1.0, T, T_c)
        scale = np.abs(eos.p_eos(rho, a, 4.0, 1.0, 0.0)).max()  # a rho^2 magnitude
        assert np.abs(p30 - pB3).max() <= 2e-3 * scale


def test_derivatives_against_finite_differences():
    a, T = 0.5, 0.6 * 0.047
    for r in (0.003, 0.05, 0.13, 0.3, 0.45):
        h = 1e-6
        fd1 = (eos.p_eos(r + h, a, T=T) - eos.p_eos(r - h, a, T=T)) / (2 * h)
        fd2 = (eos.p_eos(r + h, a, T=T) - 2 * eos.p_eos(r, a, T=T) + eos.p_eos(r - h, a, T=T)) / h ** 2
        assert eos.dp_drho(r, a, T=T) == pytest.approx(fd1, rel=1e-7, abs=1e-12)
        assert eos.d2p_drho2(r, a, T=T) == pytest.approx(fd2, rel=1e-3, abs=1e-6)


def test_maxwell_reproduces_table2_maxwell_column(golden):
    """Table II Maxwell column with T_c = 0.094 a (the paper's rounded critical temperature)."""
    for row in golden["table2"]["rows"]:
        tb, rl_p, rg_p = row[0], row[5], row[6]
        for a in (0.5, 0.25):
            rl, rg = eos.maxwell(tb * TC_PER_A * a, a)
            assert rl == pytest.approx(rl_p, rel=5e-3)
            assert rg == pytest.approx(rg_p, rel=5e-3)


def test_maxwell_density_ratio_matches_table1(golden):
    for row in golden["table1"]["rows"]:
        rl, rg = eos.maxwell(row[0] * TC_PER_A * 0.5, 0.5)
        assert rl / rg == pytest.approx(row[1], rel=5e-3)


def test_maxwell_equal_pressure_and_chemical_potential():
    """Equal-area rule <=> equal pressure and equal chemical potential.  The chemical
    potential of Eq. (30) in closed form: mu = R T [ln rho + (8 eta - 9 eta^2 + 3 eta^3)/(1-eta)^3] - 2 a rho
    (checked independently of the quadrature used by eos.maxwell)."""
    def mu(r, a, b, R, T):
        eta = b * r / 4.0
        return R * T * (math.log(r) + (8 * eta - 9 * eta ** 2 + 3 * eta ** 3) / (1 - eta) ** 3) - 2 * a * r

    for a, tb in [(0.5, 0.6), (0.25, 0.45), (1.0, 0.85), (0.5, 0.5)]:
        T = tb * TC_PER_A * a
        rl, rg = eos.maxwell(T, a)
        pl, pg = eos.p_eos(rl, a, T=T), eos.p_eos(rg, a, T=T)
        assert abs(pl - pg) <= 1e-10 * abs(pl)
        assert mu(rl, a, 4.0, 1.0, T) == pytest.approx(mu(rg, a, 4.0, 1.0, T), abs=1e-10 * a)
        # closed-form mu derivative check: d mu/d rho = (dp/drho)/rho
        r, h = 0.2, 1e-6
        dmu = (mu(r + h, a, 4.0, 1.0, T) - mu(r - h, a, 4.0, 1.0, T)) / (2 * h)
        assert dmu == pytest.approx(eos.dp_drho(r, a, T=T) / r, rel=1e-6)


def test_maxwell_depends_only_on_reduced_temperature():
    rl1, rg1 = eos.maxwell(0.6 * TC_PER_A * 1.0, 1.0)
    rl2, rg2 = eos.maxwell(0.6 * TC_PER_A * 0.25, 0.25)
    assert rl1 == pytest.approx(rl2, rel=1e-9)
    assert rg1 == pytest.approx(rg2, rel=1e-7)


def test_epsilon_of_sigma(golden):
    for s, e in golden["epsilon_of_sigma"]["pairs"]:
        assert eos.epsilon_of_sigma(s) == pytest.approx(e, abs=1e-12)
    assert eos.epsilon_of_sigma(0.0) == 0.0


def test_mechanical_stability_equal_pressure_and_sigma0_limit():
    """Eq. (21) roots share the pressure; with epsilon = 0 the original scheme's vapour
    density lies far below Maxwell at T/Tc = 0.85 (the inconsistency Sec. III.A describes),
    and epsilon = 1.76 moves it much closer."""
    a, tb = 0.5, 0.85
    T = tb * 0.047
    rl0, rg0 = eos.mechanical_stability(T, a, 0.0)
    rl1, rg1 = eos.mechanical_stability(T, a, 1.76)
    rlm, rgm = eos.maxwell(T, a)
    assert eos.p_eos(rl0, a, T=T) == pytest.approx(eos.p_eos(rg0, a, T=T), rel=1e-9)
    assert abs(rg0 - rgm) / rgm > 0.2
    assert abs(rg1 - rgm) < abs(rg0 - rgm)


def test_psi_of_eq24_is_real_over_the_droplet_range():
    a, T = 0.5, 0.6 * 0.047
    rho = np.linspace(1e-5, 0.55, 500)
    s = eos.psi(rho, a, T=T)
    assert np.all(np.isfinite(s)) and np.all(s > 0)


def test_lamb_period_formula(golden):
    """Eq. (32) with n = 2: T = 2 pi sqrt(rho_l R0^3 / (6 theta)); invert at the printed period."""
    T_a = golden["lamb"]["analytical"]
    rho_l, R0 = 0.455, math.sqrt(30 * 27)
    theta = 4 * math.pi ** 2 * rho_l * R0 ** 3 / (6 * T_a ** 2)
    assert eos.lamb_period(theta, rho_l, R0) == pytest.approx(T_a, rel=1e-12)


# ------------------------------------------------------------------ Eq. (23) pseudopotential

def test_eq23_critical_points_closed_forms():
    """p = rho/3 + G psi^2 / 2 with the Eq. (23) psi.  By hand: eps = 0 gives
    p' = 1/3 + G exp(-2/rho) / rho^2, stationary slope at rho = 1, G_c = -e^2/3;
    eps = 1 gives p' = 1/3 + G rho / (1 + rho)^3, maximal rho/(1+rho)^3 = 4/27 at
    rho = 1/2, G_c = -9/4."""
    rc0, gc0 = eos.critical_ss(0.0)
    rc1, gc1 = eos.critical_ss(1.0)
    assert rc0 == 1.0 and gc0 == pytest.approx(-math.e ** 2 / 3.0, rel=1e-14)
    assert rc1 == 0.5 and gc1 == pytest.approx(-9.0 / 4.0, rel=1e-14)
    for eps, rc, gc in ((0.0, rc0, gc0), (1.0, rc1, gc1), (0.5, *eos.critical_ss(0.5))):
        h = 1e-4
        d1 = (eos.p_ss(rc + h, gc, eps) - eos.p_ss(rc - h, gc, eps)) / (2 * h)
        d2 = (eos.p_ss(rc + h, gc, eps) - 2 * eos.p_ss(rc, gc, eps) + eos.p_ss(rc - h, gc, eps)) / h ** 2
        assert abs(d1) < 1e-8 and abs(d2) < 1e-5


def test_eq23_psi_limit_derivative_and_consistency_identity():
    """Eq. (23): the eps -> 0 limit is exp(-1/rho), and psi' / psi^(1+eps) = 1 / rho^2
    (the property the paper states), checked with finite differences of psi."""
    rho = np.array([0.05, 0.3, 1.0, 2.5])
    assert np.allclose(eos.psi_ss(rho, 1e-8), np.exp(-1.0 / rho), rtol=1e-6)
    for eps in (0.0, 0.5, 1.0, 10.0 / 31.0):
        h = 1e-6 * rho
        fd = (eos.psi_ss(rho + h, eps) - eos.psi_ss(rho - h, eps)) / (2 * h)
        assert np.allclose(eos.dpsi_ss(rho, eps), fd, rtol=1e-7)
        assert np.allclose(fd / eos.psi_ss(rho, eps) ** (1.0 + eps), 1.0 / rho ** 2, rtol=1e-7)


def test_eq23_maxwell_equal_pressure_and_chemical_potential():
    """The equal-area rule for p = rho/3 + G psi^2 / 2 <=> equal pressure and equal
    chemical potential, mu' = p'/rho.  Closed forms by hand:
      eps = 0: mu = ln(rho)/3 + G (1/(2 rho) + 1/4) exp(-2/rho);
      eps = 1: mu = ln(rho)/3 - G / (2 (1 + rho)^2)."""
    mu = {0.0: lambda r, G: math.log(r) / 3 + G * (0.5 / r + 0.25) * math.exp(-2.0 / r),
          1.0: lambda r, G: math.log(r) / 3 - G / (2.0 * (1.0 + r) ** 2)}
    for eps in (0.0, 1.0):
        _, gc = eos.critical_ss(eps)
        for f in (1.1, 1.3):
            G = f * gc
            rl, rg = eos.maxwell_ss(G, eps)
            assert rl > 1.5 * rg
            assert eos.p_ss(rl, G, eps) == pytest.approx(eos.p_ss(rg, G, eps), rel=1e-10)
            assert mu[eps](rl, G) == pytest.approx(mu[eps](rg, G), abs=1e-10)


def test_eq23_mechanical_stability_is_maxwell_when_epsilons_match():
    """Eq. (21) with the Eq. (23) psi of parameter eps reduces to Eq. (22) when the
    stencil/forcing epsilon equals eps; with epsilon = 0 it does not (eps = 1)."""
    for eps in (0.0, 0.5, 1.0):
        G = 1.2 * eos.critical_ss(eps)[1]
        ml, mg = eos.maxwell_ss(G, eps)
        tl, tg = eos.mechanical_stability_ss(G, eps, eps)
        assert tl == pytest.approx(ml, rel=1e-7) and tg == pytest.approx(mg, rel=1e-7)
    G = 1.2 * eos.critical_ss(1.0)[1]
    tl, tg = eos.mechanical_stability_ss(G, 1.0, 0.0)
    ml, mg = eos.maxwell_ss(G, 1.0)
    assert eos.p_ss(tl, G, 1.0) == pytest.approx(eos.p_ss(tg, G, 1.0), rel=1e-10)
    assert abs(tg / mg - 1) > 0.2


def test_eq23_c_oracle_matches_python():
    """The C oracle's Eq. (23) psi^2 and bulk pressure against this module's."""
    from oracle import lbref as O
    for eps in (0.0, 1.0, 10.0 / 31.0):
        p = O.Params(nx=4, ny=4, G=-2.7, psi_form=O.PSI_SS, psi_eps=eps)
        for r in (0.07, 0.4, 1.9):
            assert O.psi2(p, r) == pytest.approx(float(eos.psi_ss(r, eps)) ** 2, rel=1e-13)
            assert O.pressure(p, r) == pytest.approx(float(eos.p_ss(r, -2.7, eps)), rel=1e-12)
