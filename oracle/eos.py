"""Thermodynamics of the Carnahan-Starling pseudopotential model, FP64.

TEST INFRASTRUCTURE ONLY (oracle).  Plain NumPy/SciPy, no GPU code.

Implements, from the paper (Li, Luo & Li):
  * Eq. (30)      Carnahan-Starling equation of state p_EOS(rho);
  * Sec. IV.A     critical point (rho_c ~ 0.5218/b, a = 10.601 R T_c);
  * Eq. (33)/(B3) the non-dimensional form of the EOS (used only as a pin);
  * Eq. (22)      Maxwell equal-area construction for the coexistence densities;
  * Eq. (24)      pseudopotential psi(rho) derived from the EOS;
  * Eq. (21)      mechanical-stability coexistence for a given epsilon;
  * Eq. (29)      epsilon = -2 (alpha + 24 G sigma) / beta of the improved forcing;
  * Eq. (23)      the Sbragaglia-Shan pseudopotential and the bulk pressure it implies,
                  p = rho c_s^2 + G psi^2 / 2 (the bulk term of Eqs. (19)-(21)), with
                  its critical point, Maxwell construction and Eq. (21) coexistence.
"""
from __future__ import annotations

import math
import warnings

import numpy as np
from scipy import integrate, optimize

# quad reports round-off near its requested tolerance; the roots are checked by the tests.
warnings.filterwarnings("ignore", category=integrate.IntegrationWarning)

CS2 = 1.0 / 3.0  # c_s^2 with c = 1 (Sec. II)


def p_eos(rho, a, b=4.0, R=1.0, T=0.0282):
    """Eq. (30): p = rho R T (1 + eta + eta^2 - eta^3) / (1 - eta)^3 - a rho^2, eta = b rho / 4."""
    rho = np.asarray(rho, dtype=np.float64)
    eta = b * rho / 4.0
    return rho * R * T * (1.0 + eta + eta ** 2 - eta ** 3) / (1.0 - eta) ** 3 - a * rho ** 2


def dp_drho(rho, a, b=4.0, R=1.0, T=0.0282):
    """First density derivative of Eq. (30), written out by hand.

    With h(rho) = rho Z(eta), Z = N/D, N = 1 + eta + eta^2 - eta^3, D = (1 - eta)^3:
    dZ/deta = (4 + 4 eta - 2 eta^2) / (1 - eta)^4, so dh/drho = Z + eta dZ/deta.
    """
    eta = b * np.asarray(rho, dtype=np.float64) / 4.0
    Z = (1.0 + eta + eta ** 2 - eta ** 3) / (1.0 - eta) ** 3
    dZ = (4.0 + 4.0 * eta - 2.0 * eta ** 2) / (1.0 - eta) ** 4
    return R * T * (Z + eta * dZ) - 2.0 * a * rho


def d2p_drho2(rho, a, b=4.0, R=1.0, T=0.0282):
    """Second density derivative of Eq. (30): d2h/drho2 = (b/4)(2 dZ/deta + eta d2Z/deta2)."""
    eta = b * np.asarray(rho, dtype=np.float64) / 4.0
    dZ = (4.0 + 4.0 * eta - 2.0 * eta ** 2) / (1.0 - eta) ** 4
    d2Z = (20.0 + 8.0 * eta - 4.0 * eta ** 2) / (1.0 - eta) ** 5
    return R * T * (b / 4.0) * (2.0 * dZ + eta * d2Z) - 2.0 * a


def critical_point(a, b=4.0, R=1.0):
    """Critical point of Eq. (30): dp/drho = d2p/drho2 = 0.  Returns (rho_c, T_c, p_c).

    Eliminating R T between the two conditions leaves one equation in rho:
    rho h''(rho) = h'(rho); then R T_c = 2 a / h''(rho_c).
    """
    def h1(r):
        eta = b * r / 4.0
        Z = (1.0 + eta + eta ** 2 - eta ** 3) / (1.0 - eta) ** 3
        dZ = (4.0 + 4.0 * eta - 2.0 * eta ** 2) / (1.0 - eta) ** 4
        return Z + eta * dZ

    def h2(r):
        eta = b * r / 4.0
        dZ = (4.0 + 4.0 * eta - 2.0 * eta ** 2) / (1.0 - eta) ** 4
        d2Z = (20.0 + 8.0 * eta - 4.0 * eta ** 2) / (1.0 - eta) ** 5
        return (b / 4.0) * (2.0 * dZ + eta * d2Z)

    rho_c = optimize.brentq(lambda r: r * h2(r) - h1(r), 1e-6 / b, 3.9 / b, xtol=1e-15, rtol=1e-15)
    T_c = 2.0 * a / (R * h2(rho_c))
    p_c = float(p_eos(rho_c, a, b, R, T_c))
    return rho_c, T_c, p_c


def p_eos_nondim_B3(rho, a, b, R, T, T_c):
    """Eq. (33)/(B3) with the paper's rounded constants (0.13045, 1.3829, 2.786, 0.070663)."""
    rho_c = 0.5218 / b
    p_c = 0.070663 * a / b ** 2
    rb = np.asarray(rho, dtype=np.float64) / rho_c
    Tb = T / T_c
    x = 0.13045 * rb
    return 2.786 * p_c * rb * (Tb * (1 + x + x ** 2 - x ** 3) / (1 - x) ** 3 - 1.3829 * rb)


def spinodals(a, b=4.0, R=1.0, T=0.0282):
    """Local maximum (vapour side) and local minimum (liquid side) of p(rho) for T < T_c."""
    rho_c, T_c, _ = critical_point(a, b, R)
    if T >= T_c:
        raise ValueError("T must be below the critical temperature")
    f = lambda r: dp_drho(r, a, b, R, T)
    r_hi = 3.999 / b
    rg = optimize.brentq(f, 1e-12, rho_c, xtol=1e-16, rtol=1e-15)
    rl = optimize.brentq(f, rho_c, r_hi * 0.999, xtol=1e-16, rtol=1e-15)
    return rg, rl


def _roots_at_pressure(p0, a, b, R, T, rs_g, rs_l):
    g = lambda r: float(p_eos(r, a, b, R, T)) - p0
    rg = optimize.brentq(g, 1e-300, rs_g, xtol=1e-300, rtol=1e-15, maxiter=500)
    rl = optimize.brentq(g, rs_l, 3.9999999 / b, xtol=1e-16, rtol=1e-15, maxiter=500)
    return rg, rl


def maxwell(T, a, b=4.0, R=1.0):
    """Eq. (22): coexistence densities (rho_l, rho_g) from the equal-area rule.

    Finds p0 such that the vapour and liquid roots of p_EOS = p0 satisfy
    integral_{rho_g}^{rho_l} (p0 - p_EOS) / rho^2 d rho = 0 (adaptive quadrature).
    """
    rs_g, rs_l = spinodals(a, b, R, T)
    p_hi = float(p_eos(rs_g, a, b, R, T))
    p_lo = max(float(p_eos(rs_l, a, b, R, T)), 0.0)

    def area(p0):
        rg, rl = _roots_at_pressure(p0, a, b, R, T, rs_g, rs_l)
        val, _ = integrate.quad(lambda r: (p0 - float(p_eos(r, a, b, R, T))) / r ** 2, rg, rl,
                                points=[rs_g, rs_l], limit=400, epsabs=0.0, epsrel=1e-11)
        return val

    eps = 1e-14 * p_hi
    p0 = optimize.brentq(area, p_lo + eps, p_hi - eps, xtol=1e-18, rtol=1e-14, maxiter=500)
    rg, rl = _roots_at_pressure(p0, a, b, R, T, rs_g, rs_l)
    return rl, rg


def psi(rho, a, b=4.0, R=1.0, T=0.0282, G=-1.0):
    """Eq. (24) with c = 1: psi = sqrt(2 (p_EOS - rho c_s^2) / G)."""
    return np.sqrt(2.0 * (p_eos(rho, a, b, R, T) - CS2 * np.asarray(rho)) / G)


def epsilon_of_sigma(sigma, G=-1.0, alpha=0.0, beta=3.0):
    """Eq. (29): epsilon = -2 (alpha + 24 G sigma) / beta (nearest neighbours: alpha = 0, beta = 3)."""
    return -2.0 * (alpha + 24.0 * G * sigma) / beta


def mechanical_stability(T, a, eps, b=4.0, R=1.0, G=-1.0):
    """Eq. (21) coexistence densities (rho_l, rho_g) for a given epsilon.

    With psi from Eq. (24) the integrand (p0 - rho c_s^2 - G psi^2 / 2) psi' / psi^(1+eps)
    equals (p0 - p_EOS) psi' / psi^(1+eps); psi' = (p' - c_s^2) / (G psi).
    Used as theory context only.
    """
    rs_g, rs_l = spinodals(a, b, R, T)
    p_hi = float(p_eos(rs_g, a, b, R, T))
    p_lo = max(float(p_eos(rs_l, a, b, R, T)), 0.0)

    def integrand(r, p0):
        ps = float(psi(r, a, b, R, T, G))
        dps = (float(dp_drho(r, a, b, R, T)) - CS2) / (G * ps)
        return (p0 - float(p_eos(r, a, b, R, T))) * dps / ps ** (1.0 + eps)

    def cond(p0):
        rg, rl = _roots_at_pressure(p0, a, b, R, T, rs_g, rs_l)
        val, _ = integrate.quad(integrand, rg, rl, args=(p0,), points=[rs_g, rs_l], limit=400,
                                epsabs=0.0, epsrel=1e-11)
        return val

    eps_p = 1e-12 * p_hi
    lo, hi = p_lo + eps_p, p_hi - eps_p
    clo, chi = cond(lo), cond(hi)
    if clo * chi > 0:
        raise ValueError("no mechanical-stability solution at this temperature")
    p0 = optimize.brentq(cond, lo, hi, xtol=1e-18, rtol=1e-13, maxiter=500)
    rg, rl = _roots_at_pressure(p0, a, b, R, T, rs_g, rs_l)
    return rl, rg


# ------------------------------------------------------------------ Eq. (23) pseudopotential

def log_psi_ss(rho, eps):
    """log of the Eq. (23) psi: -1/rho for eps = 0, (log rho - log(eps + rho)) / eps otherwise."""
    rho = np.asarray(rho, dtype=np.float64)
    if eps == 0.0:
        return -1.0 / rho
    return (np.log(rho) - np.log(eps + rho)) / eps


def psi_ss(rho, eps):
    """Eq. (23): psi = exp(-1/rho) for eps = 0, (rho / (eps + rho))^(1/eps) otherwise."""
    rho = np.asarray(rho, dtype=np.float64)
    if eps == 0.0:
        return np.exp(-1.0 / rho)
    return (rho / (eps + rho)) ** (1.0 / eps)


def dpsi_ss(rho, eps):
    """d psi / d rho of Eq. (23): log psi = (log rho - log(eps + rho)) / eps, so
    psi' / psi = 1 / (rho (rho + eps)) (eps = 0: 1 / rho^2)."""
    rho = np.asarray(rho, dtype=np.float64)
    return psi_ss(rho, eps) / (rho * (rho + eps))


def p_ss(rho, G, eps):
    """Bulk pressure of the pseudopotential model with the Eq. (23) psi: rho/3 + G psi^2 / 2."""
    rho = np.asarray(rho, dtype=np.float64)
    return CS2 * rho + 0.5 * G * psi_ss(rho, eps) ** 2


def dp_ss(rho, G, eps):
    return CS2 + G * psi_ss(rho, eps) * dpsi_ss(rho, eps)


def critical_ss(eps):
    """Critical point of p_ss: dp/drho = 1/3 + G h(rho) with h = psi^2 / (rho (rho + eps));
    d log h / d rho = (2 - 2 rho - eps) / (rho (rho + eps)) vanishes at rho_c = 1 - eps/2,
    and G_c = -1 / (3 h(rho_c)).  Returns (rho_c, G_c); needs 0 <= eps < 2."""
    if not 0.0 <= eps < 2.0:
        raise ValueError("eps must lie in [0, 2)")
    rc = 1.0 - 0.5 * eps
    h = float(psi_ss(rc, eps)) ** 2 / (rc * (rc + eps))
    return rc, -1.0 / (3.0 * h)


def spinodals_ss(G, eps):
    rc, Gc = critical_ss(eps)
    if not G < Gc:
        raise ValueError("G must lie below the critical coupling")
    f = lambda r: float(dp_ss(r, G, eps))
    rg = optimize.brentq(f, 1e-3, rc, xtol=1e-16, rtol=1e-15)
    hi = 2.0 * rc
    while f(hi) < 0.0:
        hi *= 2.0
    rl = optimize.brentq(f, rc, hi, xtol=1e-16, rtol=1e-15)
    return rg, rl


def _roots_ss(p0, G, eps, rs_g, rs_l):
    g = lambda r: float(p_ss(r, G, eps)) - p0
    rg = optimize.brentq(g, 1e-3, rs_g, xtol=1e-300, rtol=1e-15, maxiter=500)
    hi = 2.0 * rs_l
    while g(hi) < 0.0:
        hi *= 2.0
    rl = optimize.brentq(g, rs_l, hi, xtol=1e-16, rtol=1e-15, maxiter=500)
    return rg, rl


def _coexistence_ss(G, eps, weight):
    """p0 with integral_{rho_g}^{rho_l} (p0 - p_ss) weight(rho) d rho = 0 at the roots of p_ss = p0."""
    rs_g, rs_l = spinodals_ss(G, eps)
    p_hi = float(p_ss(rs_g, G, eps))
    p_lo = max(float(p_ss(rs_l, G, eps)), float(p_ss(1e-3, G, eps)))

    def area(p0):
        rg, rl = _roots_ss(p0, G, eps, rs_g, rs_l)
        val, _ = integrate.quad(lambda r: (p0 - float(p_ss(r, G, eps))) * weight(r), rg, rl,
                                points=[rs_g, rs_l], limit=400, epsabs=0.0, epsrel=1e-12)
        return val

    d = 1e-13 * abs(p_hi)
    p0 = optimize.brentq(area, p_lo + d, p_hi - d, xtol=1e-18, rtol=1e-14, maxiter=500)
    rg, rl = _roots_ss(p0, G, eps, rs_g, rs_l)
    return rl, rg


def maxwell_ss(G, eps):
    """Eq. (22) for p_ss: (rho_l, rho_g) with integral (p0 - p_ss) / rho^2 = 0."""
    return _coexistence_ss(G, eps, lambda r: 1.0 / r ** 2)


def mechanical_stability_ss(G, eps_psi, eps):
    """Eq. (21) coexistence (rho_l, rho_g) with the Eq. (23) psi of parameter eps_psi and
    the weight psi' / psi^(1 + eps) of a stencil/forcing with parameter eps."""
    # psi' / psi^(1 + eps) = psi^(-eps) / (rho (rho + eps_psi)), psi^(-eps) from log psi
    return _coexistence_ss(G, eps_psi,
                           lambda r: math.exp(-eps * float(log_psi_ss(r, eps_psi))) / (r * (r + eps_psi)))


def lamb_period(theta, rho_l, R0, n=2):
    """Eq. (32): period of mode-n oscillation of a 2-D droplet of radius R0 and surface tension theta."""
    return 2.0 * math.pi * (n * (n * n - 1) * theta / (rho_l * R0 ** 3)) ** -0.5
