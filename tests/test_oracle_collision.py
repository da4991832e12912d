"""Pins of the oracle's single-site algebra (oracle/lbref.c) against textbook D2Q9
results and closed forms of the paper's equations.  CPU only.

The textbook quantities below are written from the standard D2Q9 lattice
(weights 4/9, 1/9, 1/36; c_s^2 = 1/3) and Guo's forcing term, not from the
oracle's moment tables, so a wrong row, sign or ordering in the oracle's M,
m_eq (Eq. 3) or Sbar (Eqs. 9, 25) fails here."""
import numpy as np
import pytest

from oracle import lbref as L

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def feq_textbook(rho, ux, uy):
    eu = EX * ux + EY * uy
    return W * rho * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (ux * ux + uy * uy))


def guo_textbook(ux, uy, Fx, Fy):
    """Guo et al. forcing term without the (1 - 1/(2 tau)) prefactor."""
    eu = EX * ux + EY * uy
    eF = EX * Fx + EY * Fy
    return W * (3 * ((EX - ux) * Fx + (EY - uy) * Fy) + 9 * eu * eF)


def eq3(rho, vx, vy):
    v2 = vx * vx + vy * vy
    return rho * np.array([1, -2 + 3 * v2, 1 - 3 * v2, vx, -vx, vy, -vy, vx * vx - vy * vy, vx * vy])


def eq9(vx, vy, Fx, Fy):
    vF = vx * Fx + vy * Fy
    return np.array([0, 6 * vF, -6 * vF, Fx, -Fx, Fy, -Fy, 2 * (vx * Fx - vy * Fy), vx * Fy + vy * Fx])


def test_M_rows_orthogonal_and_inverse():
    M, Minv = L.matrices()
    G = M @ M.T
    norms = np.array([9, 36, 36, 6, 12, 6, 12, 4, 4], dtype=np.float64)
    assert np.abs(G - np.diag(norms)).max() == 0.0
    assert np.abs(Minv - M.T / norms[None, :]).max() < 1e-15
    assert np.abs(M @ Minv - np.eye(9)).max() < 1e-15
    # rows 3/5 are the momentum moments, row 0 the density
    assert np.array_equal(M[0], np.ones(9)) and np.array_equal(M[3], EX) and np.array_equal(M[5], EY)


@pytest.mark.parametrize("seed", range(5))
def test_M_maps_textbook_feq_to_eq3_and_guo_to_eq9(seed):
    rng = np.random.default_rng(seed)
    M, _ = L.matrices()
    rho, ux, uy, Fx, Fy = rng.uniform(0.01, 0.5), *rng.normal(0, 0.1, 2), *rng.normal(0, 1e-3, 2)
    assert np.abs(M @ feq_textbook(rho, ux, uy) - eq3(rho, ux, uy)).max() < 1e-15
    assert np.abs(M @ guo_textbook(ux, uy, Fx, Fy) - eq9(ux, uy, Fx, Fy)).max() < 1e-17


@pytest.mark.parametrize("seed", range(6))
def test_equal_rates_reduce_to_bgk_guo(seed):
    """All s_k = 1/tau and sigma = 0: Eq. (4) must equal the BGK-Guo collision."""
    rng = np.random.default_rng(100 + seed)
    tau = rng.uniform(0.55, 1.9)
    s = 1.0 / tau
    nu = (tau - 0.5) / 3.0
    p = L.Params(nx=1, ny=1, sigma=0.0, s_rho=s, s_e=s, s_zeta=s, s_j=s, s_q=s, nu_l=nu, nu_g=nu)
    f = feq_textbook(0.3, 0.05, -0.02) + rng.normal(0, 1e-3, 9)
    rho = f.sum()
    Fx, Fy = rng.normal(0, 1e-3, 2)
    vx = (f @ EX + 0.5 * Fx) / rho
    vy = (f @ EY + 0.5 * Fy) / rho
    ref = f - (f - feq_textbook(rho, vx, vy)) / tau + (1 - 0.5 / tau) * guo_textbook(vx, vy, Fx, Fy)
    for form in (L.FORM_MOMENT, L.FORM_VELOCITY):
        out = L.collide_site(p, f, rho, vx, vy, Fx, Fy, 0.1, form)
        assert np.abs(out - ref).max() < 1e-15


@pytest.mark.parametrize("sigma", [0.11, 0.114, 0.125])
def test_improved_term_closed_form(sigma):
    """Eq. (25) minus Eq. (9), through (I - Lambda/2) and M^-1, equals
    12 sigma |F|^2 / psi^2 (s_e e_row - s_zeta eps_row) / 36 in velocity space,
    where e_row, eps_row are the energy and energy-square rows of M (norm 36)."""
    rng = np.random.default_rng(7)
    p1 = L.Params(nx=1, ny=1, sigma=sigma, s_e=0.8, s_zeta=1.3)
    p0 = L.Params(nx=1, ny=1, sigma=0.0, s_e=0.8, s_zeta=1.3)
    f = feq_textbook(0.2, 0.01, 0.02) + rng.normal(0, 1e-3, 9)
    rho, Fx, Fy, psi2 = f.sum(), 3e-3, -2e-3, 0.07
    vx, vy = 0.011, 0.019
    e_row = np.array([-4, -1, -1, -1, -1, 2, 2, 2, 2], dtype=np.float64)
    eps_row = np.array([4, -2, -2, -2, -2, 1, 1, 1, 1], dtype=np.float64)
    k = 12 * sigma * (Fx * Fx + Fy * Fy) / psi2 / 36.0
    expect = k * (0.8 * e_row - 1.3 * eps_row)
    for form in (L.FORM_MOMENT, L.FORM_VELOCITY):
        d = L.collide_site(p1, f, rho, vx, vy, Fx, Fy, psi2, form) - \
            L.collide_site(p0, f, rho, vx, vy, Fx, Fy, psi2, form)
        assert np.abs(d - expect).max() < 1e-16
    # the extra term neither creates mass nor momentum
    assert abs(expect.sum()) < 1e-18 and abs(expect @ EX) < 1e-18


@pytest.mark.parametrize("s_j", [0.7, 1.0, 1.6])
def test_collision_conserves_mass_and_adds_force(s_j):
    """With the half-force velocity of Eq. (6), one collision changes the momentum by
    exactly F for any s_j (and conserves mass)."""
    rng = np.random.default_rng(3)
    p = L.Params(nx=1, ny=1, s_j=s_j)
    f = feq_textbook(0.35, 0.03, 0.01) + rng.normal(0, 1e-3, 9)
    Fx, Fy = 2e-3, -1e-3
    rho = f.sum()
    vx = (f @ EX + 0.5 * Fx) / rho
    vy = (f @ EY + 0.5 * Fy) / rho
    out = L.collide_site(p, f, rho, vx, vy, Fx, Fy, 0.2)
    assert out.sum() == pytest.approx(rho, abs=1e-16)
    assert out @ EX - f @ EX == pytest.approx(Fx, abs=1e-17)
    assert out @ EY - f @ EY == pytest.approx(Fy, abs=1e-17)


@pytest.mark.parametrize("seed", range(4))
def test_moment_form_equals_velocity_form(seed):
    """Eq. (4) (moment space) and Eq. (1) (dense velocity-space matrices) agree."""
    rng = np.random.default_rng(50 + seed)
    p = L.Params(nx=1, ny=1, s_rho=rng.uniform(0.5, 1.5), s_e=rng.uniform(0.5, 1.5),
                 s_zeta=rng.uniform(0.5, 1.5), s_j=rng.uniform(0.5, 1.5), s_q=rng.uniform(0.5, 1.5),
                 nu_l=rng.uniform(0.01, 0.3), nu_g=rng.uniform(0.01, 0.3), sigma=0.11)
    f = feq_textbook(0.25, 0.02, -0.03) + rng.normal(0, 2e-3, 9)
    rho = f.sum()
    args = (rho, 0.02, -0.03, 1e-3, 2e-3, 0.05)
    a = L.collide_site(p, f, *args, L.FORM_MOMENT)
    b = L.collide_site(p, f, *args, L.FORM_VELOCITY)
    assert np.abs(a - b).max() < 1e-15


def test_viscosity_switch_selects_rate_by_density():
    """Sec. IV.C: nu = nu_l for rho >= rho_c, nu_g below; the shear rate enters the
    pxx/pxy moments only: the non-equilibrium pxx part relaxes by (1 - s_nu)."""
    M, Minv = L.matrices()
    p = L.Params(nx=1, ny=1, nu_l=0.1, nu_g=0.3, rho_switch=0.13045)
    for rho, nu in [(0.2, 0.1), (0.13045, 0.1), (0.1304, 0.3), (0.01, 0.3)]:
        fe = feq_textbook(rho, 0.0, 0.0)
        dm = np.zeros(9)
        dm[7] = 1e-4 * rho
        f = fe + Minv @ dm
        out = L.collide_site(p, f, rho, 0.0, 0.0, 0.0, 0.0, 0.1)
        s_nu = 1.0 / (3 * nu + 0.5)
        assert (M @ out)[7] == pytest.approx((1 - s_nu) * 1e-4 * rho, rel=1e-10)
