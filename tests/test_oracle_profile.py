"""Pins of the radial-profile oracle (oracle/profile.py): exact sample sites, profiles
inside the least-squares model's span, a brute-force normal-equation solve."""
import math

import numpy as np

from oracle import profile as P


def test_radii_window():
    r = P.radii(40.0)
    assert r.shape == (128,)
    assert r[0] == 40.0 - 31.75 and r[-1] == 40.0 + 31.75
    assert np.allclose(np.diff(r), 0.5)


def test_to_rho0_exact_at_sample_sites_and_held_outside():
    R, cx, cy, n = 40.75, 100.0, 90.0, 256
    logrho = np.linspace(-0.5, -6.0, 128) + 0.1 * np.sin(np.arange(128))
    field = P.to_rho0(logrho, R, cx, cy, n, n)
    for k in range(0, 128, 2):  # r_k = 9 + k/2 is an integer for even k
        d = int(9 + k // 2)
        assert abs(field[int(cy), int(cx) + d] - math.exp(logrho[k])) < 1e-14
        assert abs(field[int(cy) - d, int(cx)] - math.exp(logrho[k])) < 1e-14
    assert field[int(cy), int(cx)] == math.exp(logrho[0])
    # minimum image: the far corner is beyond the window
    assert field[int(cy) + 128, int(cx) + 128] == math.exp(logrho[-1])
    # R = 40.5: r_k = 8.75 + k/2, so distance 9 + j lies halfway between samples 2j and 2j+1
    half = P.to_rho0(logrho, 40.5, cx, cy, n, n)
    for j in (0, 5, 30):
        assert abs(half[int(cy), int(cx) + 9 + j] - math.exp(0.5 * (logrho[2 * j] + logrho[2 * j + 1]))) < 1e-14


def test_extract_constant_and_linear_profiles_exactly():
    n, cx, cy, R = 200, 99.5, 100.25, 60.0
    assert np.abs(P.extract(np.full((n, n), 0.37), cx, cy, R) - math.log(0.37)).max() < 1e-12
    # a linear profile is in the model's span; the smoothness term only pulls the two end
    # samples, by about lam * slope / (weight of their data)
    L = -0.7 - 0.04 * np.arange(128)
    back = P.extract(P.to_rho0(L, R, cx, cy, n, n), cx, cy, R)
    assert np.abs(back - L)[1:-1].max() < 1e-9 and np.abs(back - L).max() < 1e-8


def test_extract_recovers_a_curved_profile_in_its_span():
    n, cx, cy, R = 256, 127.5, 127.5, 50.0
    r = P.radii(R)
    L = np.log(0.26 + 0.24 * np.tanh((R - r) / 3.0))
    back = P.extract(P.to_rho0(L, R, cx, cy, n, n), cx, cy, R)
    # only the smoothness term perturbs it: lam |second difference| / (sites per hat)
    assert np.abs(back - L).max() < 1e-5


def test_extract_matches_brute_force_normal_equations():
    rng = np.random.default_rng(3)
    n, cx, cy, R = 48, 20.3, 25.9, 12.0
    rho = np.exp(rng.normal(-1.0, 0.3, (n, n)))
    d = P.min_image_distance(n, n, cx, cy).ravel()
    H = np.zeros((d.size, 128))
    r = P.radii(R)
    for i, di in enumerate(d):  # hat functions written out, end hats extended
        if di <= r[0]:
            H[i, 0] = 1.0
        elif di >= r[-1]:
            H[i, -1] = 1.0
        else:
            j = int((di - r[0]) // 0.5)
            t = (di - r[j]) / 0.5
            H[i, j] += 1.0 - t
            H[i, j + 1] += t
    D = np.zeros((127, 128))
    D[np.arange(127), np.arange(127)] = -1.0
    D[np.arange(127), np.arange(1, 128)] = 1.0
    A = H.T @ H + P.LAM * D.T @ D
    ref = np.linalg.solve(A, H.T @ np.log(rho).ravel())
    assert np.abs(P.extract(rho, cx, cy, R) - ref).max() < 1e-9


def test_empty_radii_take_the_nearest_fitted_value():
    # R = 10: r_k < 0 for k < 43.5, where no site lies; the smoothness term carries
    # the innermost fitted value inwards
    n, cx, cy, R = 64, 31.5, 31.5, 10.0
    rho = 0.3 + 0.1 * np.tanh((R - P.min_image_distance(n, n, cx, cy)) / 2.0)
    L = P.extract(rho, cx, cy, R)
    assert np.all(np.isfinite(L))
    inner = int(np.ceil(63.5 - 2 * R))
    assert np.abs(L[:inner] - L[inner]).max() < 1e-3


def test_mass_matched_field_carries_the_mass_and_shifts_the_profile():
    n, cx, cy, R = 128, 63.5, 63.5, 30.0
    r = P.radii(R)
    L = np.log(0.26 + 0.24 * np.tanh((R - r) / 2.5))
    base_field = P.to_rho0(L, R, cx, cy, n, n)
    # the unshifted field's own mass gives delta = 0 (to the bisection's resolution)
    f0, d0 = P.to_rho0_mass(L, R, cx, cy, n, n, base_field.sum())
    assert abs(d0) < 1e-12 and np.abs(f0 - base_field).max() < 1e-12
    # a larger mass moves the interface outwards by the area it needs: 2 pi R delta drho ~ dM
    dm = 0.5 * 2 * np.pi * R * (0.5 - 0.02)
    f1, d1 = P.to_rho0_mass(L, R, cx, cy, n, n, base_field.sum() + dm)
    assert abs(f1.sum() - (base_field.sum() + dm)) < 1e-9 * f1.sum()
    assert 0.45 < d1 < 0.55
    # the shifted field is the profile sampled at d - delta
    assert np.allclose(f1, P.to_rho0(L, R + d1, cx, cy, n, n))
