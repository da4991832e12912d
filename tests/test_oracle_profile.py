"""Pins of the radial-profile oracle (oracle/profile.py): fields whose angular mean
is known in closed form, a library bilinear interpolator, exact sample sites."""
import math

import numpy as np
from scipy import ndimage

from oracle import profile as P


def test_radii_window():
    r = P.radii(40.0)
    assert r.shape == (128,)
    assert r[0] == 40.0 - 31.75 and r[-1] == 40.0 + 31.75
    assert np.allclose(np.diff(r), 0.5)


def test_bilinear_matches_library_interpolator():
    rng = np.random.default_rng(0)
    rho = rng.uniform(0.1, 1.0, (23, 31))
    pts = rng.uniform(-40, 70, (200, 2))
    ref = ndimage.map_coordinates(rho, [pts[:, 1], pts[:, 0]], order=1, mode="grid-wrap")
    got = np.array([P.bilinear_periodic(rho, x, y) for x, y in pts])
    assert np.abs(got - ref).max() < 1e-13


def test_extract_of_constant_and_bilinear_fields_is_exact():
    nx, ny = 200, 160
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    assert np.abs(P.extract(np.full((ny, nx), 0.37), 97.0, 80.0, 40.0) - math.log(0.37)).max() < 1e-14
    # rho = 1 + 2e-3 x + 1e-5 x y: bilinear interpolation reproduces it, and the mean over
    # equally spaced angles of (cx + r cos)(cy + r sin) is cx cy (no wrap: r <= 72 < distances to edges)
    rho = 1.0 + 2e-3 * x + 1e-5 * x * y
    cx, cy = 99.0, 79.5
    prof = P.extract(rho, cx, cy, 40.0)
    assert np.abs(prof - math.log(1.0 + 2e-3 * cx + 1e-5 * cx * cy)).max() < 1e-13


def test_extract_of_radial_field_recovers_the_radial_function():
    nx = ny = 256
    cx = cy = 127.5
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    f = lambda s: 0.3 + 0.2 * np.tanh((50.0 - s) / 4.0)  # noqa: E731
    prof = P.extract(f(r), cx, cy, 50.0)
    # bilinear interpolation of a smooth radial function: error O(h^2 f'')
    assert np.abs(np.exp(prof) - f(P.radii(50.0))).max() < 2e-3


def test_to_rho0_exact_at_sample_sites_and_held_outside():
    R, cx, cy, n = 40.75, 100.0, 90.0, 256
    logrho = np.linspace(-0.5, -6.0, 128) + 0.1 * np.sin(np.arange(128))
    field = P.to_rho0(logrho, R, cx, cy, n, n)
    for k in range(0, 128, 2):  # r_k = 9 + k/2 is an integer for even k
        d = int(9 + k // 2)
        assert abs(field[int(cy), int(cx) + d] - math.exp(logrho[k])) < 1e-14
        assert abs(field[int(cy) - d, int(cx)] - math.exp(logrho[k])) < 1e-14
    assert field[int(cy), int(cx)] == math.exp(logrho[0])
    # minimum image: the far corner is at distance < n/sqrt(2) and beyond the window
    assert field[int(cy) + 128, int(cx) + 128] == math.exp(logrho[-1])


def test_round_trip_in_the_window():
    R, cx, cy, n = 60.0, 127.0, 128.0, 256
    logrho = np.log(0.3 + 0.2 * np.tanh((R - P.radii(R)) / 3.0))
    back = P.extract(P.to_rho0(logrho, R, cx, cy, n, n), cx, cy, R)
    # both interpolations are exact for linear data; the tanh curvature costs about
    # h^2 max|rho''| / 4 = 0.2 * 0.77 / 9 / 4 = 4e-3 in rho, 1.4e-2 in log rho at rho = 0.3
    assert np.abs(back[2:-2] - logrho[2:-2]).max() < 2e-2
    assert np.abs(back[:20] - logrho[:20]).max() < 1e-6  # flat bulk (r <= R - 22): exact up to the tanh tail
