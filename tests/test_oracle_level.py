"""Pins of the liquid-level oracle (oracle/level.py) against closed forms and
hand counts: the Chebyshev tensor basis against cos(n theta), the least-squares
fit against planted polynomials, the bands against counts by hand and the
anchoring against the affine map it must be (interface shape kept, vapour end
fixed, interior flat at the target)."""
import numpy as np
import pytest

from oracle import level as OL

D = (np.arange(128) - 63.5) * 0.5


def _features(n, seed, a_values=(0.25, 0.5, 1.0)):
    rng = np.random.default_rng(seed)
    return np.c_[rng.choice(a_values, n), rng.uniform(0.5, 0.85, n), rng.uniform(25.0, 77.0, n),
                 rng.uniform(1.0, 15.0, n)]


def test_basis_is_the_chebyshev_tensor_product_in_the_stated_column_order():
    lo = np.array([0.0, 0.0, 0.0, 0.0])
    hi = np.array([2.0, 2.0, 2.0, 2.0])
    rng = np.random.default_rng(3)
    theta = rng.uniform(0.0, np.pi, (16, 4))
    z = np.cos(theta)
    x = z + 1.0                      # maps onto z through [lo, hi] = [0, 2]
    u = x[:, 2].copy()
    x[:, 2] = 1.0 / u                # the model sees R through u = 1/R
    A = OL.design(x, lo, hi)
    for i in range(3):
        for j in range(7):
            for k in range(4):
                for m in range(2):
                    col = ((i * 7 + j) * 4 + k) * 2 + m
                    want = (np.cos(i * theta[:, 0]) * np.cos(j * theta[:, 1]) * np.cos(k * theta[:, 2])
                            * np.cos(m * theta[:, 3]))
                    np.testing.assert_allclose(A[:, col], want, rtol=0, atol=1e-12)


def test_scaling_maps_the_fit_range_onto_minus_one_one_and_clamps():
    x = _features(200, 1)
    lo, hi, _ = OL.fit(x, np.zeros(len(x)))
    z = OL.scaled(x, lo, hi)
    assert np.allclose(z.min(0), -1.0) and np.allclose(z.max(0), 1.0)
    # the largest radius has the smallest 1/R
    assert z[np.argmax(x[:, 2]), 2] == pytest.approx(-1.0)
    far = x[:1].copy()
    far[0, 1] = 2.0
    assert OL.scaled(far, lo, hi)[0, 1] == 1.0


def test_fit_recovers_a_planted_polynomial():
    x = _features(3000, 2)
    v = x.copy()
    v[:, 2] = 1.0 / v[:, 2]
    lo, hi = v.min(0), v.max(0)
    c0 = np.random.default_rng(5).standard_normal(OL.TERMS) * 1e-3
    y = OL.design(x, lo, hi) @ c0
    lo_f, hi_f, c = OL.fit(x, y)
    np.testing.assert_array_equal(lo_f, lo)
    np.testing.assert_allclose(c, c0, rtol=0, atol=1e-9)
    x_new = _features(50, 9)
    np.testing.assert_allclose(OL.evaluate((lo_f, hi_f, c), x_new), OL.design(x_new, lo, hi) @ c0, atol=1e-11)


def test_fit_with_a_single_value_of_a_feature_is_finite_and_exact_on_its_rows():
    x = _features(800, 4, a_values=(0.5,))
    y = 1e-3 * np.sin(4.0 * x[:, 1]) + 0.02 / x[:, 2]
    model = OL.fit(x, y)
    assert np.all(np.isfinite(model[2]))
    assert model[0][0] == model[1][0] == 0.5
    np.testing.assert_allclose(OL.evaluate(model, x), y, atol=1e-8)


@pytest.mark.parametrize("R, k_last_inner", [(40.0, 39), (24.0, 39), (20.0, 43), (5.0, 58), (0.0, 63)])
def test_bands_by_hand(R, k_last_inner):
    inner, outer = OL.bands(R)
    assert np.array_equal(np.nonzero(inner)[0], np.arange(k_last_inner + 1))
    assert np.array_equal(np.nonzero(outer)[0], np.arange(88, 128))


def test_levels_of_simple_profiles():
    assert OL.levels(np.full(128, -0.7), 40.0) == pytest.approx((-0.7, -0.7), abs=1e-15)
    k = np.arange(128, dtype=np.float64)
    assert OL.levels(k, 40.0) == (19.5, 107.5)
    assert OL.levels(k, 20.0) == (21.5, 107.5)


def _shape():
    """An interface shape s(d): 1 on the inner band, 0 on the outer band, smooth between."""
    s = 0.5 * (1.0 - np.tanh(2.0 * D / 5.0))
    s = (s - s[88]) / (s[39] - s[88])
    return np.clip(np.where(D <= -12, 1.0, np.where(D >= 12, 0.0, s)), 0.0, 1.0)


def test_anchor_is_the_affine_map_that_keeps_the_shape_and_the_vapour_end():
    s = _shape()
    rho_l, rho_g, target = 0.41, 0.012, 0.4132
    L = np.log(rho_g + (rho_l - rho_g) * s)
    out = OL.anchor(L, 40.0, np.log(target))
    np.testing.assert_allclose(np.exp(out), rho_g + (target - rho_g) * s, rtol=1e-14)


def test_anchor_flattens_the_interior_onto_the_target_and_is_idempotent():
    rng = np.random.default_rng(7)
    s = _shape()
    L = np.log(0.012 + (0.41 - 0.012) * s) + 1e-3 * rng.standard_normal(128)
    lev = np.log(0.4104)
    out = OL.anchor(L, 40.0, lev)
    inner, _ = OL.bands(40.0)
    np.testing.assert_allclose(out[inner], lev, rtol=0, atol=1e-15)
    assert OL.levels(out, 40.0)[0] == pytest.approx(lev, abs=1e-15)
    np.testing.assert_allclose(OL.anchor(out, 40.0, lev), out, rtol=0, atol=1e-14)
    # outside the interior the density moves by the same factor g about the vapour level
    r_out = np.exp(OL.levels(L, 40.0)[1])
    g = (np.exp(lev) - r_out) / (np.exp(OL.levels(L, 40.0)[0]) - r_out)
    np.testing.assert_allclose(np.exp(out[~inner]) - r_out, (np.exp(L[~inner]) - r_out) * g, rtol=1e-12, atol=1e-16)


def test_anchor_leaves_a_profile_alone_when_the_target_is_unusable():
    L = np.log(0.012 + 0.398 * _shape())
    for lev in (np.nan, np.inf):
        np.testing.assert_array_equal(OL.anchor(L, 40.0, lev), L)
    flat = np.full(128, -1.0)            # rho_in == rho_out
    np.testing.assert_array_equal(OL.anchor(flat, 40.0, -0.9), flat)
    # a target below the vapour level reverses the map (g < 0): a sample that overshoots
    # the interior density would go negative, so nothing is changed
    over = L.copy()
    over[50] = np.log(0.5)
    np.testing.assert_array_equal(OL.anchor(over, 40.0, np.log(1e-4)), over)
