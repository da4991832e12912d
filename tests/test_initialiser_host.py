"""Host-side logic of the learned initialiser (paper_1211_6932_amd.initialiser, no GPU):
the convergence detector and its summary on hand-built records, the equimolar radius
and the tanh base profile against closed forms, and the training schedule's
sampling without replacement and cosine learning rate."""
import math

import numpy as np
import pytest

import workloads as W
from paper_1211_6932_amd import initialiser as I


def test_sample_radii():
    r = I.radii(40.0)
    assert r[0] == 40.0 - 31.75 and r[-1] == 40.0 + 31.75 and np.allclose(np.diff(r), 0.5)


def test_n_conv_first_check_after_which_every_later_check_is_inside():
    every = 50
    u_ref, dp_ref = np.array([1.0]), np.array([2.0])
    #         check: 0     1     2     3     4     5     6
    U = np.array([[3.0, 1.02, 1.2, 1.04, 0.97, 1.01, 1.0]])
    DP = np.array([[9.0, 2.0, 2.0, 2.5, 2.03, 2.01, 2.0]])
    # max|u| alone: checks 3.. are within 5 % (check 2 is 20 % off)
    assert I.n_conv(U, DP, u_ref, dp_ref, every) == [3 * every]
    # with dp within 1 % as well: check 4 has dp 1.5 % off, so from check 5
    assert I.n_conv(U, DP, u_ref, dp_ref, every, strict=True) == [5 * every]
    # inside from the start, and outside at the last check
    assert I.n_conv(np.ones((1, 4)), np.full((1, 4), 2.0), u_ref, dp_ref, every, strict=True) == [0]
    assert I.n_conv(np.array([[1.0, 1.0, 1.3]]), np.full((1, 3), 2.0), u_ref, dp_ref, every) == [None]
    # the bounds are inclusive (5 % of max|u|, 1 % of |dp|; values chosen so that both
    # tolerances and both differences are exact in binary)
    U = np.array([[30.0, 21.0]])
    DP = np.array([[150.0, 101.0]])
    assert I.n_conv(U, DP, np.array([20.0]), np.array([100.0]), every, strict=True) == [every]


def test_summarise_medians_and_ratios():
    steps, every = 1000, 50
    res = dict(steps=steps, every=every, unstable=[False, False, True, False, False],
               n_tanh_u=[400, 600, 300, None, 980], n_learned_u=[100, None, 10, 50, 0],
               dp_err=[0.1, -0.2, 0.3, 0.4, 0.5], rho_in_err=[1e-3] * 5, rho_out_err=[2e-3] * 5,
               dp_err_start=[-0.5, 0.5, 1.0, 1.0, 1.0])
    s = I.summarise(res, "u")
    # counted: droplets 0 and 1 (2 is unstable, 3 never converges for tanh, 4 only at the
    # last check); learned: 100 and the full window for the one that never converges
    assert s["converged"] == 2 and s["unstable"] == 1 and s["learned_not_converged"] == 1
    assert s["median_steps_tanh"] == 500.0 and s["median_steps_learned"] == 550.0
    assert s["ratio_of_medians"] == pytest.approx(500.0 / 550.0)
    assert s["median_ratio"] == pytest.approx(np.median([4.0, 0.6]))
    assert s["median_abs_dp_err"] == pytest.approx(0.15) and s["max_abs_dp_err"] == pytest.approx(0.2)
    assert s["median_abs_dp_err_start"] == pytest.approx(0.5)
    # a learned run converged at check 0 counts as one check interval
    res["n_learned_u"][0] = 0
    assert I.summarise(res, "u")["median_steps_learned"] == pytest.approx(np.median([every, steps]))


def test_equimolar_radius_of_a_disc():
    nx, R, rho_in, rho_out = 256, 37.25, 0.41, 0.003
    mass = rho_out * nx * nx + (rho_in - rho_out) * math.pi * R * R
    assert I.equimolar_radius(mass, rho_in, rho_out, nx * nx) == pytest.approx(R, rel=1e-12)
    assert I.equimolar_radius(0.5 * rho_out * nx * nx, rho_in, rho_out, nx * nx) == 0.0


def test_tanh_base_is_the_eq31_profile():
    w = W.learned_eval_instances(n=3, side=128)
    base = I.tanh_base(w)
    for i, wi in enumerate(w):
        rl, rg, R = wi.info["rho_l"], wi.info["rho_g"], wi.info["R0"]
        d = I.radii(R) - R
        ref = 0.5 * (rl + rg) - 0.5 * (rl - rg) * np.tanh(2.0 * d / 5.0)
        np.testing.assert_allclose(np.exp(base[i]), ref, rtol=1e-14)
        # midpoint density halfway between the samples 63 and 64
        assert 0.5 * (math.exp(base[i][63]) + math.exp(base[i][64])) == pytest.approx(0.5 * (rl + rg), rel=1e-3)


def test_schedule_draws_without_replacement_and_decays_the_rate():
    torch = pytest.importorskip("torch")
    n, steps, mb = 1000, 12, 256
    idx, rates = I.schedule(n, steps, mb, 1e-3, 1e-5, seed=5)
    assert idx.dtype == torch.int32 and tuple(idx.shape) == (steps, mb)
    a = idx.numpy()
    assert a.min() >= 0 and a.max() < n
    # three minibatches per pass (3 * 256 <= 1000 < 4 * 256): no row twice within a pass
    for p in range(0, steps, 3):
        rows = a[p:p + 3].ravel()
        assert len(np.unique(rows)) == rows.size
    assert rates[0] == np.float32(1e-3) and rates[-1] == np.float32(1e-5)
    assert np.all(np.diff(rates) < 0)
    k = 5
    assert rates[k] == np.float32(1e-5 + 0.5 * (1e-3 - 1e-5) * (1.0 + math.cos(math.pi * k / (steps - 1))))
    # the same seed draws the same minibatches
    idx2, _ = I.schedule(n, steps, mb, 1e-3, 1e-5, seed=5)
    assert np.array_equal(a, idx2.numpy())
    with pytest.raises(ValueError):
        I.schedule(31, 2, 512, 1e-3, 1e-5, seed=1)


def test_sweep_edge_helpers():
    """The sweeps' host reductions: lowest temperature above which every run survived,
    and the lowest surviving viscosity of a grid."""
    from paper_1211_6932_amd import sweeps as S
    rows = [dict(t_over_tc=t, stable=s) for t, s in
            [(0.9, True), (0.85, True), (0.85, True), (0.8, True), (0.8, False), (0.75, True), (0.7, True)]]
    # 0.8 has a failed run, so the edge is 0.85 even though 0.75 and 0.7 survived
    assert S.lowest_stable(rows) == 0.85
    assert S.lowest_stable([dict(t_over_tc=0.9, stable=False)]) is None
    assert S.lowest_stable([dict(t_over_tc=t, stable=True) for t in (0.6, 0.9, 0.7)]) == 0.6
    nus = [0.001, 0.002, 0.004, 0.008, 0.016]
    assert S.lowest_stable_viscosity(nus, [100, 300, None, None, 50]) == 0.004
    assert S.lowest_stable_viscosity(nus, [1, 1, 1, 1, 1]) is None
    assert S.CS == pytest.approx(1.0 / math.sqrt(3.0))
