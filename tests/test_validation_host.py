"""Host-side measurement helpers of paper_1211_6932_amd.validation (no GPU): the
interface locator and the period estimator against closed forms and against the
oracle's own, separately written post-processing."""
import math

import numpy as np

import workloads as W
from oracle import post
from paper_1211_6932_amd import validation as V


def test_axis_extent_matches_closed_form_and_oracle():
    for n in (200, 201):
        w = W.oscillating_droplet(n=n)
        mid = 0.5 * (w.info["rho_l"] + w.info["rho_g"])
        got = V.axis_extent(V.centre_row(w.rho0, w.info["cy"]), w.info["cx"], mid)
        ref = post.major_axis_radius(w.rho0, w.info["cx"], w.info["cy"], mid)
        assert abs(got - ref) < 1e-12
        if n == 201:
            assert abs(got - w.info["r_max"]) < 1e-9


def test_period_from_crossings():
    for period in (2600.0, 811.3):
        t = np.arange(0, 5.1 * period, 10.0)
        x = 28.5 + 1.2 * np.exp(-t / 8000.0) * np.cos(2 * np.pi * t / period - 1.0)
        p, ups = V.period_from_crossings(t, x)
        assert abs(p / period - 1.0) < 5e-3 and len(ups) >= 4


def test_lamb_period_scaling():
    # Eq. (32): T ~ R0^(3/2) (rho_l / theta)^(1/2); mode 3 is sqrt(24 / 6) = 2 times faster
    T = V.lamb_period(0.01, 0.45, 28.46)
    assert abs(V.lamb_period(0.01, 0.45, 2 * 28.46) / T - 2 ** 1.5) < 1e-12
    assert abs(V.lamb_period(0.04, 0.45, 28.46) / T - 0.5) < 1e-12
    assert abs(V.lamb_period(0.01, 0.45, 28.46, n=3) / T - 0.5) < 1e-12
    assert abs(T - 2 * math.pi * math.sqrt(0.45 * 28.46 ** 3 / (6 * 0.01))) < 1e-9 * T


def test_effective_radius_of_a_sharp_disc():
    # a disc of area pi R^2 at rho_in in a box of rho_out
    M = 0.4 * math.pi * 30 ** 2 + 0.01 * (200 * 200 - math.pi * 30 ** 2)
    assert abs(V.effective_radius(M, 0.4, 0.01, 200 * 200) - 30.0) < 1e-12


def test_damped_cosine_fit_recovers_frequency_and_decay():
    rng = np.random.default_rng(4)
    for period, decay in ((2600.0, 4000.0), (2450.0, 2300.0)):
        t = np.arange(400.0, 13000.0, 10.0)
        x = 28.3 + 1.4 * np.exp(-t / decay) * np.cos(2 * np.pi * t / period + 0.7)
        x += 1e-4 * rng.standard_normal(t.size)
        fit = V.fit_damped_cosine(t, x, period * 0.95)
        assert abs(fit["period"] / period - 1) < 1e-3 and abs(fit["decay"] / decay - 1) < 1e-2
        g, w = 1 / decay, 2 * np.pi / period
        assert abs(fit["period0"] - 2 * np.pi / np.sqrt(w * w + g * g)) < 1e-3 * period


def test_spread_half_width_matches_closed_form_and_oracle():
    # a circle of radius 50 sunk 4 units into a flat film: on a line above the film
    # surface the liquid is the chord of the circle at that height (the line half a unit
    # above the film averages the film's own mid-density row, so it is checked against
    # the oracle's separately written measure only)
    w = W.paper_splash(0.1, 1.0, gap=-4.0)
    mid = 0.5 * (w.info["rho_l"] + w.info["rho_g"])
    film, R = w.info["film"], w.info["R"]
    cx = w.params["nx"] / 2.0
    for y in (film + 0.5, film + 3.0, film + 8.0):
        got = V.spread_half_width(V.centre_row(w.rho0, y), cx, mid)
        assert abs(got - post.spread_radius(w.rho0, cx, y, mid)) < 1e-9
        if y > film + 1.0:
            dy = (film + R - 4.0) - y  # circle centre above the line
            assert abs(got - math.sqrt(R * R - dy * dy)) < 0.01


def test_profile_parser_picks_the_time_step_instantiation():
    """prof.traffic reads the counters of d2q9_strip<store, walls, MODE 0, psi form> only."""
    from paper_1211_6932_amd import prof
    assert prof._is_step_kernel("void lbmp::d2q9_strip<0, true, 0, 0>(lbmp::Codec<0>::T const*, ...)")
    assert prof._is_step_kernel("void lbmp::d2q9_strip<5, false, 0, 1>(lbmp::Codec<5>::T const*, ...)")
    assert not prof._is_step_kernel("void lbmp::d2q9_strip<0, true, 2, 0>(lbmp::Codec<0>::T const*, ...)")
    assert not prof._is_step_kernel("void lbmp::d2q9_strip<0, true, 1, 0>(lbmp::Codec<0>::T const*, ...)")
    assert not prof._is_step_kernel("void lbmp::d2q9_batch<0, true, 0>(lbmp::BatchInstance const*, ...)")


def test_traffic_scales_each_counter_by_the_copy_probe(tmp_path):
    """prof.traffic: per-launch median of the step kernel's counter, scaled by what the same
    counter reads for the 1 GiB copy probe (FETCH_SIZE reporting half the bytes read
    gives a scale of 2), summed over read and write, against the algorithmic bytes."""
    from paper_1211_6932_amd import prof
    step = "_ZN4lbmp9d2q9_pairILb1ELi0EEEvPKDF16_PDF16_NS_9StepConstEPi"
    other = "void lbmp::d2q9_strip<5, true, 2, 0>(lbmp::Codec<5>::T const*, ...)"
    copy = "lbmp::copy_probe(HIP_vector_type<float, 4u> const*, HIP_vector_type<float, 4u>*, unsigned long)"
    for counter, name, copy_kib, vals in (("FETCH_SIZE", "fetch", 524288.0, [330000.0, 340000.0, 990000.0]),
                                          ("WRITE_SIZE", "write", 1048576.0, [660000.0, 670000.0, 680000.0])):
        d = tmp_path / name
        d.mkdir()
        rows = ["Kernel_Name,Counter_Name,Counter_Value"]
        rows += [f'"{step}",{counter},{v}' for v in vals]
        rows += [f'"{other}",{counter},123.0', f'"{copy}",{counter},{copy_kib}', f'"{copy}",OTHER,7.0']
        (d / f"{name}_counter_collection.csv").write_text("\n".join(rows) + "\n")
    sites = 1000000
    r = prof.traffic(str(tmp_path / "fetch"), str(tmp_path / "write"), "f16dest", sites)
    assert r["detail"]["read"]["scale"] == 2.0 and r["detail"]["write"]["scale"] == 1.0
    assert r["detail"]["read"]["bytes_per_launch"] == 340000.0 * 1024 * 2.0  # median, not mean
    assert r["detail"]["write"]["bytes_per_launch"] == 670000.0 * 1024
    assert r["bytes_per_launch"] == (340000.0 * 2.0 + 670000.0) * 1024
    assert r["algorithmic_bytes"] == 40 * sites and r["ratio"] == r["bytes_per_launch"] / (40 * sites)
    assert r["kernel_sha"] == prof.kernel_hash()
