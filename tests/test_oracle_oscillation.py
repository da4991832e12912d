"""Pins of the oscillation post-processing (oracle/post.py): a tanh ellipse whose
mid-level crossing is known in closed form, damped cosines of known period."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import post


def test_major_axis_radius_of_the_initial_ellipse():
    w = W.oscillating_droplet()
    mid = 0.5 * (w.info["rho_l"] + w.info["rho_g"])
    # the line y = cy lies between rows at |dy| = 1/2; both rows cross the level set
    # (x/A)^2 + (y/B)^2 = 1 of Eq. (31)'s tanh profile at dx = A sqrt(1 - (1/2B)^2)
    A, Bv = w.info["r_max"], w.info["r_min"]
    expect = A * math.sqrt(1.0 - (0.5 / Bv) ** 2)
    got = post.major_axis_radius(w.rho0, w.info["cx"], w.info["cy"], mid)
    assert abs(got - expect) < 2e-3, (got, expect)
    # a field whose axis line sits on a lattice row: exact at the major semi-axis
    w2 = W.oscillating_droplet(n=201)
    got2 = post.major_axis_radius(w2.rho0, w2.info["cx"], w2.info["cy"], mid)
    assert abs(got2 - A) < 1e-9


@pytest.mark.parametrize("period,decay,dt", [(2600.0, 5000.0, 10), (2593.8, 1e9, 25), (731.0, 2000.0, 7)])
def test_oscillation_period_of_damped_cosines(period, decay, dt):
    t = np.arange(0, 4.2 * period, dt, dtype=np.float64)
    r = 28.5 + 1.5 * np.exp(-t / decay) * np.cos(2 * np.pi * t / period + 0.3)
    assert abs(post.oscillation_period(t, r) / period - 1.0) < 5e-3
