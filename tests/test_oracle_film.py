"""Pins for the oracle's film thickness, squeeze term and dimples (paper Eq 2.3)."""

import numpy as np
import pytest

import oracle
import synth
from conftest import gap_of


def _gap(**over):
    return gap_of(synth.smooth_case(64, 32, 0), **over)


def test_concentric_film_is_clearance():
    gap = _gap()
    th = np.linspace(0, 2 * np.pi, 97)
    z = np.linspace(0, gap.L, 13)
    TH, Z = np.meshgrid(th, z)
    h = oracle.film(gap, np.zeros(4), TH, Z)
    assert np.max(np.abs(h - gap.c)) <= 1e-12 * gap.c
    h2 = oracle.film_naive(gap, np.zeros(4), TH, Z)
    assert np.max(np.abs(h2 - gap.c)) <= 1e-9 * gap.c   # naive form loses ~1e-2/1e-5 digits


@pytest.mark.parametrize("seed", range(5))
def test_stable_form_equals_eq_2_3(seed):
    gap = _gap()
    e, _ = synth.draw_state(seed)
    th = np.linspace(0, 2 * np.pi, 181)
    z = np.linspace(0, gap.L, 21)
    TH, Z = np.meshgrid(th, z)
    a = oracle.film(gap, e, TH, Z)
    b = oracle.film_naive(gap, e, TH, Z)
    assert np.max(np.abs(a - b) / np.abs(a)) < 1e-9
    assert np.all(a > 0)


def test_small_eccentricity_first_order():
    """h ~ c - e_x cos - e_y sin for |e| << c (the textbook journal-bearing film)."""
    gap = _gap()
    e = np.array([1e-9, -2e-9, 1e-9, -2e-9])
    th = np.linspace(0, 2 * np.pi, 181)
    h = oracle.film(gap, e, th, 0.0 * th + 0.3 * gap.L)
    lin = gap.c - e[0] * np.cos(th) - e[1] * np.sin(th)
    assert np.max(np.abs(h - lin)) < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_squeeze_is_time_derivative_of_film(seed):
    """dh/dt along e(t) = e + t edot, against a central difference of h itself."""
    gap = _gap()
    e, edot = synth.draw_state(seed)
    th = np.linspace(0, 2 * np.pi, 61)
    z = np.linspace(0, gap.L, 9)
    TH, Z = np.meshgrid(th, z)
    t = 1e-6
    fd = (oracle.film(gap, e + t * edot, TH, Z) - oracle.film(gap, e - t * edot, TH, Z)) / (2 * t)
    hd = oracle.film_rate(gap, e, edot, TH, Z)
    assert np.max(np.abs(fd - hd)) <= 1e-7 * np.max(np.abs(hd))


def test_dimple_cap_geometry():
    R, a, d = 10e-3, 0.5e-3, 10e-6
    tex = oracle.dimple_texture(R, [1.0], [0.02], [a], [d])
    assert abs(tex(1.0, 0.02) - d) < 1e-18
    # zero on and outside the footprint circle, positive inside
    ang = np.linspace(0, 2 * np.pi, 50)
    for r, sign in [(a * 1.0000001, 0), (1.5 * a, 0), (0.5 * a, 1)]:
        v = tex(1.0 + r * np.cos(ang) / R, 0.02 + r * np.sin(ang))
        assert (np.all(v > 0) if sign else np.all(v == 0))
    # cap volume pi d (3 a^2 + d^2) / 6 by midpoint quadrature over a fine patch
    n = 801
    s = np.linspace(-1.1 * a, 1.1 * a, n + 1)
    mid = 0.5 * (s[1:] + s[:-1])
    X, Y = np.meshgrid(mid, mid)
    vol = np.sum(tex(1.0 + X / R, 0.02 + Y)) * (s[1] - s[0]) ** 2
    exact = np.pi * d * (3 * a * a + d * d) / 6
    assert abs(vol - exact) < 2e-3 * exact


def test_dimple_wraps_around_theta_and_overlaps_take_max():
    R, a = 10e-3, 0.5e-3
    tex = oracle.dimple_texture(R, [0.01, 0.01], [0.02, 0.0202], [a, a], [5e-6, 8e-6])
    # just below 2 pi is 0.02 rad = 0.2 mm away from the centre at 0.01 rad -> inside
    assert tex(2 * np.pi - 0.01, 0.02) > 0
    one = oracle.dimple_texture(R, [0.01], [0.02], [a], [5e-6])
    two = oracle.dimple_texture(R, [0.01], [0.0202], [a], [8e-6])
    th = np.linspace(-0.1, 0.1, 41)
    zz = np.linspace(0.019, 0.021, 41)
    TH, Z = np.meshgrid(th, zz)
    assert np.array_equal(tex(TH, Z), np.maximum(one(TH, Z), two(TH, Z)))


def test_regular_dimple_layout():
    th, zc, a, d = synth.regular_dimples(0)
    assert th.size == 160 and np.all((d >= 5e-6) & (d <= 15e-6))
    assert np.all((zc > 0.2 * synth.LENGTH) & (zc < 0.8 * synth.LENGTH))
